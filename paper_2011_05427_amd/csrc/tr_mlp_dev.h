// Closure network shapes, parameter layout and bfloat16 helpers shared by the
// MLP kernels and the fused seeding kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trmlp {

constexpr int NH = 128, NINP = 8, NOUT = 2, NFEAT = 7;  // NFEAT of the NINP input columns are used
// parameter vector offsets (float32): W1 [8][128], b1, W2 [128][128], b2, W3, b3, W4 [128][2], b4
constexpr int OW1 = 0, OB1 = OW1 + NINP * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NH * NOUT, NPARAM = OB4 + NOUT;

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest, ties to even
__device__ inline uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__device__ inline float from_bf16(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Two floats -> packed bfloat16 pair (lo in bits 0-15), round to nearest,
// ties to even, by the hardware conversion (one v_cvt_pk_bf16_f32).
__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

}  // namespace trmlp
