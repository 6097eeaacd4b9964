// Learned closure network on MFMA (gfx950): 7 -> 128 -> 128 -> 128 -> 2, ReLU,
// sigmoid on output 0.  Products run in bfloat16 with float32 accumulation on
// v_mfma_f32_32x32x16_bf16; master weights, biases, gradients and the Adam
// state are float32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "tr.h"
#include "tr_mlp_dev.h"

namespace {

using namespace trmlp;

struct Gemm {
  const uint16_t *A;  // [M x K], element (m, k) at A[m * am + k * ak]
  long long am, ak;
  const uint16_t *B;  // [K x N], element (k, n) at B[k * bk + n * bn]
  long long bk, bn;
  int M, N, K;
  float *Cf;  // optional float32 output (m, n) at Cf[m * cm + n]
  uint16_t *Cb;  // optional bfloat16 output (m, n) at Cb[m * cm + n]
  long long cm;
  const float *bias;  // optional, per column n
  int relu;
  const uint16_t *mask;  // optional: zero where mask(m, n) == 0 (ReLU derivative)
  long long mm;
  float *split;  // optional scratch [64][M][N]: long reductions are split over K
  int kc;        // split-K chunk length (set by gemm(); 0: the whole K)
  int panels;    // k_gemm_rows: 32-row panels per wavefront (set by gemm())
};

// Epilogue of one output element.
__device__ inline float gemm_value(const Gemm &g, int mm, int nn, float v) {
  if (g.bias) v += g.bias[nn];
  if (g.relu) v = fmaxf(v, 0.0f);
  if (g.mask && g.mask[mm * g.mm + nn] == 0) v = 0.0f;
  return v;
}

__device__ inline void gemm_store(const Gemm &g, int mm, int nn, float v) {
  v = gemm_value(g, mm, nn, v);
  if (g.Cf) g.Cf[mm * g.cm + nn] = v;
  if (g.Cb) g.Cb[mm * g.cm + nn] = to_bf16(v);
}

// C = epilogue(A B): one wavefront per 32 x 32 output tile, K in steps of 16.
// Lane l holds A(m0 + l % 32, k0 + 8 (l / 32) + 0..7), B(k0 + 8 (l / 32) + 0..7,
// n0 + l % 32) and accumulator element j of D(m0 + 8 (j / 4) + 4 (l / 32) +
// j % 4, n0 + l % 32).  Out-of-range rows/columns read zeros and are not stored.
// With g.kc > 0, block z covers K range [z kc, (z + 1) kc) and writes its raw
// partial tile to g.split[z] (the epilogue follows in k_gemm_reduce).
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = (blockIdx.x * 2 + (wv >> 1)) * 32;
  const int n0 = (blockIdx.y * 2 + (wv & 1)) * 32;
  if (m0 >= g.M || n0 >= g.N) return;
  const int r = lane & 31, hk = (lane >> 5) * 8;
  const int m = m0 + r, n = n0 + r;
  const int kb = g.kc ? blockIdx.z * g.kc : 0;
  const int ke = g.kc ? min(g.K, kb + g.kc) : g.K;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + hk + i;
      a[i] = (m < g.M && k < ke) ? (short)g.A[m * g.am + k * g.ak] : (short)0;
      b[i] = (n < g.N && k < ke) ? (short)g.B[k * g.bk + n * g.bn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int nn = n0 + r;
  if (nn >= g.N) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int mm = m0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    if (mm >= g.M) continue;
    if (g.kc)
      g.split[((long long)blockIdx.z * g.M + mm) * g.N + nn] = acc[j];
    else
      gemm_store(g, mm, nn, acc[j]);
  }
}

// Row-panel GEMM for A contiguous in k (ak == 1) with K, N <= 128: the whole
// B is staged once per block in LDS as B^T (k contiguous, rows padded to 136
// bf16 against bank conflicts), each wavefront computes 32-row panels across
// all N columns (up to four 32 x 32 accumulators), so every A fragment is one
// 16-byte load reused for all column tiles.  Lane layout as in k_gemm.
#define TR_GEMM_ROWS_LD 136
__global__ __launch_bounds__(256) void k_gemm_rows(Gemm g) {
  __shared__ uint16_t Bt[128 * TR_GEMM_ROWS_LD];
  __shared__ uint16_t Pb[4][32 * 128];  // bf16 output panel of each wavefront
  const int Kp = (g.K + 15) & ~15;
  // consecutive threads read consecutive n (row-major B: 8 at a time, 16 B),
  // then write the transposed elements; k in [K, Kp) is zero
  if (g.bn == 1 && (g.N & 7) == 0 && (g.bk & 7) == 0) {
    const int n8 = g.N >> 3;
    for (int idx = threadIdx.x; idx < n8 * Kp; idx += 256) {
      const int k = idx / n8, n = 8 * (idx - k * n8);
      bf16x8 v;
      if (k < g.K)
        v = *reinterpret_cast<const bf16x8 *>(g.B + (long long)k * g.bk + n);
      else
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bt[(n + q) * TR_GEMM_ROWS_LD + k] = (uint16_t)v[q];
    }
  } else {
    for (int idx = threadIdx.x; idx < g.N * Kp; idx += 256) {
      const int k = idx / g.N, n = idx - k * g.N;
      Bt[n * TR_GEMM_ROWS_LD + k] = (k < g.K) ? g.B[k * g.bk + n * g.bn] : (uint16_t)0;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int ntile = (g.N + 31) >> 5;
  for (int pnl = 0; pnl < g.panels; ++pnl) {
    const int m0 = ((blockIdx.x * g.panels + pnl) * 4 + wv) * 32;
    if (m0 >= g.M) break;
    const int m = m0 + r;
    f32x16 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
    for (int k0 = 0; k0 < Kp; k0 += 16) {
      const int kk = k0 + 8 * h;
      bf16x8 a;
      if (m < g.M && kk + 8 <= g.K) {
        a = *reinterpret_cast<const bf16x8 *>(g.A + (long long)m * g.am + kk);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = (m < g.M && kk + i < g.K) ? (short)g.A[(long long)m * g.am + kk + i] : (short)0;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < ntile) {
          const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bt + (t * 32 + r) * TR_GEMM_ROWS_LD + kk);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
        }
      }
    }
    // bf16 output rows with a width of a multiple of 8 go through the
    // wavefront's LDS panel and leave as contiguous 16-byte row pieces
    const bool panel = g.Cb && (g.N & 7) == 0 && g.cm == g.N;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int nn = t * 32 + r;
      if (t >= ntile || nn >= g.N) continue;
      const float bias = g.bias ? g.bias[nn] : 0.0f;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int rr = 8 * (j >> 2) + 4 * h + (j & 3);
        const int mm = m0 + rr;
        if (mm >= g.M) continue;
        float v = acc[t][j] + bias;
        if (g.relu) v = fmaxf(v, 0.0f);
        if (g.mask && g.mask[mm * g.mm + nn] == 0) v = 0.0f;
        if (g.Cf) g.Cf[mm * g.cm + nn] = v;
        if (panel)
          Pb[wv][rr * g.N + nn] = to_bf16(v);
        else if (g.Cb)
          g.Cb[mm * g.cm + nn] = to_bf16(v);
      }
    }
    if (panel) {
      // the panel is written and read by this wavefront only
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int pieces = g.N / 8;  // 16-byte pieces per row
      for (int q = lane; q < 32 * pieces; q += 64) {
        const int rr = q / pieces, c8 = q - rr * pieces;
        if (m0 + rr < g.M)
          *reinterpret_cast<bf16x8 *>(g.Cb + (long long)(m0 + rr) * g.cm + 8 * c8) =
              *reinterpret_cast<const bf16x8 *>(&Pb[wv][rr * g.N + 8 * c8]);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Fused inference: all four layers of the network for panels of 32 samples
// per wavefront, the weights staged once per block in LDS as bf16 B^T
// (W1 with K padded from 8 to 16, W4 with N padded from 2 to 32), the
// activations of a panel kept in a per-wavefront LDS panel between layers.
// The rounding points and the order of the MFMA accumulation are those of
// the layer-by-layer kernels (fp32 bias + ReLU, then bf16), so the outputs
// are identical to forward() + k_head.  Block = 8 wavefronts (two per SIMD),
// one block per CU: 153 KB of LDS (gfx950).
#define TR_FUSED_LD 136
#define TR_FUSED_WAVES 8
__global__ __launch_bounds__(64 * TR_FUSED_WAVES) void k_mlp_fused(const float *__restrict__ params, const float *__restrict__ X,
                                                   long long n, float *__restrict__ out) {
  __shared__ uint16_t W1t[NH * 24];
  __shared__ uint16_t W2t[NH * TR_FUSED_LD];
  __shared__ uint16_t W3t[NH * TR_FUSED_LD];
  __shared__ uint16_t W4t[32 * TR_FUSED_LD];
  __shared__ float bias[3 * NH + NOUT];
  __shared__ uint16_t Pn[TR_FUSED_WAVES][32 * TR_FUSED_LD];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < NH * 24; i += nt) {
    const int nn = i / 24, k = i - nn * 24;
    W1t[i] = k < NINP ? to_bf16(params[OW1 + k * NH + nn]) : (uint16_t)0;
  }
  for (int i = tid; i < NH * NH; i += nt) {
    const int k = i / NH, nn = i - k * NH;  // coalesced reads along n
    W2t[nn * TR_FUSED_LD + k] = to_bf16(params[OW2 + i]);
    W3t[nn * TR_FUSED_LD + k] = to_bf16(params[OW3 + i]);
  }
  for (int i = tid; i < 32 * NH; i += nt) {
    const int nn = i / NH, k = i - nn * NH;
    W4t[nn * TR_FUSED_LD + k] = nn < NOUT ? to_bf16(params[OW4 + k * NOUT + nn]) : (uint16_t)0;
  }
  for (int i = tid; i < NH; i += nt) {
    bias[i] = params[OB1 + i];
    bias[NH + i] = params[OB2 + i];
    bias[2 * NH + i] = params[OB3 + i];
  }
  if (tid < NOUT) bias[3 * NH + tid] = params[OB4 + tid];
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int r = lane & 31, h = lane >> 5;
  uint16_t *P = Pn[wv];
  const long long npanel = (n + 31) / 32;
  for (long long pnl = (long long)blockIdx.x * TR_FUSED_WAVES + wv; pnl < npanel;
       pnl += (long long)gridDim.x * TR_FUSED_WAVES) {
    const long long m0 = pnl * 32;
    const long long m = m0 + r;
    f32x16 acc[4];
    // layer 1: K = 8 (second half of the 16-wide k step is zero)
    bf16x8 a;
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (h == 0 && m < n && i < NFEAT) ? (short)to_bf16(X[m * NINP + i]) : (short)0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
      const bf16x8 b = *reinterpret_cast<const bf16x8 *>(W1t + (t * 32 + r) * 24 + 8 * h);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
    }
    // hidden layers: bias + ReLU -> bf16 panel -> next product
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      const float *bl = bias + layer * NH;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float bv = bl[t * 32 + r];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int rr = 8 * (j >> 2) + 4 * h + (j & 3);
          P[rr * TR_FUSED_LD + t * 32 + r] = to_bf16(fmaxf(acc[t][j] + bv, 0.0f));
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      bf16x8 af[8];
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) af[ks] = *reinterpret_cast<const bf16x8 *>(P + r * TR_FUSED_LD + ks * 16 + 8 * h);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      if (layer < 2) {
        const uint16_t *Wt = layer == 0 ? W2t : W3t;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) {
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Wt + (t * 32 + r) * TR_FUSED_LD + ks * 16 + 8 * h);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ks], b, acc[t], 0, 0, 0);
          }
        }
      } else {
        // output layer: one 32-wide tile, columns 0 and 1 are the outputs
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[0][j] = 0.0f;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const bf16x8 b = *reinterpret_cast<const bf16x8 *>(W4t + r * TR_FUSED_LD + ks * 16 + 8 * h);
          acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ks], b, acc[0], 0, 0, 0);
        }
        if (r < NOUT) {
          const float bv = bias[3 * NH + r];
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const long long mm = m0 + 8 * (j >> 2) + 4 * h + (j & 3);
            if (mm < n) {
              const float o = acc[0][j] + bv;
              out[2 * mm + r] = r == 0 ? 1.0f / (1.0f + expf(-o)) : o;
            }
          }
        }
      }
    }
  }
}

// Split-K reduction: element (m, n) adds the nz partial tiles in order, then
// applies the epilogue.
__global__ __launch_bounds__(256) void k_gemm_reduce(Gemm g, int nz) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.M * g.N) return;
  const int mm = (int)(t / g.N), nn = (int)(t - (long long)mm * g.N);
  float v = 0.0f;
  for (int z = 0; z < nz; ++z) v += g.split[(long long)z * g.M * g.N + t];
  gemm_store(g, mm, nn, v);
}

// y[i * ldy + c] = bf16(x[i * ldx + c]) for c < ncol, zeros up to ldy.
__global__ void k_to_bf16(const float *__restrict__ x, long long ldx, int ncol, uint16_t *__restrict__ y,
                          long long ldy, long long nrow) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrow * ldy) return;
  const long long i = t / ldy;
  const int c = (int)(t - i * ldy);
  y[t] = c < ncol ? to_bf16(x[i * ldx + c]) : (uint16_t)0;
}

// out[i] = (sigmoid(o[i][0]), o[i][1])
__global__ void k_head(const float *__restrict__ o, float *__restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[2 * i] = 1.0f / (1.0f + expf(-o[2 * i]));
  out[2 * i + 1] = o[2 * i + 1];
}

// dL/do for the mean-squared loss and per-block loss sums (fixed order).
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ o, const float *__restrict__ Y, int n,
                                              float *__restrict__ dO, uint16_t *__restrict__ dOb,
                                              float *__restrict__ part) {
  __shared__ float red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (i < n) {
    const float fh = 1.0f / (1.0f + expf(-o[2 * i]));
    const float d0 = fh - Y[2 * i], d1 = o[2 * i + 1] - Y[2 * i + 1];
    l = d0 * d0 + d1 * d1;
    const float g0 = 2.0f * d0 * fh * (1.0f - fh) / n, g1 = 2.0f * d1 / n;
    dO[2 * i] = g0;
    dO[2 * i + 1] = g1;
    dOb[2 * i] = to_bf16(g0);
    dOb[2 * i + 1] = to_bf16(g1);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Column sums out[c] = sum_i x[i * ld + c] (bias gradients) in two passes
// with a fixed summation order.  Pass 1: block = (tile of 64 columns, chunk q
// of `rows` rows); its 4 wavefronts add the rows q rows + w, + 4, ... and are
// combined in LDS in wavefront order.  Pass 2 adds the chunk partials in
// chunk order.
#define TR_COLSUM_CHUNKS 64
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ x, long long ld, int ncol, int nrow,
                                                     int rows, float *__restrict__ part) {
  __shared__ float sh[4][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, q = blockIdx.y;
  const int c = blockIdx.x * 64 + l;
  float acc = 0.0f;
  if (c < ncol) {
    const int i1 = min(nrow, (q + 1) * rows);
    for (int i = q * rows + w; i < i1; i += 4) acc += x[(long long)i * ld + c];
  }
  sh[w][l] = acc;
  __syncthreads();
  if (w == 0 && c < ncol) part[(long long)q * ncol + c] = ((sh[0][l] + sh[1][l]) + sh[2][l]) + sh[3][l];
}

__global__ void k_colsum_fin(const float *__restrict__ part, int ncol, int nchunk, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  float acc = 0.0f;
  for (int q = 0; q < nchunk; ++q) acc += part[(long long)q * ncol + c];
  out[c] = acc;
}

void colsum(const float *x, long long ld, int ncol, int nrow, float *out, float *part, hipStream_t st) {
  const int nchunk = std::max(1, std::min(TR_COLSUM_CHUNKS, (nrow + 63) / 64));
  const int rows = (nrow + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_colsum_part, dim3((ncol + 63) / 64, nchunk), dim3(256), 0, st, x, ld, ncol, nrow, rows, part);
  hipLaunchKernelGGL(k_colsum_fin, dim3((ncol + 63) / 64), dim3(64), 0, st, part, ncol, nchunk, out);
}

__global__ void k_accum(float *__restrict__ dst, const float *__restrict__ src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

__global__ void k_sum(const float *__restrict__ part, int n, float *__restrict__ out, float scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float acc = 0.0f;
  for (int i = 0; i < n; ++i) acc += part[i];
  *out = acc * scale;
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather(const float *__restrict__ src, int w, const int *__restrict__ idx, int n,
                         float *__restrict__ dst) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * w) return;
  const long long i = t / w;
  const int c = (int)(t - i * w);
  dst[t] = src[(long long)idx[i] * w + c];
}

// work layout (bytes, 256-aligned pieces)
struct Work {
  uint16_t *Xb, *Wb, *H1, *H2, *H3, *dOb, *dZb;
  float *O, *dO, *dZf, *part, *gtmp, *cpart, *split;
};

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr size_t work_bytes(long long n) {
  size_t b = 0;
  b += align256(n * NINP * 2);            // Xb
  b += align256((size_t)NPARAM * 2);       // Wb (bf16 copy of the parameter vector)
  b += 3 * align256(n * NH * 2);           // H1..H3
  b += align256(n * NOUT * 2);             // dOb
  b += align256(n * NH * 2);               // dZb
  b += align256(n * NOUT * 4);             // O
  b += align256(n * NOUT * 4);             // dO
  b += align256(n * NH * 4);               // dZf
  b += align256(((n + 255) / 256) * 4);    // loss partials
  b += align256((size_t)NPARAM * 4);       // gradient scratch
  b += align256((size_t)TR_COLSUM_CHUNKS * NH * 4);  // column-sum chunk partials
  b += align256((size_t)64 * NH * NH * 4);            // split-K partial tiles
  return b;
}

Work carve(void *w, long long n) {
  char *p = static_cast<char *>(w);
  Work k;
  auto take = [&](size_t bytes) {
    char *q = p;
    p += align256(bytes);
    return q;
  };
  k.Xb = (uint16_t *)take(n * NINP * 2);
  k.Wb = (uint16_t *)take((size_t)NPARAM * 2);
  k.H1 = (uint16_t *)take(n * NH * 2);
  k.H2 = (uint16_t *)take(n * NH * 2);
  k.H3 = (uint16_t *)take(n * NH * 2);
  k.dOb = (uint16_t *)take(n * NOUT * 2);
  k.dZb = (uint16_t *)take(n * NH * 2);
  k.O = (float *)take(n * NOUT * 4);
  k.dO = (float *)take(n * NOUT * 4);
  k.dZf = (float *)take(n * NH * 4);
  k.part = (float *)take(((n + 255) / 256) * 4);
  k.gtmp = (float *)take((size_t)NPARAM * 4);
  k.cpart = (float *)take((size_t)TR_COLSUM_CHUNKS * NH * 4);
  k.split = (float *)take((size_t)64 * NH * NH * 4);
  return k;
}

// Long reductions over few output tiles (the weight gradients, K = batch) are
// split over K into up to 64 chunks of at least 128 so the chip fills.
void gemm(const Gemm &g0, hipStream_t st) {
  Gemm g = g0;
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64);
  int nz = 1;
  if (g.split && g.K >= 512 && (long long)g.M * g.N <= (long long)NH * NH) {
    nz = std::min(64, g.K / 128);
    g.kc = ((g.K + nz - 1) / nz + 15) / 16 * 16;
    nz = (g.K + g.kc - 1) / g.kc;
  }
  if (nz == 1) {
    g.kc = 0;
    if (g.ak == 1 && g.K <= 128 && g.N <= 128) {
      // enough panels per block to amortise staging B, while keeping >= 512 blocks
      g.panels = std::max(1, std::min(32, g.M / (128 * 512)));
      const int rows = 4 * 32 * g.panels;
      hipLaunchKernelGGL(k_gemm_rows, dim3((unsigned)((g.M + rows - 1) / rows)), dim3(256), 0, st, g);
    } else {
      hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
    }
    return;
  }
  grid.z = nz;
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
  const long long n = (long long)g.M * g.N;
  hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, nz);
}

Gemm gemm_nn(const uint16_t *A, long long am, long long ak, const uint16_t *B, long long bk, long long bn, int M,
             int N, int K) {
  Gemm g{};
  g.A = A;
  g.am = am;
  g.ak = ak;
  g.B = B;
  g.bk = bk;
  g.bn = bn;
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

// forward pass; keeps the bf16 activations in the work area
void forward(const float *params, const float *X, long long n, const Work &w, hipStream_t st) {
  const int tb = 256;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((NPARAM + tb - 1) / tb)), dim3(tb), 0, st, params, 1LL, 1, w.Wb,
                     1LL, (long long)NPARAM);
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n * NINP + tb - 1) / tb)), dim3(tb), 0, st, X, (long long)NINP, NFEAT,
                     w.Xb, (long long)NINP, n);
  const uint16_t *W1 = w.Wb + OW1, *W2 = w.Wb + OW2, *W3 = w.Wb + OW3, *W4 = w.Wb + OW4;
  Gemm g = gemm_nn(w.Xb, NINP, 1, W1, NH, 1, (int)n, NH, NINP);
  g.Cb = w.H1;
  g.cm = NH;
  g.bias = params + OB1;
  g.relu = 1;
  gemm(g, st);
  g = gemm_nn(w.H1, NH, 1, W2, NH, 1, (int)n, NH, NH);
  g.Cb = w.H2;
  g.cm = NH;
  g.bias = params + OB2;
  g.relu = 1;
  gemm(g, st);
  g = gemm_nn(w.H2, NH, 1, W3, NH, 1, (int)n, NH, NH);
  g.Cb = w.H3;
  g.cm = NH;
  g.bias = params + OB3;
  g.relu = 1;
  gemm(g, st);
  g = gemm_nn(w.H3, NH, 1, W4, NOUT, 1, (int)n, NOUT, NH);
  g.Cf = w.O;
  g.cm = NOUT;
  g.bias = params + OB4;
  gemm(g, st);
}

// gradient of the mean-squared loss; grad [NPARAM], loss (device float)
void backward(const float *params, const float *X, const float *Y, long long n, float *grad, float *loss,
              const Work &w, hipStream_t st) {
  forward(params, X, n, w, st);
  const int nb = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, st, w.O, Y, (int)n, w.dO, w.dOb, w.part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, w.part, nb, loss, 1.0f / (float)n);
  const uint16_t *W2 = w.Wb + OW2, *W3 = w.Wb + OW3, *W4 = w.Wb + OW4;
  // layer 4: dW4 = H3^T dO, db4 = sum dO, dZ3 = (dO W4^T) * [H3 > 0]
  Gemm g = gemm_nn(w.H3, 1, NH, w.dOb, NOUT, 1, NH, NOUT, (int)n);
  g.Cf = grad + OW4;
  g.split = w.split;
  g.cm = NOUT;
  gemm(g, st);
  colsum(w.dO, (long long)NOUT, NOUT, (int)n, grad + OB4, w.cpart, st);
  g = gemm_nn(w.dOb, NOUT, 1, W4, 1, NOUT, (int)n, NH, NOUT);
  g.Cf = w.dZf;
  g.Cb = w.dZb;
  g.cm = NH;
  g.mask = w.H3;
  g.mm = NH;
  gemm(g, st);
  // layer 3
  g = gemm_nn(w.H2, 1, NH, w.dZb, NH, 1, NH, NH, (int)n);
  g.Cf = grad + OW3;
  g.split = w.split;
  g.cm = NH;
  gemm(g, st);
  colsum(w.dZf, (long long)NH, NH, (int)n, grad + OB3, w.cpart, st);
  g = gemm_nn(w.dZb, NH, 1, W3, 1, NH, (int)n, NH, NH);
  g.Cf = w.dZf;
  g.Cb = w.dZb;
  g.cm = NH;
  g.mask = w.H2;
  g.mm = NH;
  gemm(g, st);
  // layer 2
  g = gemm_nn(w.H1, 1, NH, w.dZb, NH, 1, NH, NH, (int)n);
  g.Cf = grad + OW2;
  g.split = w.split;
  g.cm = NH;
  gemm(g, st);
  colsum(w.dZf, (long long)NH, NH, (int)n, grad + OB2, w.cpart, st);
  g = gemm_nn(w.dZb, NH, 1, W2, 1, NH, (int)n, NH, NH);
  g.Cf = w.dZf;
  g.Cb = w.dZb;
  g.cm = NH;
  g.mask = w.H1;
  g.mm = NH;
  gemm(g, st);
  // layer 1
  g = gemm_nn(w.Xb, 1, NINP, w.dZb, NH, 1, NINP, NH, (int)n);
  g.Cf = grad + OW1;
  g.split = w.split;
  g.cm = NH;
  gemm(g, st);
  colsum(w.dZf, (long long)NH, NH, (int)n, grad + OB1, w.cpart, st);
}

// Scratch of the allocation-free gradient entry point: the pass work of
// TR_MLP_NOALLOC_MAX_N samples in one file-scope array.  Every GPU the library
// runs on holds its own copy at its own address (found once per device with
// hipGetSymbolAddress); host code passes that address, never the array's name.
constexpr size_t kNoAllocBytes = work_bytes(TR_MLP_NOALLOC_MAX_N);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (resolved on the
// first call per device).
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TR_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return TR_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TR_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TR_OK;
}

}  // namespace

extern "C" {

int tr_mlp_nparam(void) { return NPARAM; }

size_t tr_mlp_work_bytes(long long n) { return work_bytes(n); }

int tr_mlp_forward(const float *params, const float *X, long long n, float *out, void *work, hipStream_t st) {
  if (!params || !X || !out || !work || n <= 0) return TR_EINVAL;
  // fused inference: at most one block per CU (the weights are staged once
  // per block), wavefronts loop over the 32-sample panels
  const long long npanel = (n + 31) / 32;
  const unsigned nb = (unsigned)std::min<long long>(256, (npanel + TR_FUSED_WAVES - 1) / TR_FUSED_WAVES);
  hipLaunchKernelGGL(k_mlp_fused, dim3(nb), dim3(64 * TR_FUSED_WAVES), 0, st, params, X, n, out);
  return hipGetLastError() == hipSuccess ? TR_OK : TR_EHIP;
}

int tr_mlp_grad(const float *params, const float *X, const float *Y, long long n, float *grad, float *loss,
                void *work, hipStream_t st) {
  if (!params || !X || !Y || !grad || !loss || !work || n <= 0) return TR_EINVAL;
  const Work w = carve(work, n);
  backward(params, X, Y, n, grad, loss, w, st);
  return hipGetLastError() == hipSuccess ? TR_OK : TR_EHIP;
}

int tr_mlp_grad_noalloc(const float *params, const float *X, const float *Y, long long n, float *grad, float *loss,
                        hipStream_t st) {
  if (!params || !X || !Y || !grad || !loss || n <= 0 || n > TR_MLP_NOALLOC_MAX_N) return TR_EINVAL;
  void *work = nullptr;
  const int rc = scratch_address(&work);
  if (rc != TR_OK) return rc;
  // every word of the pass work is written before it is read within one call
  const Work w = carve(work, n);
  backward(params, X, Y, n, grad, loss, w, st);
  return hipGetLastError() == hipSuccess ? TR_OK : TR_EHIP;
}

int tr_mlp_adam(float *params, float *m, float *v, const float *grad, int t, float lr, hipStream_t st) {
  if (!params || !m || !v || !grad || t < 1) return TR_EINVAL;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, m, v, grad, NPARAM, lr, b1, b2,
                     1e-8f, c1, c2);
  return hipGetLastError() == hipSuccess ? TR_OK : TR_EHIP;
}

int tr_mlp_train_epoch(float *params, float *m, float *v, int *t, float lr, const float *X, const float *Y,
                       long long n, const int *perm, int batch, void *work, float *loss_sum, hipStream_t st) {
  if (!params || !m || !v || !t || !X || !Y || !perm || batch <= 0 || !work || !loss_sum || n <= 0)
    return TR_EINVAL;
  // work holds: gathered X [batch][8], Y [batch][2], gradient, loss, then the pass work
  char *p = static_cast<char *>(work);
  float *Xg = (float *)p;
  p += align256((size_t)batch * NINP * 4);
  float *Yg = (float *)p;
  p += align256((size_t)batch * NOUT * 4);
  float *grad = (float *)p;
  p += align256((size_t)NPARAM * 4);
  float *lossb = (float *)p;
  p += align256(4);
  const Work w = carve(p, batch);
  for (long long s = 0; s + batch <= n; s += batch) {
    hipLaunchKernelGGL(k_gather, dim3((batch * NINP + 255) / 256), dim3(256), 0, st, X, NINP, perm + s, batch, Xg);
    hipLaunchKernelGGL(k_gather, dim3((batch * NOUT + 255) / 256), dim3(256), 0, st, Y, NOUT, perm + s, batch, Yg);
    backward(params, Xg, Yg, batch, grad, lossb, w, st);
    *t += 1;
    int rc = tr_mlp_adam(params, m, v, grad, *t, lr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_accum, dim3(1), dim3(64), 0, st, loss_sum, lossb);
  }
  return hipGetLastError() == hipSuccess ? TR_OK : TR_EHIP;
}

size_t tr_mlp_train_work_bytes(int batch) {
  return align256((size_t)batch * NINP * 4) + align256((size_t)batch * NOUT * 4) + align256((size_t)NPARAM * 4) +
         align256(4) + work_bytes(batch);
}

}  // extern "C"
