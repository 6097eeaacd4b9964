// Device helpers: Planck group integrals, opacity law, tridiagonal solver.
#pragma once

#include "tr_common.h"

// ---------------------------------------------------------------------------
// 1/x from the hardware reciprocal estimate refined by two Newton steps,
// which take the estimate's error to the binary64 rounding level.  For
// normal, finite x of moderate exponent (what the low-order systems hold);
// a * rcp_nr(b) then differs from a / b by a couple of ulps at most.
// ---------------------------------------------------------------------------
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// ---------------------------------------------------------------------------
// Planck integral  Q(x) = int_0^x t^3/(e^t - 1) dt  (total pi^4/15).
// Below x = 2 the Bernoulli series t/(e^t-1) = sum B_k t^k / k! integrated
// term by term; above, the geometric expansion 1/(e^t-1) = sum_n e^{-n t}
// integrated exactly:  int_x^inf t^3 e^{-n t} dt = e^{-nx}(x^3/n + 3x^2/n^2 +
// 6x/n^3 + 6/n^4).  Both coefficient tables live in constant memory,
// initialised when the code object loads.
// ---------------------------------------------------------------------------
#define TR_NHEAD 40

static constexpr double TR_PI4_15 = 6.4939394022668291491;  // pi^4 / 15
static constexpr double TR_XSW = 2.0;

// Head coefficients c_k = B_k / (k! (k + 3)): c_0 = 1/3, c_1 = -1/8, odd k > 1
// vanish, and for even k, B_k / k! = (-1)^(k/2 + 1) 2 zeta(k) / (2 pi)^k with
// zeta(2) = pi^2 / 6 and zeta(k), k >= 4, summed directly over n < 64 plus the
// Euler-Maclaurin remainder N^(1-k)/(k-1) + N^-k/2 + k N^(-k-1)/12 - k(k+1)(k+2)
// N^(-k-3)/720 at N = 64 (below 1e-25 relative to zeta(k)).
struct TrHeadCoef {
  double c[TR_NHEAD];
};
constexpr double tr_ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}
constexpr TrHeadCoef tr_make_head_coef() {
  TrHeadCoef h{};
  const double pi = 3.14159265358979323846;
  h.c[0] = 1.0 / 3.0;
  h.c[1] = -0.5 / 4.0;
  for (int k = 2; k < TR_NHEAD; k += 2) {
    double zeta;
    if (k == 2) {
      zeta = pi * pi / 6.0;
    } else {
      const int N = 64;
      double acc = 0.0;
      for (int n = N - 1; n >= 1; --n) acc += 1.0 / tr_ipow((double)n, k);
      const double Nk = tr_ipow((double)N, k);
      acc += (double)N / Nk / (k - 1) + 0.5 / Nk + k / (Nk * N) / 12.0 -
             (double)k * (k + 1) * (k + 2) / (Nk * N * N * N) / 720.0;
      zeta = acc;
    }
    const double sign = ((k / 2) % 2 == 1) ? 1.0 : -1.0;
    h.c[k] = sign * 2.0 * zeta / tr_ipow(2.0 * pi, k) / (k + 3);
  }
  return h;
}
extern __constant__ TrHeadCoef tr_head;  // = tr_make_head_coef(), statically initialised

// Head part int_0^x (x < 2): x^3 (c_0 + c_1 x + sum_{j>=1} c_2j x^2j); the
// odd coefficients beyond c_1 vanish, so the even part is a polynomial in x^2.
__device__ inline double q_head(double x) {
  const double y = x * x;
  double acc = tr_head.c[TR_NHEAD - 2];
#pragma unroll
  for (int k = TR_NHEAD - 4; k >= 2; k -= 2) acc = fma(acc, y, tr_head.c[k]);
  acc = fma(acc, y, fma(tr_head.c[1], x, tr_head.c[0]));
  return acc * y * x;
}

// Tail part int_x^inf (x >= 2), given ex = e^{-x}.  Terms decay like e^{-nx};
// n_max = 40/x + 2 (at most TR_NTAIL) keeps the truncation below 1e-17
// relative.  The reciprocals 1/n come from a constant table (scalar loads
// that run beside the vector arithmetic).
#define TR_NTAIL 22
extern __constant__ double tr_recip[TR_NTAIL + 1];  // 1/n, statically initialised
__device__ inline double q_tail(double x, double ex) {
  if (!(ex > 0.0)) return 0.0;
  const int nmax = min(TR_NTAIL, (int)(40.0 / x) + 2);
  double en = ex, acc = 0.0;
  double x2 = x * x, x3 = x2 * x;
  for (int n = 1; n <= nmax; ++n) {
    const double rn = tr_recip[n];
    // x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4 = (x^3 + (3x^2 + (6x + 6/n)/n)/n)/n
    double poly = fma(rn, fma(rn, fma(rn, 6.0, 6.0 * x), 3.0 * x2), x3);
    acc = fma(en * rn, poly, acc);
    en *= ex;
  }
  return acc;
}

// One group edge: x = nu/T with its head/tail representation.
struct EdgeQ {
  double x;     // nu / T (may be +inf)
  double head;  // int_0^x if x < 2
  double tail;  // int_x^inf if x >= 2
  double g4;    // x^4 / (e^x - 1) (0 at x = 0 and x = inf)
  int is_tail;
};

// inv_T = 1 / T (one reciprocal per cell, shared by its edges).  In the tail
// range 1 - e^{-x} >= 0.86 is computed directly (no cancellation).
__device__ inline EdgeQ edge_q(double nu, double inv_T) {
  EdgeQ e;
  double x = nu * inv_T;
  e.x = x;
  if (nu == 0.0) {
    e.head = 0.0; e.tail = 0.0; e.g4 = 0.0; e.is_tail = 0;
  } else if (x < TR_XSW) {
    e.head = q_head(x); e.tail = 0.0; e.is_tail = 0;
    double x2 = x * x;
    e.g4 = x2 * x2 * rcp_nr(expm1(x));
  } else if (x >= 746.0) {  // e^{-x} underflows to zero (x = +inf included)
    e.head = 0.0; e.tail = 0.0; e.g4 = 0.0; e.is_tail = 1;
  } else {
    double ex = exp(-x);
    e.head = 0.0; e.tail = q_tail(x, ex); e.is_tail = 1;
    double x2 = x * x;
    e.g4 = (ex > 0.0) ? x2 * x2 * ex * rcp_nr(1.0 - ex) : 0.0;
  }
  return e;
}

// int_{x_lo}^{x_hi} t^3/(e^t-1) dt from two edge representations.
__device__ inline double q_interval(const EdgeQ &lo, const EdgeQ &hi) {
  if (lo.is_tail) return lo.tail - hi.tail;           // both in the tail range
  if (!hi.is_tail) return hi.head - lo.head;          // both in the head range
  return (TR_PI4_15 - hi.tail) - lo.head;             // straddles x = 2
}

// ---------------------------------------------------------------------------
// Partitioned tridiagonal solver for one system per thread block.
//
// Rows j = 0..N-1:  a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j  (a_0 = c_{N-1} = 0).
// Thread t owns rows s = tK .. e = tK + K - 1 (rows >= N are identity rows).
// Local elimination gives, for every partition, a row of x_s in terms of the
// neighbours x_{s-1} (last row of partition t-1) and x_e, and a row of x_e in
// terms of x_s and x_{e+1} (first row of partition t+1).  These R = 2T rows
// form a tridiagonal "interface" system, which one wavefront solves (see
// tri_interface_wave); the interior rows then follow by back substitution.
// The systems here are column diagonally dominant M-matrices, so no pivoting
// is needed.  T is a multiple of 64 (at most 512); lds must hold
// tri_lds_doubles(T) doubles.  On return lds[u] holds x_{uK}, the first
// unknown of partition u, for every u < T.
// ---------------------------------------------------------------------------
// Stride of the solver's LDS arrays: R rows at skewed positions (see below).
__host__ __device__ constexpr int tri_lds_stride(int T) { return 2 * T + 64; }
__host__ __device__ constexpr int tri_lds_doubles(int T) { return 7 * tri_lds_stride(T); }

// The interface system, solved by wavefront 0 (lanes l = 0..63).  Lane l owns
// the M = R / 64 consecutive rows lM .. lM + M - 1, stored at positions
// l (M + 1) + i (one spare slot per lane, so that the lanes' strided accesses
// spread over the LDS banks) of the arrays A, B, C, D.  The lane eliminates
// its rows by itself, as a thread does its K rows: its first row in terms of
// the previous lane's last unknown and its own last, its last row in terms of
// its first unknown and the next lane's first.  These 128 rows are tridiagonal
// again and are solved by cyclic reduction across the lanes with shuffles (no
// block barrier); the lane's inner rows then follow by back substitution from
// the rows its forward elimination left in H, Q (reciprocal pivots) and G.
// Every unknown is written over its row's d in D.
__device__ inline void tri_interface_wave(const double *__restrict__ A, const double *__restrict__ B,
                                          const double *__restrict__ C, double *__restrict__ D,
                                          double *__restrict__ H, double *__restrict__ Q, double *__restrict__ G,
                                          int M) {
  const int l = threadIdx.x;
  const int p0 = l * (M + 1);
  // forward (rows 1 .. M-1 in terms of x_first) and backward (rows M-2 .. 0
  // in terms of x_last) elimination, interleaved: they are independent chains
  double eta = A[p0 + 1], bet = B[p0 + 1], del = D[p0 + 1], cpr = C[p0 + 1];
  double ib = rcp_nr(bet);
  H[p0 + 1] = eta;
  Q[p0 + 1] = ib;
  G[p0 + 1] = del;
  double ual = A[p0 + M - 2], ube = B[p0 + M - 2], uga = C[p0 + M - 2], ude = D[p0 + M - 2];
  for (int k = 0; k < M - 2; ++k) {
    const int id = p0 + k + 2, iu = p0 + M - 3 - k;
    const double ad = A[id], bd = B[id], cd = C[id], dd = D[id];
    const double au = A[iu], bu = B[iu], cu = C[iu], du = D[iu];
    const double r = ad * ib;
    eta = -r * eta;
    bet = bd - r * cpr;
    del = dd - r * del;
    cpr = cd;
    ib = rcp_nr(bet);
    if (k + 2 <= M - 2) {
      H[id] = eta;
      Q[id] = ib;
      G[id] = del;
    }
    const double ru = cu * rcp_nr(ube);
    ube = bu - ru * ual;
    uga = -ru * uga;
    ude = du - ru * ude;
    ual = au;
  }
  // the lane's two rows, scaled to a unit diagonal:
  // row 0: a0 x_{prev last} + x_first + c0 x_last = d0
  // row 1: a1 x_first + x_last + c1 x_{next first} = d1
  const double s0 = rcp_nr(ube), s1 = ib;
  double a0 = ual * s0, c0 = uga * s0, d0 = ude * s0;
  double a1 = eta * s1, c1 = cpr * s1, d1 = del * s1;
  // cyclic reduction over the 128 rows 2l + q: at distance st, row i takes
  // rows i - st and i + st (zero outside 0..127) and then couples i -+ 2 st
#pragma unroll
  for (int st = 1; st < 128; st <<= 1) {
    double la0, lc0, ld0, ua0, uc0, ud0, la1, lc1, ld1, ua1, uc1, ud1;
    if (st == 1) {
      const bool lo = l >= 1, hi = l <= 62;
      const double pa = __shfl_up(a1, 1), pc = __shfl_up(c1, 1), pd = __shfl_up(d1, 1);
      const double na = __shfl_down(a0, 1), nc = __shfl_down(c0, 1), nd = __shfl_down(d0, 1);
      la0 = lo ? pa : 0.0; lc0 = lo ? pc : 0.0; ld0 = lo ? pd : 0.0;
      ua0 = a1; uc0 = c1; ud0 = d1;
      la1 = a0; lc1 = c0; ld1 = d0;
      ua1 = hi ? na : 0.0; uc1 = hi ? nc : 0.0; ud1 = hi ? nd : 0.0;
    } else {
      const int sh = st >> 1;
      const bool lo = l >= sh, hi = l + sh <= 63;
      const double p0a = __shfl_up(a0, sh), p0c = __shfl_up(c0, sh), p0d = __shfl_up(d0, sh);
      const double p1a = __shfl_up(a1, sh), p1c = __shfl_up(c1, sh), p1d = __shfl_up(d1, sh);
      const double n0a = __shfl_down(a0, sh), n0c = __shfl_down(c0, sh), n0d = __shfl_down(d0, sh);
      const double n1a = __shfl_down(a1, sh), n1c = __shfl_down(c1, sh), n1d = __shfl_down(d1, sh);
      la0 = lo ? p0a : 0.0; lc0 = lo ? p0c : 0.0; ld0 = lo ? p0d : 0.0;
      la1 = lo ? p1a : 0.0; lc1 = lo ? p1c : 0.0; ld1 = lo ? p1d : 0.0;
      ua0 = hi ? n0a : 0.0; uc0 = hi ? n0c : 0.0; ud0 = hi ? n0d : 0.0;
      ua1 = hi ? n1a : 0.0; uc1 = hi ? n1c : 0.0; ud1 = hi ? n1d : 0.0;
    }
    const double n0 = rcp_nr(1.0 - a0 * lc0 - c0 * ua0), n1 = rcp_nr(1.0 - a1 * lc1 - c1 * ua1);
    const double na0 = -a0 * la0 * n0, nc0 = -c0 * uc0 * n0, nd0 = (d0 - a0 * ld0 - c0 * ud0) * n0;
    const double na1 = -a1 * la1 * n1, nc1 = -c1 * uc1 * n1, nd1 = (d1 - a1 * ld1 - c1 * ud1) * n1;
    a0 = na0; c0 = nc0; d0 = nd0;
    a1 = na1; c1 = nc1; d1 = nd1;
  }
  const double xf = d0, xl = d1;
  D[p0] = xf;
  D[p0 + M - 1] = xl;
  double xn = xl;
  for (int i = M - 2; i >= 1; --i) {
    const double xi = (G[p0 + i] - H[p0 + i] * xf - C[p0 + i] * xn) * Q[p0 + i];
    D[p0 + i] = xi;
    xn = xi;
  }
}

template <int K>
__device__ inline void tri_solve_block(const double (&a)[K], const double (&b)[K], const double (&c)[K],
                                       const double (&d)[K], double (&x)[K], double *lds, int T) {
  const int t = threadIdx.x;
  // downward: rows s+1..e in terms of x_s:  ah_i x_s + bh_i x_i + c_i x_{i+1} = dh_i
  double ah[K], bh[K], dh[K], ib[K];
  ah[1] = a[1];
  bh[1] = b[1];
  dh[1] = d[1];
  ib[1] = rcp_nr(b[1]);
#pragma unroll
  for (int i = 2; i < K; ++i) {
    const double r = a[i] * ib[i - 1];
    ah[i] = -r * ah[i - 1];
    bh[i] = b[i] - r * c[i - 1];
    dh[i] = d[i] - r * dh[i - 1];
    ib[i] = rcp_nr(bh[i]);
  }
  // upward: rows e-1..s in terms of x_e:  a_i x_{i-1} + bv_i x_i + cv_i x_e = dv_i
  double bv = b[K - 2], cv = c[K - 2], dv = d[K - 2];
#pragma unroll
  for (int i = K - 3; i >= 0; --i) {
    const double r = c[i] * rcp_nr(bv);
    bv = b[i] - r * a[i + 1];
    cv = -r * cv;
    dv = d[i] - r * dv;
  }
  // interface rows 2t (x_s) and 2t + 1 (x_e), both in lane 2t / M's range
  const int M = T >> 5, S = tri_lds_stride(T);
  double *A = lds, *B = lds + S, *C = lds + 2 * S, *D = lds + 3 * S;
  const int ps = 2 * t + (2 * t) / M;
  A[ps] = a[0];
  B[ps] = bv;
  C[ps] = cv;
  D[ps] = dv;
  A[ps + 1] = ah[K - 1];
  B[ps + 1] = bh[K - 1];
  C[ps + 1] = c[K - 1];
  D[ps + 1] = dh[K - 1];
  __syncthreads();
  if (t < 64) tri_interface_wave(A, B, C, D, lds + 4 * S, lds + 5 * S, lds + 6 * S, M);
  __syncthreads();
  const double xs = D[ps], xe = D[ps + 1];
  x[0] = xs;
  x[K - 1] = xe;
#pragma unroll
  for (int i = K - 2; i >= 1; --i) x[i] = (dh[i] - ah[i] * xs - c[i] * x[i + 1]) * ib[i];
  // publish the first unknown of every partition for neighbours (the A
  // array is no longer read)
  lds[t] = xs;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Block-wide max reductions (exact, order independent).
// ---------------------------------------------------------------------------
// Six maxima at once; lds: 6 * blockDim doubles.
__device__ inline void block_max6(double (&v)[6], double *lds) {
  const int t = threadIdx.x, n = blockDim.x;
#pragma unroll
  for (int q = 0; q < 6; ++q) lds[q * n + t] = v[q];
  __syncthreads();
  for (int st = n >> 1; st > 0; st >>= 1) {
    if (t < st) {
#pragma unroll
      for (int q = 0; q < 6; ++q) lds[q * n + t] = fmax(lds[q * n + t], lds[q * n + t + st]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) v[q] = lds[q * n];
  __syncthreads();
}

// lds: blockDim doubles.
__device__ inline double block_max(double v, double *lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
    if (t < st) lds[t] = fmax(lds[t], lds[t + st]);
    __syncthreads();
  }
  double r = lds[0];
  __syncthreads();
  return r;
}
