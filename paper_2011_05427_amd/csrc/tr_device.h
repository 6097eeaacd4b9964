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
// terms of x_s and x_{e+1} (first row of partition t+1).  These 2T rows form a
// tridiagonal "interface" system solved by parallel cyclic reduction in LDS;
// the interior rows then follow by back substitution.  The systems here are
// column diagonally dominant M-matrices, so no pivoting is needed.
// lds must hold 8 * T doubles.
// ---------------------------------------------------------------------------
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
  // interface rows: 2t -> x_s, 2t+1 -> x_e
  double *ra = lds, *rb = lds + 2 * T, *rc = lds + 4 * T, *rd = lds + 6 * T;
  ra[2 * t] = a[0];
  rb[2 * t] = bv;
  rc[2 * t] = cv;
  rd[2 * t] = dv;
  ra[2 * t + 1] = ah[K - 1];
  rb[2 * t + 1] = bh[K - 1];
  rc[2 * t + 1] = c[K - 1];
  rd[2 * t + 1] = dh[K - 1];
  __syncthreads();
  const int R = 2 * T;
  for (int st = 1; st < R; st <<= 1) {
    double na[2], nb[2], nc[2], nd[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int i = 2 * t + q;
      double ai = ra[i], bi = rb[i], ci = rc[i], di = rd[i];
      double al = 0.0, ga = 0.0;
      double am = 0.0, cm = 0.0, dm = 0.0, ap = 0.0, cp = 0.0, dp = 0.0;
      if (i - st >= 0) {
        al = ai * rcp_nr(rb[i - st]);
        am = ra[i - st];
        cm = rc[i - st];
        dm = rd[i - st];
      }
      if (i + st < R) {
        ga = ci * rcp_nr(rb[i + st]);
        ap = ra[i + st];
        cp = rc[i + st];
        dp = rd[i + st];
      }
      na[q] = -al * am;
      nc[q] = -ga * cp;
      nb[q] = bi - al * cm - ga * ap;
      nd[q] = di - al * dm - ga * dp;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int i = 2 * t + q;
      ra[i] = na[q];
      rb[i] = nb[q];
      rc[i] = nc[q];
      rd[i] = nd[q];
    }
    __syncthreads();
  }
  const double xs = rd[2 * t] * rcp_nr(rb[2 * t]);
  const double xe = rd[2 * t + 1] * rcp_nr(rb[2 * t + 1]);
  x[0] = xs;
  x[K - 1] = xe;
#pragma unroll
  for (int i = K - 2; i >= 1; --i) x[i] = (dh[i] - ah[i] * xs - c[i] * x[i + 1]) * ib[i];
  __syncthreads();
  // publish the first unknown of every partition for neighbours (reuse ra)
  ra[t] = xs;
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
