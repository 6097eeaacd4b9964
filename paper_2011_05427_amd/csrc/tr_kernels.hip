// HIP kernels (gfx950, FP64) of the MLQD step with multigrid in frequency.
//
// Every kernel is batched over slabs through a work table (Item = slab, index)
// and can be predicated on the per-slab iteration control, so one launch
// sequence serves a batch of slabs that converge at different iterations.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstddef>

#include "tr.h"
#include "tr_device.h"
#include "tr_kernels.h"
#include "tr_mlp_dev.h"

// Coefficients of the Planck integral series: the Bernoulli head (computed at
// compile time) and 1/n for the tail (index 0 unused).
__constant__ TrHeadCoef tr_head = tr_make_head_coef();
__constant__ double tr_recip[TR_NTAIL + 1] = {
    0.0,        1.0,        1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,  1.0 / 6,  1.0 / 7,
    1.0 / 8,    1.0 / 9,    1.0 / 10, 1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15,
    1.0 / 16,   1.0 / 17,   1.0 / 18, 1.0 / 19, 1.0 / 20, 1.0 / 21, 1.0 / 22};

// Ratios whose denominator is at or below this value (zero, negative, or close
// to the subnormal range where intensities have lost their precision) use the
// isotropic quadrature value or the unweighted mean instead.
#define TR_TINY 1e-290

// ---------------------------------------------------------------------------
// predication
// ---------------------------------------------------------------------------
// The four leading fields of the control record (active, s, ncyc,
// inner_done) are read with one 16-byte load and combined without
// short-circuit evaluation, so a predicated kernel waits for one round trip.
static_assert(offsetof(Ctl, active) == 0 && offsetof(Ctl, s) == 4 && offsetof(Ctl, ncyc) == 8 &&
                  offsetof(Ctl, inner_done) == 12 && sizeof(Ctl) % 16 == 0,
              "control record header");
__device__ inline bool pred_ok(const Ctl *ctl, int slab, int mode, int l) {
  if (ctl == nullptr || mode == PRED_ALL) return true;
  const int4 h = *reinterpret_cast<const int4 *>(ctl + slab);
  const bool active = h.x != 0, s_pos = h.y > 0, at_l = h.z == l, running = h.w == 0;
  switch (mode) {
    case PRED_CYCLE:  // body of cycle l+1 of the current transport iteration
      return active & running & at_l;
    case PRED_DONECYC:  // the slab has just completed cycle l
      return active & at_l;
    case PRED_SWEEP:  // start of a transport iteration s >= 1
      return active & running & (h.z == 0) & s_pos;
    case PRED_ACTIVE:
      return active;
  }
  return true;
}

// 1 - e^{-y} for 0 <= y < 0.1 by its Taylor series y - y^2/2! + ... - y^10/10!
// (the remainder is below y^11/11! < 3e-19 relative).
__device__ inline double om_series(double y) {
  double p = -1.0 / 3628800.0;                 // -1/10!
  p = fma(p, y, 1.0 / 362880.0);               //  1/9!
  p = fma(p, y, -1.0 / 40320.0);               // -1/8!
  p = fma(p, y, 1.0 / 5040.0);                 //  1/7!
  p = fma(p, y, -1.0 / 720.0);                 // -1/6!
  p = fma(p, y, 1.0 / 120.0);                  //  1/5!
  p = fma(p, y, -1.0 / 24.0);                  // -1/4!
  p = fma(p, y, 1.0 / 6.0);                    //  1/3!
  p = fma(p, y, -0.5);                         // -1/2!
  p = fma(p, y, 1.0);
  return p * y;
}

// Opacity and group Planck function of group g (centre nu, edge integrals
// lo / hi) in a cell (1/T = iT, opacity constant Cc, scale = a_R c T^4 / 2 /
// (pi^4 / 15)); returns the group's term of dS = d/dT sum 2 kappa B.  Shared
// by the table kernel and the stage restriction, so both give the same bits.
__device__ inline double planck_group(double nu, const EdgeQ &lo, const EdgeQ &hi, double iT, double Cc,
                                      double scale, double &kap, double &Bg) {
  Bg = scale * q_interval(lo, hi);
  const double dBg = (4.0 * Bg - scale * (hi.g4 - lo.g4)) * iT;
  const double y = nu * iT;
  // 1 - e^{-y}: from the same exponential for y >= 0.1 (relative error
  // below 1e-15), else by its Taylor series (degree 10, below 1e-17); e^{-y}
  // underflows to zero from y = 746 on
  double ey = 0.0;
  if (y < 746.0) ey = exp(-y);
  const double om = y >= 0.1 ? 1.0 - ey : om_series(y);
  const double inu = rcp_nr(nu);
  const double cn = Cc * inu * inu;
  kap = cn * inu * om;
  const double dkap = -cn * ey * iT * iT;
  return 2.0 * (dkap * Bg + kap * dBg);
}

// Group Planck integral of a narrow interior group (nu_hi / nu_lo - 1 <=
// 0.005) by 3-point Gauss-Legendre in x = nu / T: B_g = scale int x^3 / (e^x
// - 1) and dB_g/dT = (scale / T) int x^4 e^x / (e^x - 1)^2 over [a/T, b/T]
// (relative error below 1e-16 where the group carries emission); kappa as in
// planck_group.  Returns the group's dS term.
__device__ inline double planck_group_gl(double nu, double a, double b, double iT, double Cc, double scale,
                                         double &kap, double &Bg) {
  const double xa = a * iT, xb = b * iT;
  const double hh = 0.5 * (xb - xa), xm = 0.5 * (xa + xb);
  constexpr double r35 = 0.77459666924148337704;  // sqrt(3/5)
  double q1 = 0.0, q2 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double t = xm + hh * (j == 0 ? -r35 : j == 1 ? 0.0 : r35);
    const double w = j == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
    const double et = exp(-t);
    const double om = t >= 0.1 ? 1.0 - et : om_series(t);
    const double ri = rcp_nr(om);
    const double i1 = t * t * t * et * ri;
    q1 = fma(w, i1, q1);
    q2 = fma(w, i1 * t * ri, q2);
  }
  Bg = scale * hh * q1;
  const double dBg = scale * iT * hh * q2;
  const double y = nu * iT;
  const double ey = exp(-y);
  const double omk = y >= 0.1 ? 1.0 - ey : om_series(y);
  const double inu = rcp_nr(nu);
  const double cn = Cc * inu * inu;
  kap = cn * inu * omk;
  const double dkap = -cn * ey * iT * iT;
  return 2.0 * (dkap * Bg + kap * dBg);
}

// sum_{j=0..k} y^j / j! (Horner), so that int_y^inf t^k e^{-t} dt =
// k! e^{-y} tail_poly<k>(y).
template <int K>
__device__ inline double tail_poly(double y) {
  double t = 1.0;
#pragma unroll
  for (int j = K; j >= 1; --j) t = fma(t, y * (1.0 / j), 1.0);
  return t;
}

// Group averages of the spectral opacity sigma(nu, T) = Cc / nu^3 (1 -
// e^{-nu/T}) over the group [a, b] (b may be +inf), paper Sec. 2 and Sec. 3.1:
//  - src = sigma_B,g B_g = int sigma B(nu, T) dnu, closed form (the factor
//    1 - e^{-nu/T} cancels the Planck denominator): Cc K T e^{-a/T} (1 -
//    e^{-(b-a)/T}), K = a_R c / 2 / (pi^4 / 15); returns its dS term
//    2 d(src)/dT = 2 Cc K e^{-a/T} ((1 + a/T)(1 - e^{-d}) - d e^{-d}), d = (b-a)/T;
//  - sE = sigma_E,g(T, T_r), sR = sigma_R,g(T, T_r) from Gauss-Legendre
//    panels (8 nodes) in y = nu / T_r over [a/T_r, min(b/T_r, max(a/T_r, 8) +
//    64)]: panel width 1 (2.5 from y = 8 on), or with rho = T_r / T > 1
//    min(1, max(1/rho, y/2)) from the panel's start y.  The factor e^{-y rho} grows off the real axis
//    at the rate rho, so panels close to y = 0 must be short on the scale
//    1/rho and may grow geometrically away from it (their width then stays
//    below half their distance to the imaginary axis, where the poles of
//    1/(1 - e^{-y rho}) lie; those of 1/(1 - e^{-y}) are at 2 pi i k).  Both
//    integrals of a ratio carry the common factor e^{a/T_r}, so no weight
//    over- or underflows in the Wien tail.
// Groups that lie wholly in the Wien tail of both weights (a / T_r >= 40,
// a / T >= 40, (b - a) / T_r >= 0.5) take the closed forms of the four
// integrals instead of the panels.
__device__ inline double spectral_group(double a, double b, double T, double Tr, double Cc, double K, double &sE,
                                        double &src, double &sR) {
  constexpr double gx[4] = {0.18343464249564978, 0.525532409916329, 0.7966664774136267, 0.9602898564975362};
  constexpr double gw[4] = {0.36268378337836177, 0.31370664587788705, 0.22238103445337434, 0.10122853629037669};
  const double iT = 1.0 / T;
  const double xa = a * iT, d = (b - a) * iT;
  const double ea = exp(-xa);
  const double omd = -expm1(-d);  // 1 for the open group
  src = Cc * K * T * ea * omd;
  const double tl = isinf(d) ? 0.0 : d * exp(-d);
  const double dS = 2.0 * Cc * K * ea * ((1.0 + xa) * omd - tl);
  const double iTr = 1.0 / Tr, rho = Tr * iT;
  const double ya = a * iTr, yb = b * iTr;
  const double sc = Cc * iTr * iTr * iTr;
  if (ya >= 40.0 && ya * rho >= 40.0 && yb - ya >= 0.5) {
    // Wien tail of both weights over the whole group: 1 / (1 - e^{-y}) and
    // 1 - e^{-y rho} equal 1 to below 1e-17, and the integrals are closed:
    // int_ya^yb y^k e^{ya - y} dy = k! (p_k(ya) - p_k(yb) e^{ya - yb})
    const double E = isinf(yb) ? 0.0 : exp(ya - yb);
    const double pb = isinf(yb) ? 0.0 : E;  // multiplies p_k(yb); zero for the open group
    const double ybf = isinf(yb) ? ya : yb;
    const double i0 = 1.0 - E;
    const double i3 = 6.0 * (tail_poly<3>(ya) - tail_poly<3>(ybf) * pb);
    const double i4 = 24.0 * (tail_poly<4>(ya) - tail_poly<4>(ybf) * pb);
    const double i7 = 5040.0 * (tail_poly<7>(ya) - tail_poly<7>(ybf) * pb);
    sE = sc * i0 / i3;
    sR = sc * i4 / i7;
    return dS;
  }
  const double ytop = fmin(yb, fmax(ya, 8.0) + 64.0);
  const double hs = rho > 1.0 ? 1.0 / rho : 1.0;
  const double eya = exp(-ya);  // e^{-y} = e^{ya - y} e^{-ya} (zero beyond the double range)
  double nE = 0.0, dE = 0.0, nR = 0.0, dR = 0.0;
  double y0 = ya;
  for (int panel = 0; y0 < ytop && panel < 4096; ++panel) {
    // width 2.5 from y = 8 on (every factor but e^{ya - y} is flat there; the
    // 8-point rule's error on e^{-y} is then below 1e-16 relative)
    const double y1 = fmin(ytop, y0 + fmin(y0 >= 8.0 ? 2.5 : 1.0, fmax(hs, 0.5 * y0)));
    const double hm = 0.5 * (y1 - y0), cm = 0.5 * (y1 + y0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = q < 4 ? 3 - q : q - 4;
      const double y = cm + (q < 4 ? -hm : hm) * gx[k];
      const double wq = hm * gw[k];
      const double e1 = exp(ya - y);
      // 1 - e^{-y} and 1 - e^{-y rho}: from the exponentials for arguments
      // of 0.1 and more, else by their Taylor series
      const double omy = y >= 0.1 ? 1.0 - e1 * eya : om_series(y);
      const double yr = y * rho;
      const double oz = yr >= 0.1 ? 1.0 - exp(-yr) : om_series(yr);
      const double io = 1.0 / omy;
      const double y3 = y * y * y;
      const double bw = e1 * io;           // B(nu, T_r) e^{a/T_r} / (K T_r^3 y^3)
      const double rw = y3 * y * bw * io;  // dB/dT'(nu, T_r) e^{a/T_r} / (K T_r^2)
      nE += wq * oz * bw;
      dE += wq * y3 * bw;
      nR += wq * rw;
      dR += wq * rw * y3 / oz;
    }
    y0 = y1;
  }
  sE = sc * nE / dE;
  sR = sc * nR / dR;
  return dS;
}

// ---------------------------------------------------------------------------
// A1: opacity and group Planck tables at T, with the 64-group chunk partial
// sums of dS = d/dT sum_g 2 kappa_g B_g.  Block = one 64-group chunk x 4 RUN
// cells; thread = (run of RUN consecutive groups, cell): adjacent groups of a
// run share their common edge integral.  RUN = 4 saves edge work on large
// tables; RUN = 1 gives the shortest dependent chain per thread for small
// ones.  The 64 / RUN run sums of a cell are added in LDS in a fixed order.
// ---------------------------------------------------------------------------
// One block (256 threads) of the opacity work: work item `it`.
// SPEC: slabs of the spectral model get the group averages at (T, T_r =
// (Eg / a_R)^(1/4); Eg null: T_r = T) with sigma_R in sgr (one group per step:
// the panel sums do not share edge work).
template <int RUN, bool SPEC>
__device__ inline void opacity_block(const SlabDev *__restrict__ sd, const ProbDev &pd, const Item it, const Ctl *ctl,
                                     int pmode, int lcyc, const double *__restrict__ T, double *__restrict__ kappa,
                                     double *__restrict__ B, double *__restrict__ dSpart,
                                     const double *__restrict__ Eg = nullptr, double *__restrict__ sgr = nullptr,
                                     double *__restrict__ dem = nullptr) {
  constexpr int CB = 4 * RUN, NR = 64 / RUN;  // cells per block, runs per chunk
  __shared__ double part[NR][CB + 1];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng;
  const int ncb = (nx + CB - 1) / CB;
  const int chunk = it.idx / ncb, cb = it.idx - chunk * ncb;
  const int run = threadIdx.x / CB, cl = threadIdx.x - run * CB;
  const int i = cb * CB + cl;
  const int g0 = chunk * 64 + run * RUN, g1 = min(ng, g0 + RUN);
  double dS = 0.0;
  if (i < nx && g0 < ng) {
    const double Ti = T[S.o_cell + i];
    const double Cc = pd.Ccell[S.o_cell + i];
    const double iT = 1.0 / Ti;
    const double T2 = Ti * Ti;
    const double scale = S.aR * S.c * T2 * T2 * 0.5 / TR_PI4_15;
    const double *nue = pd.nu_e + S.o_nu;
    const double *nuc = pd.nu_c + S.o_g;
    if (SPEC && S.opac == TR_OPAC_SPECTRAL) {
      const double Tr = Eg ? sqrt(sqrt(fmax(Eg[S.o_cell + i], 1e-300) / S.aR)) : Ti;
      const double K = S.aR * S.c * 0.5 / TR_PI4_15;
      for (int g = g0; g < g1; ++g) {
        double sE, src, sR;
        const double d = spectral_group(nue[g], nue[g + 1], Ti, Tr, Cc, K, sE, src, sR);
        dS += d;
        const long long o = S.o_gi + (long long)g * nx + i;
        kappa[o] = sE;
        B[o] = src / sE;
        sgr[o] = sR;
        if (dem) dem[o] = d;
      }
    } else {
      EdgeQ lo = edge_q(nue[g0], iT);
#pragma unroll
      for (int q = 0; q < RUN; ++q) {
        const int g = g0 + q;
        if (g >= g1) break;
        const EdgeQ hi = edge_q(nue[g + 1], iT);
        double kap, Bg;
        const double d = planck_group(nuc[g], lo, hi, iT, Cc, scale, kap, Bg);
        dS += d;
        const long long o = S.o_gi + (long long)g * nx + i;
        kappa[o] = kap;
        B[o] = Bg;
        if (dem) dem[o] = d;
        // a context with spectral slabs reads sigma_R from its own table:
        // the point law's sigma_R is kappa
        if (SPEC) sgr[o] = kap;
        lo = hi;
      }
    }
  }
  part[run][cl] = dS;
  __syncthreads();
  // runs r = run, run + 8, ... by the first 8 runs, then the 8 partials
  if (run < 8) {
    double acc = 0.0;
#pragma unroll
    for (int r = run; r < NR; r += 8) acc += part[r][cl];
    part[run][cl] = acc;
  }
  __syncthreads();
  if (run == 0 && i < nx) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) acc += part[r][cl];
    dSpart[S.o_chunk + (long long)chunk * nx + i] = acc;
  }
}

template <int RUN, bool SPEC>
__global__ __launch_bounds__(256) void k_opacity(const SlabDev *__restrict__ sd, ProbDev pd,
                                                 const Item *__restrict__ tab, const Ctl *ctl, int pmode, int lcyc,
                                                 const double *__restrict__ T, double *__restrict__ kappa,
                                                 double *__restrict__ B, double *__restrict__ dSpart,
                                                 const double *__restrict__ Eg, double *__restrict__ sgr,
                                                 double *__restrict__ dem) {
  opacity_block<RUN, SPEC>(sd, pd, tab[blockIdx.x], ctl, pmode, lcyc, T, kappa, B, dSpart, Eg, sgr, dem);
}

// Sums the 64-group chunk partials of dS for every cell.  Block = 64 cells
// (lanes) x 4 wavefronts; wavefront w adds the chunks q = w, w + 4, ... and
// the four partial sums are combined in a fixed order, so the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_dS_sum(const SlabDev *__restrict__ sd, const Item *__restrict__ tab,
                                                const Ctl *ctl, int pmode, int lcyc, const double *__restrict__ dSpart,
                                                double *__restrict__ dS) {
  __shared__ double part[4][64];
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, nchunk = S.nchunk;
  const long long o_chunk = S.o_chunk, o_cell = S.o_cell;
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = it.idx + lane;
  double acc = 0.0;
  if (i < nx) {
    const double *row = dSpart + o_chunk + i;
    int q = w;
    for (; q + 12 < nchunk; q += 16) {
      const double v0 = row[(long long)q * nx], v1 = row[(long long)(q + 4) * nx];
      const double v2 = row[(long long)(q + 8) * nx], v3 = row[(long long)(q + 12) * nx];
      acc += v0;
      acc += v1;
      acc += v2;
      acc += v3;
    }
    for (; q < nchunk; q += 4) acc += row[(long long)q * nx];
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < nx) dS[o_cell + i] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// ---------------------------------------------------------------------------
// A2 (+ partial A3): SCB sweep.  Work unit = (slab, group, half range).
// Per cell the 2x2 corner system makes the outflow an affine function of the
// inflow, I_dn = al I_in + be and I_up = ga I_in + de.  A pass covers 64 K
// cells in sweep order; lane l owns K consecutive of them.  A lane first
// composes its K maps in turn, one wavefront prefix scan of the 64 lane maps
// then gives every lane its inflow, and the lane applies its maps in turn;
// passes are chained by the total map of the previous pass.  Directions of
// the half range are processed in turn; the cell-average moments sum w Ibar
// and sum w mu^2 Ibar accumulate in registers.
//
// Memory: every intensity row is accessed through a raw buffer resource whose
// range is the row, so lanes past the end of the slab load zeros and their
// stores are dropped by the hardware; the loop body has no branches around
// memory operations, and the corner pairs of the next direction are loaded
// while the current one is computed.  The scan uses DPP lane moves (row
// shifts and row broadcasts), the carries between passes are lane reads.
// ---------------------------------------------------------------------------
typedef unsigned int tr_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int tr_u32x2 __attribute__((ext_vector_type(2)));
// Word 3 of a raw (unswizzled, range-checked) buffer resource on gfx9-family
// targets: 32-bit data format.
#define TR_BUF_WORD3 0x00020000

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, TR_BUF_WORD3);
}

// Corner-pair storage of the intensities: binary64 or binary32 (the sweep
// computes in binary64 either way).  When the intensity arrays are larger
// than the last-level cache the sweep streams them (each read once and
// written once per sweep, gigabytes apart from their next use) and its loads
// and stores carry the non-temporal hint (cache policy NT); smaller ones keep
// the default policy, so that the next sweep finds them cached.  `load`
// without a hint serves data read again soon (the moment partials).
#define TR_CPOL_NT 2
template <typename TI>
struct Pair;
template <>
struct Pair<double> {
  typedef double2 V;
  static __device__ inline V load(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  template <bool NT>
  static __device__ inline V load_stream(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? TR_CPOL_NT : 0));
  }
  template <bool NT>
  static __device__ inline void store_stream(V v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(tr_u32x4, v), r, off, 0, NT ? TR_CPOL_NT : 0);
  }
};
template <>
struct Pair<float> {
  typedef float2 V;
  template <bool NT>
  static __device__ inline V load_stream(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, NT ? TR_CPOL_NT : 0));
  }
  template <bool NT>
  static __device__ inline void store_stream(V v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(tr_u32x2, v), r, off, 0, NT ? TR_CPOL_NT : 0);
  }
};

__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// DPP lane move of a binary64 value; lanes without a source (or in rows not
// enabled by ROWM) keep `old`.
template <int CTRL, int ROWM>
__device__ inline double dpp_f64(double v, double old) {
  const long long vi = __double_as_longlong(v), oi = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)vi, CTRL, ROWM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(vi >> 32), CTRL, ROWM, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double readlane_f64(double v, int lane) {
  const long long vi = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)vi, lane);
  const int hi = __builtin_amdgcn_readlane((int)(vi >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One step of the inclusive scan of affine maps x -> A x + B (composition
// with the map of the source lane, applied first); the identity map is the
// value for lanes without a source.
template <int CTRL, int ROWM>
__device__ inline void scan_step(double &A, double &B) {
  const double Ap = dpp_f64<CTRL, ROWM>(A, 1.0);
  const double Bp = dpp_f64<CTRL, ROWM>(B, 0.0);
  B = fma(A, Bp, B);
  A = A * Ap;
}

enum {
  DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118,
  DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143
};

// LDS transposition buffer of a wavefront (K > 1): 64 K slots of 16 bytes;
// pass position p (sweep order) lives in slot p ^ ((p >> 3) & 7), so that
// any 8 consecutive lanes of both the segment-major accesses (lane l,
// position 64 k + l) and the lane-serial ones (lane l, position K l + k)
// touch 8 different 16-byte bank groups.
__device__ inline int tr_slot(int p) { return p ^ ((p >> 3) & 7); }

// Doubles of LDS a sweep block needs (launch argument).
__host__ __device__ inline int sweep_lds_doubles(int K, int split) {
  const int nw = split == 1 ? 4 : split;
  const int tcol = K > 1 ? 128 * K : 0;  // transposition buffer per wavefront
  return nw * tcol + (split == 1 ? 0 : split * (K * 128 + 3));
}

// One work unit's share of directions, sweeping in the direction of
// decreasing x (REV, mu < 0) or increasing x.
template <int K, typename TI, bool REV, bool NT>
__device__ inline void sweep_unit(const SlabDev &S, ProbDev pd, int g, int sub, int split,
                                  const double *__restrict__ kappa, const double *__restrict__ Bt,
                                  const TI *__restrict__ Ip, TI *__restrict__ Io, double *__restrict__ mom,
                                  double *__restrict__ bnd, double *sred) {
  typedef Pair<TI> P;
  typedef typename P::V PV;
  const int lane = threadIdx.x & 63;
  const int half = REV ? 1 : 0;
  const int nx = S.nx, ng = S.ng, M = S.nmu, Mh = M >> 1;
  const int m0 = REV ? 0 : Mh;  // mu ascending: mu < 0 first
  // this wavefront's directions m0 + [j0, j1)
  const int dw = (Mh + split - 1) / split;
  const int j0 = min(Mh, sub * dw), j1 = min(Mh, j0 + dw);
  // LDS: transposition buffers of the block's wavefronts, then (split > 1)
  // the partial moments [split][K][64] (phi, chi) and outflow sums [split][3]
  const int nw = split == 1 ? 4 : split;
  const int wslot = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2 *tb = reinterpret_cast<double2 *>(sred) + (K > 1 ? wslot * 64 * K : 0);
  double2 *red = reinterpret_cast<double2 *>(sred) + (K > 1 ? nw * 64 * K : 0);
  double *sb = reinterpret_cast<double *>(red + split * K * 64);
  const double inv_cdt = S.inv_cdt;
  const __amdgpu_buffer_rsrc_t r_dx = buf_rsrc(pd.dx + S.o_cell, nx * 8);
  const __amdgpu_buffer_rsrc_t r_kp = buf_rsrc(kappa + S.o_gi + (long long)g * nx, nx * 8);
  const __amdgpu_buffer_rsrc_t r_bp = buf_rsrc(Bt + S.o_gi + (long long)g * nx, nx * 8);
  const TI *ip = Ip + S.o_I + (long long)g * M * nx * 2;
  TI *io = Io + S.o_I + (long long)g * M * nx * 2;
  const int rowb = nx * 2 * (int)sizeof(TI);
  const double *mu = pd.mu + S.o_mu;
  const double *w = pd.w + S.o_mu;
  double carry = pd.inc[2 * S.o_g + half * ng + g];  // lane j: inflow of direction m0 + j
  const __amdgpu_buffer_rsrc_t r_mp =
      buf_rsrc(mom + 4 * S.o_gi + (long long)half * 2 * ng * nx + (long long)g * nx * 2, nx * 16);
  const int npass = (nx + 64 * K - 1) / (64 * K);
  // cells of a pass: position q in sweep order; lane l computes positions
  // K l .. K l + K - 1 (lane-serial) and moves positions 64 k + l to and from
  // memory (segment-major: each access is one contiguous block); cells
  // outside [0, nx) map to offsets outside the row's range
  auto cell_at = [&](int pass, int q) {
    const int c = pass * 64 * K + q;
    return REV ? nx - 1 - c : c;
  };
  auto cell_mem = [&](int pass, int k) { return cell_at(pass, K > 1 ? k * 64 + lane : lane); };
  auto cell_own = [&](int pass, int k) { return cell_at(pass, lane * K + k); };
  PV nxt[K];
  {
    // a wavefront without directions reads nothing (empty range)
    const __amdgpu_buffer_rsrc_t r =
        buf_rsrc(ip + (long long)(m0 + (j0 < j1 ? j0 : 0)) * nx * 2, j0 < j1 ? rowb : 0);
#pragma unroll
    for (int k = 0; k < K; ++k) nxt[k] = P::template load_stream<NT>(r, cell_mem(0, k) * 2 * (int)sizeof(TI));
  }
  for (int pass = 0; pass < npass; ++pass) {
    double bb[K], ee[K], phi[K], chi[K], hh[K];
    int off[K];
    bool ok[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = cell_own(pass, k);
      ok[k] = i >= 0 && i < nx;
      off[k] = cell_mem(pass, k) * 2 * (int)sizeof(TI);
      const double dxi = buf_load_f64(r_dx, i * 8);
      const double kap = buf_load_f64(r_kp, i * 8);
      const double bpl = buf_load_f64(r_bp, i * 8);
      bb[k] = 0.5 * (kap + inv_cdt) * dxi;
      ee[k] = 0.5 * dxi * kap * bpl;
      hh[k] = 0.5 * dxi * inv_cdt;
      phi[k] = 0.0;
      chi[k] = 0.0;
    }
    for (int j = j0; j < j1; ++j) {
      const int m = m0 + j;
      double cx[K], cy[K];  // corner pair of the lane's cells (left, right)
      if (K > 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) tb[tr_slot(k * 64 + lane)] = make_double2((double)nxt[k].x, (double)nxt[k].y);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double2 v = tb[tr_slot(K * lane + k)];
          cx[k] = v.x;
          cy[k] = v.y;
        }
      } else {
        cx[0] = (double)nxt[0].x;
        cy[0] = (double)nxt[0].y;
      }
      {
        // next direction of this pass, else the first direction of the next
        // pass (past the last pass every offset is out of range)
        const bool same = j + 1 < j1;
        const __amdgpu_buffer_rsrc_t r = buf_rsrc(ip + (long long)(same ? m + 1 : m0 + j0) * nx * 2, rowb);
#pragma unroll
        for (int k = 0; k < K; ++k) nxt[k] = P::template load_stream<NT>(r, cell_mem(same ? pass : pass + 1, k) * 2 * (int)sizeof(TI));
      }
      const double mum = mu[m], wm = w[m];
      const double amu = fabs(mum), a = 0.5 * amu, a2 = a * a, aamu = a * amu;
      const double wmu2 = wm * mum * mum;
      double al[K], be[K], ga[K], de[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double up = REV ? cy[k] : cx[k];
        const double dn = REV ? cx[k] : cy[k];
        const double s_up = fma(hh[k], up, ee[k]);
        const double s_dn = fma(hh[k], dn, ee[k]);
        const double apb = a + bb[k];
        const double r = rcp_nr(fma(apb, apb, a2));
        al[k] = ok[k] ? aamu * r : 1.0;
        ga[k] = ok[k] ? apb * amu * r : 0.0;
        be[k] = ok[k] ? fma(apb, s_dn, a * s_up) * r : 0.0;
        de[k] = ok[k] ? fma(apb, s_up, -a * s_dn) * r : 0.0;
      }
      // the lane's map: its K cell maps composed in sweep order
      double A = al[0], Bc = be[0];
#pragma unroll
      for (int k = 1; k < K; ++k) {
        Bc = fma(al[k], Bc, be[k]);
        A = A * al[k];
      }
      // inclusive scan of the lane maps
      scan_step<DPP_ROW_SHR1, 0xf>(A, Bc);
      scan_step<DPP_ROW_SHR2, 0xf>(A, Bc);
      scan_step<DPP_ROW_SHR4, 0xf>(A, Bc);
      scan_step<DPP_ROW_SHR8, 0xf>(A, Bc);
      scan_step<DPP_ROW_BCAST15, 0xa>(A, Bc);
      scan_step<DPP_ROW_BCAST31, 0xc>(A, Bc);
      // inflow of the lane: the maps of the lanes before it applied to the
      // pass inflow
      const double cin = readlane_f64(carry, j);
      const double Ae = dpp_f64<DPP_WAVE_SHR1, 0xf>(A, 1.0);
      const double Be = dpp_f64<DPP_WAVE_SHR1, 0xf>(Bc, 0.0);
      double Iin = fma(Ae, cin, Be);
      double ox[K], oy[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double Iup = fma(ga[k], Iin, de[k]);
        const double Idn = fma(al[k], Iin, be[k]);
        ox[k] = REV ? Idn : Iup;
        oy[k] = REV ? Iup : Idn;
        const double Ibar = 0.5 * (Iup + Idn);
        phi[k] = fma(wm, Ibar, phi[k]);
        chi[k] = fma(wmu2, Ibar, chi[k]);
        Iin = Idn;
      }
      const __amdgpu_buffer_rsrc_t ro = buf_rsrc(io + (long long)m * nx * 2, rowb);
      if (K > 1) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) tb[tr_slot(K * lane + k)] = make_double2(ox[k], oy[k]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double2 v = tb[tr_slot(k * 64 + lane)];
          PV o;
          o.x = (TI)v.x;
          o.y = (TI)v.y;
          P::template store_stream<NT>(o, ro, off[k]);
        }
        __builtin_amdgcn_wave_barrier();
      } else {
        PV o;
        o.x = (TI)ox[0];
        o.y = (TI)oy[0];
        P::template store_stream<NT>(o, ro, off[0]);
      }
      const double cout = fma(readlane_f64(A, 63), cin, readlane_f64(Bc, 63));
      if (lane == j) carry = cout;
    }
    // cell moments of the pass (lane-serial) to memory (segment-major)
    if (split > 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) red[(sub * K + k) * 64 + lane] = make_double2(phi[k], chi[k]);
      __syncthreads();
      if (sub == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          for (int q = 1; q < split; ++q) {
            const double2 v = red[(q * K + k) * 64 + lane];
            phi[k] += v.x;
            chi[k] += v.y;
          }
        }
      }
    }
    if (sub == 0) {
      if (K > 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) tb[tr_slot(K * lane + k)] = make_double2(phi[k], chi[k]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double2 o = tb[tr_slot(k * 64 + lane)];
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(tr_u32x4, o), r_mp, cell_mem(pass, k) * 16, 0,
                                                 0);
        }
        __builtin_amdgcn_wave_barrier();
      } else {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(tr_u32x4, make_double2(phi[0], chi[0])), r_mp,
                                               cell_mem(pass, 0) * 16, 0, 0);
      }
    }
    if (split > 1) __syncthreads();
  }
  // outflow-edge sums of this half range: carry = intensity leaving the slab
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (lane >= j0 && lane < j1) {
    const double wl = w[m0 + lane], ml = mu[m0 + lane];
    s0 = wl * carry;
    s1 = wl * ml * carry;
    s2 = wl * ml * ml * carry;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    s0 += __shfl_xor(s0, d);
    s1 += __shfl_xor(s1, d);
    s2 += __shfl_xor(s2, d);
  }
  double *bo = bnd + 6 * S.o_g + (long long)half * 3 * ng + 3 * g;
  if (split == 1) {
    if (lane == 0) {
      bo[0] = s0;
      bo[1] = s1;
      bo[2] = s2;
    }
    return;
  }
  if (lane == 0) {
    sb[3 * sub] = s0;
    sb[3 * sub + 1] = s1;
    sb[3 * sub + 2] = s2;
  }
  __syncthreads();
  if (sub == 0 && lane < 3) {
    double t = sb[lane];
    for (int q = 1; q < split; ++q) t += sb[3 * q + lane];
    bo[lane] = t;
  }
}

// split = 1: a wavefront sweeps all directions of one (group, half range);
// blocks of 4 such wavefronts.  split = 2 or 4: a block of split wavefronts
// shares one (group, half range), wavefront `sub` taking a contiguous share
// of its directions; the moment and outflow partials are added through LDS
// in wavefront order (more wavefronts in flight for small problems).
template <int K, typename TI, bool NT>
__global__ __launch_bounds__(256) void k_sweep(const SlabDev *__restrict__ sd, ProbDev pd,
                                               const Item *__restrict__ tab, int nitems, int split, const Ctl *ctl,
                                               int pmode, int lcyc, const double *__restrict__ kappa,
                                               const double *__restrict__ Bt, const TI *__restrict__ Ip,
                                               TI *__restrict__ Io, double *__restrict__ mom,
                                               double *__restrict__ bnd) {
  extern __shared__ double sred[];  // split > 1: [split][K][64] (phi, chi), then [split][3]
  // wavefront indices, made visibly uniform so that the descriptors and the
  // per-direction quantities live in scalar registers (split is uniform: the
  // whole block of a split sweep exits together)
  const int unit = split == 1
                       ? __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6))
                       : (int)blockIdx.x;
  const int sub = split == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int item = unit >> 1, half = unit & 1;
  if (item >= nitems) return;
  const Item it = tab[item];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  if (half)
    sweep_unit<K, TI, true, NT>(S, pd, it.idx, sub, split, kappa, Bt, Ip, Io, mom, bnd, sred);
  else
    sweep_unit<K, TI, false, NT>(S, pd, it.idx, sub, split, kappa, Bt, Ip, Io, mom, bnd, sred);
}

// ---------------------------------------------------------------------------
// A3: QD factors from the half-range partials.  Thread = (slab, g, i); the
// i = 0 thread of each group also forms the boundary factors.
// ---------------------------------------------------------------------------
// Cell factor f = chi / phi of the summed half-range moments (the isotropic
// value where phi underflows).
__device__ inline double cell_factor(double phi, double chi, double f_iso) {
  return (phi > TR_TINY && chi > 0.0) ? chi / phi : f_iso;
}

// Boundary factors of a group from the outflow sums of the half range
// leaving at x = 0 (b1: mu < 0) and at x = X (b0: mu > 0) and the incoming
// intensities inl / inr: edge factors, C and Phi = F_in - c C E_in per side.
struct BndFac {
  double fb0, fb1, C0, C1, P0, P1;
};
__device__ inline BndFac boundary_factors(const SlabDev &S, double inl, double inr, const double *b0,
                                          const double *b1) {
  BndFac o;
  {
    const double den = b1[0] + inl * S.wpos, num = b1[2] + inl * S.wmu2pos;
    o.fb0 = (den > TR_TINY && num > 0.0) ? num / den : S.f_iso;
    o.C0 = (b1[0] > TR_TINY) ? b1[1] / b1[0] : -S.c_iso;
    o.P0 = inl * S.wmupos - S.c * o.C0 * (inl * S.wpos / S.c);
  }
  {
    const double den = b0[0] + inr * S.wneg, num = b0[2] + inr * S.wmu2neg;
    o.fb1 = (den > TR_TINY && num > 0.0) ? num / den : S.f_iso;
    o.C1 = (b0[0] > TR_TINY) ? b0[1] / b0[0] : S.c_iso;
    o.P1 = inr * S.wmuneg - S.c * o.C1 * (inr * S.wneg / S.c);
  }
  return o;
}

__global__ __launch_bounds__(256) void k_moments(const SlabDev *__restrict__ sd, ProbDev pd,
                                                 const Item *__restrict__ tab, const Ctl *ctl, int pmode, int lcyc,
                                                 const double *__restrict__ mom, const double *__restrict__ bnd,
                                                 double *__restrict__ f, double *__restrict__ fbnd,
                                                 double *__restrict__ C, double *__restrict__ Phi) {
  const Item it = tab[blockIdx.x];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng;
  const int idx = it.idx + threadIdx.x;
  if (idx >= ng * nx) return;
  const int g = idx / nx, i = idx - g * nx;
  const double *h0 = mom + 4 * S.o_gi + 2LL * idx;
  const double *h1 = h0 + 2LL * ng * nx;
  const double phi = h0[0] + h1[0];
  const double chi = h0[1] + h1[1];
  f[S.o_gi + idx] = cell_factor(phi, chi, S.f_iso);
  if (i != 0) return;
  const double inl = pd.inc[2 * S.o_g + g], inr = pd.inc[2 * S.o_g + ng + g];
  const double *b0 = bnd + 6 * S.o_g + 3 * g;            // mu > 0: leaves at x = X
  const double *b1 = bnd + 6 * S.o_g + 3 * ng + 3 * g;   // mu < 0: leaves at x = 0
  const long long o2 = 2 * S.o_g + 2 * g;
  const BndFac o = boundary_factors(S, inl, inr, b0, b1);
  fbnd[o2] = o.fb0;
  C[o2] = o.C0;
  Phi[o2] = o.P0;
  fbnd[o2 + 1] = o.fb1;
  C[o2 + 1] = o.C1;
  Phi[o2 + 1] = o.P1;
}

// Phi = F_in - c C E_in from given C and the current incoming (step start).
__device__ inline void phi_groups(const SlabDev *__restrict__ sd, const ProbDev &pd, const Item it,
                                  const double *__restrict__ C, double *__restrict__ Phi) {
  const SlabDev &S = sd[it.slab];
  const int g = it.idx + threadIdx.x;
  if (g >= S.ng) return;
  const double inl = pd.inc[2 * S.o_g + g], inr = pd.inc[2 * S.o_g + S.ng + g];
  const long long o2 = 2 * S.o_g + 2 * g;
  Phi[o2] = inl * S.wmupos - S.c * C[o2] * (inl * S.wpos / S.c);
  Phi[o2 + 1] = inr * S.wmuneg - S.c * C[o2 + 1] * (inr * S.wneg / S.c);
}

// ---------------------------------------------------------------------------
// Edge and cell coefficients of one LO level.
//   edge e (0..nx):  h_e, A_e = h_e / (c dt), a_e, b_e, sigma_R,e, F^old_e
//   cell i:          sigma_E,i, e_i (emission), E^old_i
// MODE 0: fine grid from kappa/B tables and QD factors; MODE 1: level arrays.
// ---------------------------------------------------------------------------
struct LevelView {
  int nx;
  const double *dx;
  // fine (sgr: cell sigma_R, the kappa table under the point law)
  const double *kap, *Bt, *f, *fbnd, *sgr;
  // coarse
  const double *sigE, *emis, *a, *b, *sigR;
  // both
  const double *C, *Phi, *Eold, *Fold;
};

__device__ inline double lv_h(const LevelView &v, int e) {
  if (e == 0) return 0.5 * v.dx[0];
  if (e == v.nx) return 0.5 * v.dx[v.nx - 1];
  return 0.5 * (v.dx[e - 1] + v.dx[e]);
}

template <bool FINE>
__device__ inline void lv_edge(const LevelView &v, int e, double &ae, double &be, double &sr) {
  const int nx = v.nx;
  if (FINE) {
    ae = (e < nx) ? v.f[e] : v.fbnd[1];
    be = (e > 0) ? v.f[e - 1] : v.fbnd[0];
    if (e == 0)
      sr = v.sgr[0];
    else if (e == nx)
      sr = v.sgr[nx - 1];
    else
      sr = (v.sgr[e - 1] * v.dx[e - 1] + v.sgr[e] * v.dx[e]) / (v.dx[e - 1] + v.dx[e]);
  } else {
    ae = v.a[e];
    be = v.b[e];
    sr = v.sigR[e];
  }
}

template <bool FINE>
__device__ inline void lv_cell(const LevelView &v, int i, double &se, double &em) {
  if (FINE) {
    se = v.kap[i];
    em = 2.0 * v.kap[i] * v.Bt[i];
  } else {
    se = v.sigE[i];
    em = v.emis[i];
  }
}

// Level data of the K rows of this thread (row k = unknown j = t K + k;
// j = 0 and j = nx + 1 are the boundary unknowns, cell i = j - 1 otherwise):
// edges e = t K - 1 .. t K + K - 1.  Loaded in one batch so that the loads
// are in flight together.
template <int K>
struct RowData {
  double ae[K + 1], be[K + 1], sr[K + 1], h[K + 1], Fo[K + 1];
  double dx[K], Eo[K], se[K], em[K];
  double C0, C1, P0, P1;
};

// Factor source of the first fine solve of an iteration with a sweep: the
// group's half-range partial rows (phi, chi per cell), its boundary factors
// and the row its cell factors are written to.
struct FacSrc {
  __amdgpu_buffer_rsrc_t r0, r1, rf;
  double f_iso;
  BndFac bf;
};

template <int K, bool FINE, bool MOM = false>
__device__ inline void lo_load(const LevelView &v, RowData<K> &R, const FacSrc *fs = nullptr) {
  // branch-free: buffer loads outside a row's range return zero, so every
  // load of the thread is issued before the first use
  const int t = threadIdx.x, nx = v.nx;
  const int cb = nx * 8, eb = (nx + 1) * 8;
  const __amdgpu_buffer_rsrc_t r_dx = buf_rsrc(v.dx, cb), r_Fo = buf_rsrc(v.Fold, eb), r_Eo = buf_rsrc(v.Eold, cb);
  // MOM: factors of cells t K - 2 .. t K + K - 1 from the partials (zero
  // outside the slab, as the factor loads are); the thread's own cells
  // t K - 1 .. t K + K - 2 are written (stores outside the row are dropped)
  double fc[K + 2];
  if (MOM) {
#pragma unroll
    for (int j = 0; j < K + 2; ++j) {
      const int i = t * K - 2 + j;
      const double2 h0 = Pair<double>::load(fs->r0, i * 16), h1 = Pair<double>::load(fs->r1, i * 16);
      fc[j] = (i >= 0 && i < nx) ? cell_factor(h0.x + h1.x, h0.y + h1.y, fs->f_iso) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(tr_u32x2, fc[k + 1]), fs->rf, (t * K - 1 + k) * 8, 0,
                                            0);
  }
  // cell values of cells t K - 2 .. t K + K - 1 (the thread's cells and one
  // on each side), each loaded once: edge q = e - t K + 1 lies between cells
  // q and q + 1 of these
  double dxv[K + 2], fv[K + 2], sgv[K + 2];
#pragma unroll
  for (int j = 0; j < K + 2; ++j) {
    const int i = t * K - 2 + j;
    dxv[j] = buf_load_f64(r_dx, i * 8);
    if (FINE) {
      fv[j] = MOM ? fc[j] : buf_load_f64(buf_rsrc(v.f, cb), i * 8);
      sgv[j] = buf_load_f64(buf_rsrc(v.sgr, cb), i * 8);
    }
  }
#pragma unroll
  for (int q = 0; q <= K; ++q) {
    const int e = t * K - 1 + q;
    const bool in = e >= 0 && e <= nx;
    const double dxm = dxv[q], dxe = dxv[q + 1];
    R.h[q] = in ? 0.5 * (dxm + dxe) : 1.0;
    R.Fo[q] = buf_load_f64(r_Fo, e * 8);
    if (FINE) {
      // cell sigma_R of the edge's two cells (the kappa table under the point law)
      const double fe = fv[q + 1], fm = fv[q];
      const double ke = sgv[q + 1], km = sgv[q];
      // boundary factors are added (the cell loads are zero there), so that
      // no load is conditional
      R.ae[q] = fe + (e == nx ? (MOM ? fs->bf.fb1 : v.fbnd[1]) : 0.0);
      R.be[q] = fm + (e == 0 ? (MOM ? fs->bf.fb0 : v.fbnd[0]) : 0.0);
      // width-weighted sigma_R of the two cells (one cell on the boundary)
      const double id = (e > 0 && e < nx) ? 1.0 / (dxm + dxe) : 0.0;
      const double wm = (e == nx) ? 1.0 : dxm * id, we = (e == 0) ? 1.0 : dxe * id;
      R.sr[q] = km * wm + ke * we;
    } else {
      R.ae[q] = buf_load_f64(buf_rsrc(v.a, eb), e * 8);
      R.be[q] = buf_load_f64(buf_rsrc(v.b, eb), e * 8);
      R.sr[q] = buf_load_f64(buf_rsrc(v.sigR, eb), e * 8);
    }
  }
  // kappa is the sigma_R table itself unless a separate one is given
  const bool kap_is_sgr = FINE && v.kap == v.sgr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k - 1;
    R.dx[k] = dxv[k + 1];
    R.Eo[k] = buf_load_f64(r_Eo, i * 8);
    if (FINE) {
      const double kap = kap_is_sgr ? sgv[k + 1] : buf_load_f64(buf_rsrc(v.kap, cb), i * 8);
      R.se[k] = kap;
      R.em[k] = 2.0 * kap * buf_load_f64(buf_rsrc(v.Bt, cb), i * 8);
    } else {
      R.se[k] = buf_load_f64(buf_rsrc(v.sigE, cb), i * 8);
      R.em[k] = buf_load_f64(buf_rsrc(v.emis, cb), i * 8);
    }
  }
  if (MOM) {
    R.C0 = fs->bf.C0;
    R.C1 = fs->bf.C1;
    R.P0 = fs->bf.P0;
    R.P1 = fs->bf.P1;
  } else {
    R.C0 = v.C[0];
    R.C1 = v.C[1];
    R.P0 = v.Phi[0];
    R.P1 = v.Phi[1];
  }
}

// Builds the K rows of this thread from its level data; with eff = true the
// absorption / emission of the cell of row k come from se_eff[k] / em_eff[k]
// (the grey level coupled to the MEB).
template <int K>
__device__ inline void lo_build(const RowData<K> &R, int nx, double c, double dt, double inv_cdt, bool eff,
                                const double (&se_eff)[K], const double (&em_eff)[K], double (&ra)[K],
                                double (&rb)[K], double (&rc)[K], double (&rd)[K], double (&Ak)[K + 1],
                                double (&ca)[K + 1], double (&cb)[K + 1]) {
  const int t = threadIdx.x;
  const double inv_dt = 1.0 / dt;
#pragma unroll
  for (int q = 0; q <= K; ++q) {
    const double A = R.h[q] * inv_cdt;
    const double ke = rcp_nr(A + R.sr[q] * R.h[q]);
    Ak[q] = ke * A * R.Fo[q];
    ca[q] = c * ke * R.ae[q];
    cb[q] = c * ke * R.be[q];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = t * K + k;
    if (j == 0) {
      ra[k] = 0.0;
      rb[k] = cb[k + 1] - c * R.C0;
      rc[k] = -ca[k + 1];
      rd[k] = R.P0 - Ak[k + 1];
    } else if (j <= nx) {
      const double se = eff ? se_eff[k] : R.se[k];
      const double em = eff ? em_eff[k] : R.em[k];
      const double dxi = R.dx[k];
      ra[k] = -cb[k];
      rb[k] = dxi * inv_dt + c * se * dxi + cb[k + 1] + ca[k];
      rc[k] = -ca[k + 1];
      rd[k] = dxi * em + dxi * inv_dt * R.Eo[k] - Ak[k + 1] + Ak[k];
    } else if (j == nx + 1) {
      ra[k] = -cb[k];
      rb[k] = ca[k] + c * R.C1;
      rc[k] = 0.0;
      rd[k] = Ak[k] - R.P1;
    } else {
      ra[k] = 0.0;
      rb[k] = 1.0;
      rc[k] = 0.0;
      rd[k] = 0.0;
    }
  }
}

// Builds the K rows of this thread (load + build).
template <int K, bool FINE>
__device__ inline void lo_rows(const LevelView &v, double c, double dt, double inv_cdt, bool eff,
                               const double (&se_eff)[K], const double (&em_eff)[K], double (&ra)[K],
                               double (&rb)[K], double (&rc)[K], double (&rd)[K], double (&Ak)[K + 1],
                               double (&ca)[K + 1], double (&cb)[K + 1]) {
  RowData<K> R;
  lo_load<K, FINE>(v, R);
  lo_build<K>(R, v.nx, c, dt, inv_cdt, eff, se_eff, em_eff, ra, rb, rc, rd, Ak, ca, cb);
}

// Writes E, boundary E and F of one system after tri_solve_block.
template <int K>
__device__ inline void lo_store(int nx, const double (&x)[K], const double (&Ak)[K + 1], const double (&ca)[K + 1],
                                const double (&cb)[K + 1], const double *first, double *E, double *F,
                                double *Ebnd) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = t * K + k;
    if (j == 0)
      Ebnd[0] = x[k];
    else if (j <= nx)
      E[j - 1] = x[k];
    else if (j == nx + 1)
      Ebnd[1] = x[k];
    // flux on edge e = j: u_e = x[k], u_{e+1} = next row
    if (j <= nx) {
      const double un = (k + 1 < K) ? x[k + 1] : first[t + 1];  // row j + 1 < T K
      F[j] = Ak[k + 1] - ca[k + 1] * un + cb[k + 1] * x[k];
    }
  }
}

template <bool FINE>
__device__ inline LevelView make_view(const SlabDev &S, ProbDev pd, int level, const LoIn &in, int p) {
  LevelView v;
  v.nx = S.nx;
  v.dx = pd.dx + S.o_cell;
  const int nx = S.nx;
  if (FINE) {
    const long long gi = S.o_gi + (long long)p * nx, g2 = 2 * S.o_g + 2 * p;
    v.kap = in.kappa + gi;
    v.sgr = (in.sgr ? in.sgr : in.kappa) + gi;
    v.Bt = in.B + gi;
    v.f = in.f + gi;
    v.fbnd = in.fbnd + g2;
    v.C = in.C + g2;
    v.Phi = in.Phi + g2;
    v.Eold = in.Eold + gi;
    v.Fold = in.Fold + S.o_ge + (long long)p * (nx + 1);
    v.sigE = v.emis = v.a = v.b = v.sigR = nullptr;
  } else {
    const long long pi = S.o_lpi[level] + (long long)p * nx;
    const long long pe = S.o_lpe[level] + (long long)p * (nx + 1);
    const long long p2 = S.o_lp2[level] + 2 * p;
    v.sigE = in.sigE + pi;
    v.emis = in.emis + pi;
    v.a = in.a + pe;
    v.b = in.b + pe;
    v.sigR = in.sigR + pe;
    v.C = in.C + p2;
    v.Phi = in.Phi + p2;
    v.Eold = in.Eold + pi;
    v.Fold = in.Fold + pe;
    v.kap = v.Bt = v.f = v.fbnd = v.sgr = nullptr;
  }
  return v;
}

template <bool FINE>
__device__ inline void level_out(const SlabDev &S, int level, int p, const LoSol &sol, double *&E, double *&F,
                                 double *&Eb) {
  const int nx = S.nx;
  if (FINE) {
    E = sol.E + S.o_gi + (long long)p * nx;
    F = sol.F + S.o_ge + (long long)p * (nx + 1);
    Eb = sol.Ebnd + 2 * S.o_g + 2 * p;
  } else {
    E = sol.E + S.o_lpi[level] + (long long)p * nx;
    F = sol.F + S.o_lpe[level] + (long long)p * (nx + 1);
    Eb = sol.Ebnd + S.o_lp2[level] + 2 * p;
  }
}

// ---------------------------------------------------------------------------
// A4 / A6: LO solve, one thread block per (slab, group of the level).
// ---------------------------------------------------------------------------
// MOM (fine level, first cycle of an iteration with a sweep): the group's QD
// factors are formed here from the sweep's half-range partials, with the
// arithmetic of k_moments, and written for the restriction and later cycles.
template <int K, bool FINE, bool MOM>
__global__ __launch_bounds__(512) void k_lo(const SlabDev *__restrict__ sd, ProbDev pd, const Item *__restrict__ tab,
                                            const Ctl *ctl, int pmode, int lcyc, int level, LoIn in, LoSol sol) {
  extern __shared__ double lds[];  // tri_lds_doubles(blockDim) doubles (launch argument)
  const Item it = tab[blockIdx.x];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int p = it.idx;
  const LevelView v = make_view<FINE>(S, pd, level, in, p);
  double ra[K], rb[K], rc[K], rd[K], x[K], Ak[K + 1], ca[K + 1], cb[K + 1], dummy[K];
  if (MOM) {
    const int nx = S.nx, ng = S.ng;
    FacSrc fs;
    fs.r0 = buf_rsrc(in.mom + 4 * S.o_gi + 2LL * p * nx, nx * 16);
    fs.r1 = buf_rsrc(in.mom + 4 * S.o_gi + 2LL * ng * nx + 2LL * p * nx, nx * 16);
    fs.rf = buf_rsrc(in.f_out + S.o_gi + (long long)p * nx, nx * 8);
    fs.f_iso = S.f_iso;
    const double inl = pd.inc[2 * S.o_g + p], inr = pd.inc[2 * S.o_g + ng + p];
    fs.bf = boundary_factors(S, inl, inr, in.bnd + 6 * S.o_g + 3 * p, in.bnd + 6 * S.o_g + 3 * ng + 3 * p);
    if (threadIdx.x == 0) {
      const long long o2 = 2 * S.o_g + 2 * p;
      in.fbnd_out[o2] = fs.bf.fb0;
      in.fbnd_out[o2 + 1] = fs.bf.fb1;
      in.C_out[o2] = fs.bf.C0;
      in.C_out[o2 + 1] = fs.bf.C1;
      in.Phi_out[o2] = fs.bf.P0;
      in.Phi_out[o2 + 1] = fs.bf.P1;
    }
    RowData<K> R;
    lo_load<K, true, true>(v, R, &fs);
    lo_build<K>(R, nx, S.c, S.dt, S.inv_cdt, false, dummy, dummy, ra, rb, rc, rd, Ak, ca, cb);
  } else {
    lo_rows<K, FINE>(v, S.c, S.dt, S.inv_cdt, false, dummy, dummy, ra, rb, rc, rd, Ak, ca, cb);
  }
  tri_solve_block<K>(ra, rb, rc, rd, x, lds, blockDim.x);
  double *E, *F, *Eb;
  level_out<FINE>(S, level, p, sol, E, F, Eb);
  lo_store<K>(S.nx, x, Ak, ca, cb, lds, E, F, Eb);
}

// ---------------------------------------------------------------------------
// A5: restriction.  Sum records per (block of finer groups, edge e): e < nx
// also carries the sums of cell e, e = 0 / nx the boundary sums of side 0 / 1.
// ---------------------------------------------------------------------------
// The old-time sums (R_EOLD, R_FOLD) are constant during a time step: a step
// restricts them in its first cycle only (OLD); records without them hold
// R_NC fields.  In a grey stage (Alg. 3) the fine-to-coarse restriction
// computes kappa and B at the stage temperature itself (mode RM_OPAC) and
// leaves per-cell partial sums of dS; the coarse-to-grey restriction of the
// same stage adds them up as one more record field, R_DS (mode RM_DSF).
enum {
  R_E = 0, R_SEE, R_SE, R_EM,               // cell
  R_ER, R_AER, R_A, R_EL, R_BEL, R_B,       // edge: right / left weights
  R_AF, R_SAF, R_S, R_SF, R_F,              // edge: |F| weights, flux sums
  R_EB, R_CEB, R_C, R_PHI,                  // boundary side
  R_EOLD, R_FOLD,                           // old-time cell / edge sums
  R_N,
  R_DS = R_N,                               // stage dS of cell e (RM_DSF)
  R_NA                                      // accumulator size
};
constexpr int R_NC = R_EOLD;
enum { RM_PLAIN = 0, RM_OPAC = 1, RM_DSF = 2 };
// Fields of a record: the present sums in enum order, then R_DS (RM_DSF).
template <bool OLD, int MODE>
constexpr int rec_fields() { return (OLD ? R_N : R_NC) + (MODE == RM_DSF ? 1 : 0); }
template <bool OLD>
__device__ inline int rec_src(int k) {  // accumulator index of record field k
  return k < (OLD ? R_N : R_NC) ? k : R_DS;
}

// Values of one finer group at edge e (lane), loaded without branches:
// buffer loads out of a row's range (cell e = nx, cell e - 1 = -1, lanes past
// the last edge) return zero, and boundary values are selected per lane.
struct EdgeVals {
  double se, em;           // cell e (zero for e = nx)
  double ae, be, sr;       // edge e
  double ER, EL, F;        // E right / left of the edge, flux
  double Eo, Fo;           // old-time cell / edge values (OLD only)
  double ds;               // stage dS partials of cell e (RM_DSF only)
  double Eb0, Eb1, C0, C1, P0, P1;  // group boundary values (wave-uniform)
};

// Per-lane geometry of edge e: weights of the left / right cell in the
// width-weighted fine sigma_R average (0 / 1 and 1 / 0 on the boundary edges)
// and h, the half width of the cells beside the edge (of the one cell on a
// boundary edge).
struct EdgeGeo {
  int e, nx;
  double wm, we, h;
};

__device__ inline EdgeGeo edge_geo(const SlabDev &S, ProbDev pd, int e) {
  EdgeGeo q;
  q.e = e;
  q.nx = S.nx;
  const __amdgpu_buffer_rsrc_t r = buf_rsrc(pd.dx + S.o_cell, S.nx * 8);
  const double dm = buf_load_f64(r, (e - 1) * 8), de = buf_load_f64(r, e * 8);
  // widths outside the slab read as zero
  const double id = (e > 0 && e < S.nx) ? rcp_nr(dm + de) : 0.0;
  q.wm = (e == S.nx) ? 1.0 : dm * id;
  q.we = (e == 0) ? 1.0 : de * id;
  q.h = 0.5 * (dm + de);
  return q;
}

// Stage opacity of the lane's own cell c = e - 1 (RM_OPAC): 1 / T, the
// opacity constant and the Planck scale, zero for cells outside the slab.
struct CellOpac {
  double iT, Cc, scale;
  const double *nue, *nuc;
};

__device__ inline CellOpac cell_opac(const SlabDev &S, ProbDev pd, const double *T, int c) {
  CellOpac o;
  const bool in = c >= 0 && c < S.nx;
  const double Tc = in ? buf_load_f64(buf_rsrc(T + S.o_cell, S.nx * 8), c * 8) : 1.0;
  o.Cc = buf_load_f64(buf_rsrc(pd.Ccell + S.o_cell, S.nx * 8), c * 8);
  o.iT = 1.0 / Tc;
  const double T2 = Tc * Tc;
  o.scale = in ? S.aR * S.c * T2 * T2 * 0.5 / TR_PI4_15 : 0.0;
  o.nue = pd.nu_e + S.o_nu;
  o.nuc = pd.nu_c + S.o_g;
  return o;
}

// Loads group g of level `from` at edge q.e (g wave-uniform).  With valid
// false every value is zero (empty buffer ranges, boundary values times 0),
// so that the caller can add it without a branch.  RM_OPAC: the cell values
// kappa / B come from the caller (km, ke: cells e - 1, e; Be: cell e).
// RM_DSF: v.ds = the dS partials of coarse group g at cell e (dsp partials
// per coarse group, row stride nx).
template <bool FINE, bool OLD, int MODE>
__device__ inline void load_group(const SlabDev &S, int from, const LoIn &in, const LoSol &sol, int g, bool valid,
                                  const EdgeGeo &q, double km, double ke, double Be, const double *dsop, int dsp,
                                  EdgeVals &v) {
  const int nx = S.nx, e = q.e;
  const int oe = e * 8, om = (e - 1) * 8;
  const int cb = valid ? nx * 8 : 0, eb = valid ? (nx + 1) * 8 : 0;
  const double m = valid ? 1.0 : 0.0;
  if (FINE) {
    const long long gi = S.o_gi + (long long)g * nx, ge = S.o_ge + (long long)g * (nx + 1);
    const long long g2 = 2 * S.o_g + 2 * (long long)g;
    double sre, srm;  // cell sigma_R right / left of the edge
    if (MODE != RM_OPAC) {
      const __amdgpu_buffer_rsrc_t rk = buf_rsrc(in.kappa + gi, cb), rb = buf_rsrc(in.B + gi, cb);
      ke = buf_load_f64(rk, oe);
      km = buf_load_f64(rk, om);
      Be = buf_load_f64(rb, oe);
      if (in.sgr && in.sgr != in.kappa) {  // spectral slabs: a table of its own
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(in.sgr + gi, cb);
        sre = buf_load_f64(rs, oe);
        srm = buf_load_f64(rs, om);
      } else {
        sre = ke;
        srm = km;
      }
    } else {
      sre = ke;
      srm = km;
    }
    const __amdgpu_buffer_rsrc_t rf = buf_rsrc(in.f + gi, cb), rE = buf_rsrc(sol.E + gi, cb);
    const __amdgpu_buffer_rsrc_t rF = buf_rsrc(sol.F + ge, eb);
    const double fe = buf_load_f64(rf, oe), fm = buf_load_f64(rf, om);
    const double Ee = buf_load_f64(rE, oe), Em = buf_load_f64(rE, om);
    v.F = buf_load_f64(rF, oe);
    if (OLD) {
      v.Eo = buf_load_f64(buf_rsrc(in.Eold + gi, cb), oe);
      v.Fo = buf_load_f64(buf_rsrc(in.Fold + ge, eb), oe);
    }
    const double fb0 = m * in.fbnd[g2], fb1 = m * in.fbnd[g2 + 1];
    v.Eb0 = m * sol.Ebnd[g2];
    v.Eb1 = m * sol.Ebnd[g2 + 1];
    v.C0 = m * in.C[g2];
    v.C1 = m * in.C[g2 + 1];
    v.P0 = m * in.Phi[g2];
    v.P1 = m * in.Phi[g2 + 1];
    v.se = m * ke;
    v.em = m * (2.0 * ke * Be);
    // out-of-range loads are zero: boundary values are added, not selected,
    // so that every load is used on every lane (no branch around a load)
    v.ae = fe + (e == nx ? fb1 : 0.0);
    v.be = fm + (e == 0 ? fb0 : 0.0);
    v.sr = m * (srm * q.wm + sre * q.we);
    v.ER = Ee + (e == nx ? v.Eb1 : 0.0);
    v.EL = Em + (e == 0 ? v.Eb0 : 0.0);
  } else {
    const long long pi = S.o_lpi[from] + (long long)g * nx, pe = S.o_lpe[from] + (long long)g * (nx + 1);
    const long long p2 = S.o_lp2[from] + 2 * (long long)g;
    v.se = buf_load_f64(buf_rsrc(in.sigE + pi, cb), oe);
    v.em = buf_load_f64(buf_rsrc(in.emis + pi, cb), oe);
    v.ae = buf_load_f64(buf_rsrc(in.a + pe, eb), oe);
    v.be = buf_load_f64(buf_rsrc(in.b + pe, eb), oe);
    v.sr = buf_load_f64(buf_rsrc(in.sigR + pe, eb), oe);
    const __amdgpu_buffer_rsrc_t rE = buf_rsrc(sol.E + pi, cb);
    const double Ee = buf_load_f64(rE, oe), Em = buf_load_f64(rE, om);
    v.F = buf_load_f64(buf_rsrc(sol.F + pe, eb), oe);
    if (OLD) {
      v.Eo = buf_load_f64(buf_rsrc(in.Eold + pi, cb), oe);
      v.Fo = buf_load_f64(buf_rsrc(in.Fold + pe, eb), oe);
    }
    if (MODE == RM_DSF) {
      const double *row = dsop + S.o_dsop + (long long)g * dsp * nx;
      double t = 0.0;
      for (int b = 0; b < dsp; ++b) t += buf_load_f64(buf_rsrc(row + (long long)b * nx, cb), oe);
      v.ds = t;
    }
    v.Eb0 = m * sol.Ebnd[p2];
    v.Eb1 = m * sol.Ebnd[p2 + 1];
    v.C0 = m * in.C[p2];
    v.C1 = m * in.C[p2 + 1];
    v.P0 = m * in.Phi[p2];
    v.P1 = m * in.Phi[p2 + 1];
    v.ER = Ee + (e == nx ? v.Eb1 : 0.0);
    v.EL = Em + (e == 0 ? v.Eb0 : 0.0);
  }
}

template <bool OLD, int MODE>
__device__ inline void add_group(const EdgeVals &v, const EdgeGeo &q, double (&r)[R_NA]) {
  r[R_E] += v.ER;  // cell sums of e = nx are not used
  r[R_SEE] += v.se * v.ER;
  r[R_SE] += v.se;
  r[R_EM] += v.em;
  if (OLD) r[R_EOLD] += v.Eo;
  r[R_ER] += v.ER;
  r[R_AER] += v.ae * v.ER;
  r[R_A] += v.ae;
  r[R_EL] += v.EL;
  r[R_BEL] += v.be * v.EL;
  r[R_B] += v.be;
  const double aF = fabs(v.F);
  r[R_AF] += aF;
  r[R_SAF] += v.sr * aF;
  r[R_S] += v.sr;
  r[R_SF] += v.sr * v.F;
  r[R_F] += v.F;
  if (OLD) r[R_FOLD] += v.Fo;
  if (MODE == RM_DSF) r[R_DS] += v.ds;
  const bool b0 = q.e == 0, b1 = q.e == q.nx;
  const double Eb = b0 ? v.Eb0 : b1 ? v.Eb1 : 0.0;
  const double Cs = b0 ? v.C0 : b1 ? v.C1 : 0.0;
  r[R_EB] += Eb;
  r[R_CEB] += Cs * Eb;
  r[R_C] += Cs;
  r[R_PHI] += b0 ? v.P0 : b1 ? v.P1 : 0.0;
}

// Adds one finer group in RM_OPAC: kappa, B of the lane's own cell (ka, Ba);
// the right cell of the edge is the own cell of the next lane.
template <bool OLD, int MODE>
__device__ inline void acc_opac_group(EdgeVals &a, const EdgeGeo &q, double ka, double Ba, double (&acc)[R_NA]) {
  const double ke = dpp_f64<DPP_WAVE_SHL1, 0xf>(ka, 0.0), Be = dpp_f64<DPP_WAVE_SHL1, 0xf>(Ba, 0.0);
  a.se = ke;
  a.em = 2.0 * ke * Be;
  a.sr = ka * q.wm + ke * q.we;
  add_group<OLD, MODE>(a, q, acc);
}

// Adds finer groups [g0, g1) (wave-uniform) at this lane's edge, two groups'
// loads in flight per step, in ascending group order (a missing second group
// of an odd count adds zeros, which leaves the sums unchanged).  RM_OPAC:
// the lane also evaluates kappa, B of its own cell c = e - 1 for every group
// (the right cell's values come from the next lane) and returns the cell's
// dS partial sum over the groups.
template <bool FINE, bool OLD, int MODE>
__device__ inline double acc_groups(const SlabDev &S, ProbDev pd, int from, const LoIn &in, const LoSol &sol,
                                    int g0, int g1, const EdgeGeo &q, const double *T, const double *dsop,
                                    double (&acc)[R_NA]) {
  double dS = 0.0;
  if (MODE == RM_OPAC) {
    // one group per step: its loads are issued first and are in flight while
    // the group's opacity and Planck integrals are evaluated
    const CellOpac co = cell_opac(S, pd, T, q.e - 1);
    // narrow groups (Gauss-Legendre) first, then the wide ones by their edge
    // integrals, each in ascending order: the edge series' coefficients are
    // not live while the narrow groups are evaluated, and a wavefront with no
    // wide group skips their loop (and the coefficients' loads) entirely
    bool any_wide = false;
    for (int g = g0; g < g1; ++g) {
      const double na = co.nue[g], nb = co.nue[g + 1];
      if (!(na > 0.0 && nb <= 1.005 * na)) {  // wavefront-uniform
        any_wide = true;
        continue;
      }
      EdgeVals a;
      load_group<FINE, OLD, RM_OPAC>(S, from, in, sol, g, true, q, 0.0, 0.0, 0.0, dsop, 0, a);
      double ka, Ba;
      dS += planck_group_gl(co.nuc[g], na, nb, co.iT, co.Cc, co.scale, ka, Ba);
      acc_opac_group<OLD, MODE>(a, q, ka, Ba, acc);
    }
    EdgeQ lo;
    bool lo_ok = false;  // lo holds edge g
    for (int g = g0; any_wide && g < g1; ++g) {
      const double na = co.nue[g], nb = co.nue[g + 1];
      if (na > 0.0 && nb <= 1.005 * na) {
        lo_ok = false;
        continue;
      }
      EdgeVals a;
      load_group<FINE, OLD, RM_OPAC>(S, from, in, sol, g, true, q, 0.0, 0.0, 0.0, dsop, 0, a);
      double ka, Ba;
      if (!lo_ok) lo = edge_q(na, co.iT);
      const EdgeQ hi = edge_q(nb, co.iT);
      dS += planck_group(co.nuc[g], lo, hi, co.iT, co.Cc, co.scale, ka, Ba);
      lo = hi;
      lo_ok = true;
      acc_opac_group<OLD, MODE>(a, q, ka, Ba, acc);
    }
  } else {
    const int dsp = MODE == RM_DSF ? S.dsnp[from] / S.lev_ng[from] : 0;
    for (int g = g0; g < g1; g += 2) {
      const bool two = g + 1 < g1;
      EdgeVals a, b;
      load_group<FINE, OLD, MODE>(S, from, in, sol, g, true, q, 0.0, 0.0, 0.0, dsop, dsp, a);
      load_group<FINE, OLD, MODE>(S, from, in, sol, two ? g + 1 : g, two, q, 0.0, 0.0, 0.0, dsop, dsp, b);
      add_group<OLD, MODE>(a, q, acc);
      add_group<OLD, MODE>(b, q, acc);
    }
  }
  return dS;
}

// dS of cell i from the chunk partials of the opacity tables, for the grey
// restriction: eight interleaved partial sums (chunks q = k mod 8) keep
// eight loads in flight and are combined in a fixed order.
__device__ inline void finalize_dS(const SlabDev &S, int i, const LoOut &o) {
  if (!o.dS || i >= S.nx) return;
  const double *row = o.dSpart + S.o_chunk + i;
  const long long nx = S.nx;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  int q = 0;
  for (; q + 8 <= S.nchunk; q += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += row[(q + k) * nx];
  }
  for (int k = 0; q + k < S.nchunk; ++k) acc[k] += row[(q + k) * nx];
  o.dS[S.o_cell + i] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Final coefficients of coarse group p at edge e from the block sums.
template <bool OLD, int MODE>
__device__ inline void finalize(const SlabDev &S, int to, int p, int e, double h, int r, const double (&s)[R_NA],
                                const LoOut &o) {
  const int nx = S.nx;
  if (MODE == RM_DSF) {
    if (o.dS && e < nx) o.dS[S.o_cell + e] = s[R_DS];
  } else if (p == 0) {
    finalize_dS(S, e, o);
  }
  // weighted averages by refined reciprocals (one per weight sum, within an
  // ulp or two of the quotients); the plain average below TR_TINY weights
  const double rinv = rcp_nr((double)r);
  const double c = S.c, ic = rcp_nr(c);
  const long long pi = S.o_lpi[to] + (long long)p * nx;
  const long long pe = S.o_lpe[to] + (long long)p * (nx + 1);
  const long long p2 = S.o_lp2[to] + 2 * p;
  if (e < nx) {
    o.sigE[pi + e] = (s[R_E] > TR_TINY) ? s[R_SEE] * rcp_nr(s[R_E]) : s[R_SE] * rinv;
    o.emis[pi + e] = s[R_EM];
    if (OLD) o.Eold[pi + e] = s[R_EOLD];
    o.Esum[pi + e] = s[R_E];
  }
  const double iER = rcp_nr(s[R_ER]), iEL = rcp_nr(s[R_EL]);
  const double abar = (s[R_ER] > TR_TINY) ? s[R_AER] * iER : s[R_A] * rinv;
  const double bbar = (s[R_EL] > TR_TINY) ? s[R_BEL] * iEL : s[R_B] * rinv;
  const double sR = (s[R_AF] > TR_TINY) ? s[R_SAF] * rcp_nr(s[R_AF]) : s[R_S] * rinv;
  const double xi = h * (s[R_SF] - sR * s[R_F]);
  const double eh = (xi > 0.0 && s[R_ER] > TR_TINY) ? xi * ic * iER : 0.0;
  const double ec = (xi < 0.0 && s[R_EL] > TR_TINY) ? -xi * ic * iEL : 0.0;
  o.a[pe + e] = abar + eh;
  o.b[pe + e] = bbar + ec;
  o.sigR[pe + e] = sR;
  if (OLD) o.Fold[pe + e] = s[R_FOLD];
  if (e == 0 || e == nx) {
    const int side = (e == 0) ? 0 : 1;
    o.C[p2 + side] = (s[R_EB] > TR_TINY) ? s[R_CEB] / s[R_EB] : s[R_C] * rinv;
    o.Phi[p2 + side] = s[R_PHI];
  }
}

// Edges per wavefront tile: 64, or 63 in RM_OPAC (lane l owns cell
// 63 t + l - 1 and edge 63 t + l; lane 63 only supplies its cell's values).
template <int MODE>
__device__ __host__ constexpr int rtile() { return MODE == RM_OPAC ? 63 : 64; }

// Stage dS partials of the lanes' own cells (RM_OPAC): lanes 1..63 write
// cells 63 t .. 63 t + 62 of partial row `row`.
__device__ inline void store_dS_part(const SlabDev &S, double *dsop, long long row, int c, double v) {
  if ((threadIdx.x & 63) >= 1 && c >= 0 && c < S.nx) dsop[S.o_dsop + row * S.nx + c] = v;
}

// One-pass restriction (r <= 16 finer groups per coarse group): wavefront =
// (coarse group p, tile of edges), lane = edge; block = 4 consecutive
// wavefront items of a slab (item index 4 it.idx + w).
template <bool FINE, bool OLD, int MODE>
__global__ __launch_bounds__(256) void k_restrict(const SlabDev *__restrict__ sd, ProbDev pd,
                                                  const Item *__restrict__ tab, const Ctl *ctl, int pmode, int lcyc,
                                                  int from, int to, LoIn in, LoSol sol, LoOut out,
                                                  const double *T, double *dsop) {
  const Item it = tab[blockIdx.x];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ne = nx + 1;
  const int nto = S.lev_ng[to];
  const int r = S.lev_ng[from] / nto;
  constexpr int TE = rtile<MODE>();
  const int ntile = (ne + TE - 1) / TE;
  const int wi = 4 * it.idx + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (wi >= nto * ntile) return;
  const int p = wi / ntile, et = wi - p * ntile;
  const int lane = threadIdx.x & 63;
  const int e = et * TE + lane;
  const EdgeGeo q = edge_geo(S, pd, e);
  double acc[R_NA];
#pragma unroll
  for (int k = 0; k < R_NA; ++k) acc[k] = 0.0;
  const double dS = acc_groups<FINE, OLD, MODE>(S, pd, from, in, sol, p * r, (p + 1) * r, q, T, dsop, acc);
  if (MODE == RM_OPAC) store_dS_part(S, dsop, p, e - 1, dS);
  if (e < ne && lane < TE) finalize<OLD, MODE>(S, to, p, e, q.h, r, acc, out);
}

// Chunk pass (r > 16): block = (slab, chunk record qq = p cpb + bc, tile of
// edges); wavefront w adds groups p r + (4 bc + w) rcw + [0, rcw), lane =
// edge.  The four wavefront sums are combined through LDS in a fixed order,
// ((w0 + w2) + (w1 + w3)), and the record [edges][fields] is written
// contiguously.  RM_OPAC: the dS partials of the four wavefronts are
// combined the same way into partial row qq.
template <bool FINE, bool OLD, int MODE>
__global__ __launch_bounds__(256) void k_restrict_part(const SlabDev *__restrict__ sd, ProbDev pd,
                                                       const Item *__restrict__ tab, const Ctl *ctl, int pmode,
                                                       int lcyc, int from, int to, LoIn in, LoSol sol,
                                                       double *__restrict__ red, const double *T, double *dsop) {
  constexpr int NF = rec_fields<OLD, MODE>();
  __shared__ double sh[2][64 * NF];
  __shared__ double sds[4][64];
  const Item it = tab[blockIdx.x];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ne = nx + 1;
  const int r = S.lev_ng[from] / S.lev_ng[to];
  const int nto = S.lev_ng[to];
  const int rcw = restrict_rcw(r, nto, ne, S.rtarget), cpb = restrict_cpb(r, nto, ne, S.rtarget);
  constexpr int TE = rtile<MODE>();
  const int ntile = (ne + TE - 1) / TE;
  const int qq = it.idx / ntile, et = it.idx - qq * ntile;
  const int p = qq / cpb, bc = qq - p * cpb;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int e = et * TE + lane;
  const int g0 = p * r + (bc * 4 + w) * rcw;
  const int g1 = min(g0 + rcw, (p + 1) * r);
  const EdgeGeo q = edge_geo(S, pd, e);
  double acc[R_NA];
#pragma unroll
  for (int k = 0; k < R_NA; ++k) acc[k] = 0.0;
  const double dS = acc_groups<FINE, OLD, MODE>(S, pd, from, in, sol, g0, g1, q, T, dsop, acc);
  if (MODE == RM_OPAC) sds[w][lane] = dS;
  double *slot = sh[w & 1] + lane * NF;
  if (w >= 2) {
#pragma unroll
    for (int k = 0; k < NF; ++k) slot[k] = acc[rec_src<OLD>(k)];
  }
  __syncthreads();
  if (w < 2) {
#pragma unroll
    for (int k = 0; k < NF; ++k) acc[rec_src<OLD>(k)] += slot[k];
  }
  __syncthreads();
  if (w == 1) {
#pragma unroll
    for (int k = 0; k < NF; ++k) slot[k] = acc[rec_src<OLD>(k)];
  }
  __syncthreads();
  if (w == 0) {
    double *s1 = sh[1] + lane * NF, *s0 = sh[0] + lane * NF;
#pragma unroll
    for (int k = 0; k < NF; ++k) s0[k] = acc[rec_src<OLD>(k)] + s1[k];
    if (MODE == RM_OPAC)
      store_dS_part(S, dsop, qq, e - 1, (sds[0][lane] + sds[2][lane]) + (sds[1][lane] + sds[3][lane]));
  }
  __syncthreads();
  const int nval = min(TE, ne - et * TE) * NF;
  double *rec = red + S.o_red + ((long long)qq * ne + et * TE) * NF;
  for (int j = threadIdx.x; j < nval; j += 256) rec[j] = sh[0][j];
}

// Final pass: block = restrict_fin_edges(cpb) edges of one coarse group;
// thread = (part u, edge, field) adds the chunk records q = u, u + U, ...
// (U = 4 parts for 16 or more records, else 1); the parts are combined in a
// fixed order, ((u0 + u1) + (u2 + u3)).
template <bool OLD, int MODE>
__global__ __launch_bounds__(256) void k_restrict_final(const SlabDev *__restrict__ sd, ProbDev pd,
                                                        const Item *__restrict__ tab, const Ctl *ctl, int pmode,
                                                        int lcyc, int from, int to, LoOut out,
                                                        const double *__restrict__ red) {
  constexpr int NF = rec_fields<OLD, MODE>();
  static_assert(TR_RFIN_E * (R_NA) <= 256 && 4 * (TR_RFIN_E / 4) * R_NA <= 256, "final pass block");
  __shared__ double sums[TR_RFIN_E * R_NA];
  const Item it = tab[blockIdx.x];
  if (!pred_ok(ctl, it.slab, pmode, lcyc)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ne = nx + 1;
  const int nfrom = S.lev_ng[from], nto = S.lev_ng[to];
  const int r = nfrom / nto;
  const int cpb = restrict_cpb(r, nto, ne, S.rtarget);
  const int RE = restrict_fin_edges(cpb), U = cpb >= 16 ? 4 : 1;
  const int NP = RE * NF;  // (edge, field) pairs of the block
  const int nb = (ne + RE - 1) / RE;
  const int p = it.idx / nb, b = it.idx - p * nb;
  const int t = threadIdx.x;
  const int u = t / NP, pr = t - u * NP;
  const int el = pr / NF, k = pr - el * NF;
  const int e = b * RE + el;
  if (u < U) {
    double acc = 0.0;
    if (e < ne) {
      const long long stride = (long long)ne * NF;
      const double *rec = red + S.o_red + ((long long)p * cpb * ne + e) * NF + k + u * stride;
      // unrolled so that a part's records (16 at 64 records and 4 parts) are
      // all loaded before the first add; the adds keep their order
#pragma unroll 16
      for (int q = u; q < cpb; q += U, rec += U * stride) acc += *rec;
    }
    sums[u * NP + pr] = acc;
  }
  __syncthreads();
  if (t < RE && b * RE + t < ne) {
    double s[R_NA];
#pragma unroll
    for (int q = 0; q < R_NA; ++q) s[q] = 0.0;
    for (int q = 0; q < NF; ++q) {
      const int j = t * NF + q;
      s[rec_src<OLD>(q)] = U == 4 ? (sums[j] + sums[NP + j]) + (sums[2 * NP + j] + sums[3 * NP + j]) : sums[j];
    }
    finalize<OLD, MODE>(S, to, p, b * RE + t, edge_geo(S, pd, b * RE + t).h, r, s, out);
  }
}

// ---------------------------------------------------------------------------
// A7 + A8: grey LOQD + MEB (one Newton iteration) per slab, one thread block;
// at the end of a cycle it also applies the inner / outer convergence tests.
// The kernel is a single block on the critical path of every cycle, so all of
// its global loads (slab descriptor, control record, cell data, convergence
// references) are issued before the first dependent computation, and the
// block reductions use wavefront shuffles with one LDS exchange.
// ---------------------------------------------------------------------------
// Sums nfl and takes the maxima of v over the block (exact, order independent
// for the maxima; the integer sum is exact).  Up to 16 wavefronts; lds: 7 * 16
// doubles, which may still be read by other wavefronts on entry.
__device__ inline void block_reduce_grey(double (&v)[6], int &nfl, double *lds) {
  __syncthreads();
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] = fmax(v[q], __shfl_xor(v[q], d));
    nfl += __shfl_xor(nfl, d);
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) lds[q * 16 + w] = v[q];
    lds[96 + w] = (double)nfl;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double m = lds[q * 16];
    for (int k = 1; k < nw; ++k) m = fmax(m, lds[q * 16 + k]);
    v[q] = m;
  }
  double ns = lds[96];
  for (int k = 1; k < nw; ++k) ns += lds[96 + k];
  nfl = (int)ns;
  __syncthreads();
}

template <int K>
__global__ __launch_bounds__(512) void k_grey(const SlabDev *__restrict__ sd, ProbDev pd,
                                              const Item *__restrict__ tab, Ctl *ctl, int pmode, int lcyc,
                                              GreyArgs ga) {
  extern __shared__ double lds[];  // tri_lds_doubles(blockDim) doubles (launch argument)
  __shared__ int s_flag[2];
  // every scalar input (work item, descriptor, control record) is read
  // without branches so that the loads overlap: the control record is read
  // from slot 0 of a valid array even without control (then unused)
  const Item it = tab[blockIdx.x];
  const int slab = it.slab;
  const SlabDev &S = sd[slab];
  const int nx = S.nx;
  const long long o_cell = S.o_cell, pi = S.o_gpi;
  const double c = S.c, dt = S.dt, cv = S.cv;
  const bool has_ctl = ctl != nullptr;
  const Ctl &kc = has_ctl ? ctl[slab] : *ga.ctl_dummy;
  const int4 hd = *reinterpret_cast<const int4 *>(&kc);  // active, s, ncyc, inner_done
  const int c_ncyc = hd.z, c_s = hd.y, c_nrep = kc.n_replay, c_hasprev = kc.has_prev;
  // counters updated at the end, read with the other control fields so that
  // the update is no further round trip
  const long long c_nfloor = kc.n_floor, c_nc = kc.n_c, c_nlo = kc.n_lo;
  if (has_ctl && !pred_ok(ctl, slab, pmode, lcyc)) return;
  const int c_rep = (has_ctl && c_nrep > 0) ? kc.replay[c_s] : 0;
  const int t = threadIdx.x;
  const bool use_prev = has_ctl && c_hasprev && ga.secant;
  // per-cell inputs of this thread's rows (row k is cell t K + k - 1)
  double Ts[K], sig[K], Sst[K], Es[K], dS[K], Tol[K], Tpv[K], spv[K], Dx[K], rT[K], rE[K], sT[K], sE[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k - 1;
    const bool ok = i >= 0 && i < nx;
    const long long oc = o_cell + (ok ? i : 0), op = pi + (ok ? i : 0);
    Ts[k] = ok ? ga.Tstar[oc] : 1.0;
    sig[k] = ok ? ga.grey.sigE[op] : 0.0;
    Sst[k] = ok ? ga.grey.emis[op] : 0.0;
    Es[k] = ok ? ga.Estar[op] : 0.0;
    dS[k] = ok ? ga.dS[oc] : 0.0;
    Tol[k] = ok ? ga.Told[oc] : 0.0;
    Dx[k] = (ok && ga.D) ? ga.D[oc] : 0.0;
    Tpv[k] = (ok && use_prev) ? ga.Tprev[oc] : 0.0;
    spv[k] = (ok && use_prev) ? ga.sigprev[oc] : 0.0;
    const bool ref = ok && ga.end_cycle;
    rT[k] = ref ? ga.Tcyc[oc] : 0.0;
    rE[k] = ref ? ga.Ecyc[oc] : 0.0;
    sT[k] = ref ? ga.Ts[oc] : 0.0;
    sE[k] = ref ? ga.Es[oc] : 0.0;
  }
  // grey level coefficients of the rows (same batch of loads)
  LevelView v;
  v.nx = nx;
  v.dx = pd.dx + o_cell;
  v.sigE = ga.grey.sigE + pi;
  v.emis = ga.grey.emis + pi;
  v.a = ga.grey.a + S.o_gpe;
  v.b = ga.grey.b + S.o_gpe;
  v.sigR = ga.grey.sigR + S.o_gpe;
  v.C = ga.grey.C + S.o_gp2;
  v.Phi = ga.grey.Phi + S.o_gp2;
  v.Eold = ga.grey.Eold + pi;
  v.Fold = ga.grey.Fold + S.o_gpe;
  v.kap = v.Bt = v.f = v.fbnd = nullptr;
  RowData<K> R;
  lo_load<K, false>(v, R);
  // Newton coefficients: T - T* = alpha + beta E per cell
  double alpha[K], beta[K], se_eff[K], em_eff[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k - 1;
    alpha[k] = beta[k] = se_eff[k] = em_eff[k] = 0.0;
    if (i < 0 || i >= nx) continue;
    double D = 0.0;
    if (ga.D) {
      D = Dx[k];
    } else if (use_prev) {
      const double dT = Ts[k] - Tpv[k];
      if (fabs(dT) > 1e-8 * fabs(Ts[k])) D = (sig[k] - spv[k]) / dT;
      if (c * D * Es[k] > 0.5 * (cv / dt + dS[k])) D = 0.0;
    }
    const double iden = rcp_nr(cv / dt + dS[k] - c * D * Es[k]);
    const double al = (cv * (Tol[k] - Ts[k]) / dt - Sst[k]) * iden;
    const double gg = c * D * Es[k] - dS[k];
    alpha[k] = al;
    beta[k] = c * sig[k] * iden;
    se_eff[k] = sig[k] + gg * sig[k] * iden;
    em_eff[k] = Sst[k] - gg * al;
  }
  // rows of the grey level with effective absorption / emission
  double ra[K], rb[K], rc[K], rd[K], x[K], Ak[K + 1], ca[K + 1], cb[K + 1];
  lo_build<K>(R, nx, c, dt, S.inv_cdt, true, se_eff, em_eff, ra, rb, rc, rd, Ak, ca, cb);
  tri_solve_block<K>(ra, rb, rc, rd, x, lds, blockDim.x);
  double *E = ga.sol.E + pi, *F = ga.sol.F + S.o_gpe, *Eb = ga.sol.Ebnd + S.o_gp2;
  lo_store<K>(nx, x, Ak, ca, cb, lds, E, F, Eb);
  // temperature update, secant memory, norms
  double red[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // dTc, dEc, dTs, dEs, Tmax, Emax
  double Tn[K];
  int nfl = 0;
  double *Tout = ga.Tout + o_cell;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k - 1;
    Tn[k] = 0.0;
    if (i < 0 || i >= nx) continue;
    double T1 = Ts[k] + alpha[k] + beta[k] * x[k];
    if (T1 < 0.5 * Ts[k]) {
      T1 = 0.5 * Ts[k];
      ++nfl;
    }
    Tn[k] = T1;
    if (has_ctl) {
      ga.Tprev[o_cell + i] = Ts[k];
      ga.sigprev[o_cell + i] = sig[k];
    }
    Tout[i] = T1;
    const double En = x[k];
    if (ga.Egrey) ga.Egrey[o_cell + i] = En;
    if (ga.end_cycle) {
      red[0] = fmax(red[0], fabs(T1 - rT[k]));
      red[1] = fmax(red[1], fabs(En - rE[k]));
      red[2] = fmax(red[2], fabs(T1 - sT[k]));
      red[3] = fmax(red[3], fabs(En - sE[k]));
      // NaN propagates through fmax as the other argument; flag it explicitly
      red[4] = (T1 == T1) ? fmax(red[4], fabs(T1)) : INFINITY;
      red[5] = (En == En) ? fmax(red[5], fabs(En)) : INFINITY;
    }
  }
  if (!has_ctl) return;
  block_reduce_grey(red, nfl, lds);
  if (!ga.end_cycle) {
    if (t == 0) {
      ctl[slab].n_floor = c_nfloor + nfl;
      ctl[slab].has_prev = 1;
    }
    return;
  }
  if (t == 0) {
    Ctl &cc = ctl[slab];
    const double dTc = red[0], dEc = red[1], dTs = red[2], dEs = red[3], Tmax = red[4], Emax = red[5];
    const int ncyc = c_ncyc + 1;
    cc.n_floor = c_nfloor + nfl;
    cc.has_prev = 1;
    cc.ncyc = ncyc;
    cc.n_c = c_nc + 1;
    // LO solves of the cycle: the fine groups, the grey level and every stage
    int cost = S.lev_ng[0] + 1;
    for (int l = 1; l < TR_MAXLEV; ++l)
      if ((ga.stage_mask >> l) & 1) cost += S.lev_ng[l] + 1;
    cc.n_lo = c_nlo + cost;
    int inner_done, outer_done = 0;
    if (!isfinite(Tmax) || !isfinite(Emax)) {
      cc.err = -5;
      inner_done = 1;
      outer_done = 1;
    } else {
      const bool conv_in = dTc <= ga.eps_inner * Tmax && dEc <= ga.eps_inner * Emax;
      if (c_nrep > 0)
        inner_done = ncyc >= c_rep;
      else
        inner_done = conv_in || ncyc >= ga.lmax;
      if (inner_done) {
        if (c_s < TR_MAXOUT) cc.cycles[c_s] = ncyc;
        const bool conv_out = c_s >= 1 && dTs <= ga.eps * Tmax && dEs <= ga.eps * Emax;
        outer_done = (c_nrep > 0) ? (c_s + 1 >= c_nrep) : conv_out;
      }
    }
    cc.inner_done = inner_done;
    s_flag[0] = inner_done;
    s_flag[1] = outer_done;
  }
  __syncthreads();
  const int inner_done = s_flag[0];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t * K + k - 1;
    if (i < 0 || i >= nx) continue;
    ga.Tcyc[o_cell + i] = Tn[k];
    ga.Ecyc[o_cell + i] = x[k];
    if (inner_done) {
      ga.Ts[o_cell + i] = Tn[k];
      ga.Es[o_cell + i] = x[k];
    }
  }
  // deactivation is published last so that the cell arrays above are final
  __syncthreads();
  if (t == 0 && s_flag[1]) ctl[slab].active = 0;
}

// ---------------------------------------------------------------------------
// Control and state kernels.
// ---------------------------------------------------------------------------
// End of a transport iteration: slabs whose inner iteration finished start
// iteration s + 1 (or stop at the iteration limit / replay length), and the
// number of slabs still active is written to out[0] (out[1]: those in the
// middle of an inner iteration, ncyc > 0); when no slab is active the
// control records are also copied to hout (host memory).  One block of 256
// threads; slabs s = t, t + 256, ...; the count is summed exactly.
__global__ __launch_bounds__(256) void k_outer_end(Ctl *ctl, int nslab, int max_outer, int *out, Ctl *hout,
                                                   int *serial) {
  __shared__ int part[4], partm[4];
  // only this kernel writes the serial: read it now, with the records
  const int ser0 = threadIdx.x == 0 ? *serial : 0;
  int n = 0, nm = 0;
  for (int s = threadIdx.x; s < nslab; s += blockDim.x) {
    Ctl &c = ctl[s];
    if (c.active && c.inner_done) {
      c.s += 1;
      if (c.s > max_outer || (c.n_replay > 0 && c.s >= c.n_replay)) {
        if (c.n_replay == 0) c.err = -4;
        c.active = 0;
      } else {
        c.inner_done = 0;
        c.ncyc = 0;
        c.n_ti += 1;
      }
    }
    n += c.active;
    nm += (c.active && c.ncyc > 0) ? 1 : 0;  // inner iteration not finished by the graph
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    n += __shfl_xor(n, d);
    nm += __shfl_xor(nm, d);
  }
  if ((threadIdx.x & 63) == 0) {
    part[threadIdx.x >> 6] = n;
    partm[threadIdx.x >> 6] = nm;
  }
  __syncthreads();
  const int total = (part[0] + part[1]) + (part[2] + part[3]);
  // once every slab has stopped, the final control records go straight to
  // the host copy
  if (total == 0) {
    for (int s = threadIdx.x; s < nslab; s += blockDim.x) hout[s] = ctl[s];
    __threadfence_system();
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = total;
    out[1] = (partm[0] + partm[1]) + (partm[2] + partm[3]);
    // the iteration's serial number last: a host that sees it also sees the
    // counts and records written above
    const int ser = ser0 + 1;
    *serial = ser;
    __threadfence_system();
    out[2] = ser;
  }
}

// Step start: copies of the state into the step's references (T into Told,
// Ts, Tcyc, Tstar; Egrey into Es, Ecyc; E into Eold; F into Fold).
struct StepCopies {
  const double *T, *Egrey, *E, *F;
  double *Told, *Ts, *Tcyc, *Tstar, *Es, *Ecyc, *Eold, *Fold;
  long long n_cell, n_gi, n_ge;
  const int *ctl_in;  // control records in coherent pinned host memory (n_ctl words)
  int *ctl;
  long long n_ctl;
  // blocks from copy_blocks on: Phi of 256 groups per work item of tab_g;
  // from phi_end on: the opacity tables at T, one work item of tab_op each
  unsigned copy_blocks, phi_end;
  const SlabDev *sd;
  ProbDev pd;
  const Item *tab_g;
  const double *C;
  double *Phi;
  const Item *tab_op;
  double *kappa, *B, *dSpart;
  double *sgr;  // sigma_R table of spectral slabs (SPEC)
};

template <int RUN, bool SPEC>
__global__ __launch_bounds__(256) void k_step_start(StepCopies a) {
  if (blockIdx.x >= a.phi_end) {
    // the group averages of spectral slabs at the radiation temperature of
    // the state's grey energy density (read here, copied by other blocks)
    opacity_block<RUN, SPEC>(a.sd, a.pd, a.tab_op[blockIdx.x - a.phi_end], nullptr, PRED_ALL, 0, a.T, a.kappa, a.B,
                             a.dSpart, a.Egrey, a.sgr);
    return;
  }
  if (blockIdx.x >= a.copy_blocks) {
    phi_groups(a.sd, a.pd, a.tab_g[blockIdx.x - a.copy_blocks], a.C, a.Phi);
    return;
  }
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n_cell) {
    const double t = a.T[i], e = a.Egrey[i];
    a.Told[i] = t;
    a.Ts[i] = t;
    a.Tcyc[i] = t;
    a.Tstar[i] = t;
    a.Es[i] = e;
    a.Ecyc[i] = e;
  }
  if (i < a.n_gi) a.Eold[i] = a.E[i];
  if (i < a.n_ge) a.Fold[i] = a.F[i];
  if (i < a.n_ctl) a.ctl[i] = a.ctl_in[i];
}

// Elementwise copy over a pooled range.
__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src, double *__restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Fills a pooled cell array with a constant.
__global__ __launch_bounds__(256) void k_fill(double *__restrict__ dst, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

// Initial state from the B table at T0: I^0 = B in every corner/direction,
// E = sum w B / c, F = 0 (edges), synthetic sweep partials of I^0 for the
// moments kernel.  Thread = (slab, g, i).
template <typename TI>
__global__ __launch_bounds__(256) void k_init_state(const SlabDev *__restrict__ sd, ProbDev pd,
                                                    const Item *__restrict__ tab, const double *__restrict__ Bt,
                                                    TI *__restrict__ I, double *__restrict__ E,
                                                    double *__restrict__ F, double *__restrict__ Ebnd,
                                                    double *__restrict__ mom, double *__restrict__ bnd) {
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng, M = S.nmu;
  const int idx = it.idx + threadIdx.x;
  if (idx >= ng * nx) return;
  const int g = idx / nx, i = idx - g * nx;
  const double b = Bt[S.o_gi + idx];
  TI *ip = I + S.o_I + ((long long)g * M * nx + i) * 2;
  for (int m = 0; m < M; ++m) {
    ip[(long long)m * nx * 2] = (TI)b;
    ip[(long long)m * nx * 2 + 1] = (TI)b;
  }
  const double Ec = b * (S.wpos + S.wneg) / S.c;
  E[S.o_gi + idx] = Ec;
  F[S.o_ge + (long long)g * (nx + 1) + i] = 0.0;
  if (i == nx - 1) F[S.o_ge + (long long)g * (nx + 1) + nx] = 0.0;
  double *h0 = mom + 4 * S.o_gi + 2LL * idx;
  double *h1 = h0 + 2LL * ng * nx;
  h0[0] = b * S.wpos;
  h0[1] = b * S.wmu2pos;
  h1[0] = b * S.wneg;
  h1[1] = b * S.wmu2neg;
  if (i == 0) {
    Ebnd[2 * S.o_g + 2 * g] = Ec;
    double *b1 = bnd + 6 * S.o_g + 3 * ng + 3 * g;  // mu < 0 leaves at x = 0
    b1[0] = b * S.wneg;
    b1[1] = b * S.wmuneg;
    b1[2] = b * S.wmu2neg;
  }
  if (i == nx - 1) {
    Ebnd[2 * S.o_g + 2 * g + 1] = Ec;
    double *b0 = bnd + 6 * S.o_g + 3 * g;  // mu > 0 leaves at x = X
    b0[0] = b * S.wpos;
    b0[1] = b * S.wmupos;
    b0[2] = b * S.wmu2pos;
  }
}

// Grey energy density of the fine spectrum: Egrey_i = sum_g E_g,i.  Thread = cell.
__global__ __launch_bounds__(256) void k_group_sum(const SlabDev *__restrict__ sd, const Item *__restrict__ tab,
                                                   const double *__restrict__ E, double *__restrict__ out) {
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int i = it.idx + threadIdx.x;
  if (i >= S.nx) return;
  double acc = 0.0;
#pragma unroll 8
  for (int g = 0; g < S.ng; ++g) acc += E[S.o_gi + (long long)g * S.nx + i];  // loads in flight, group order
  out[S.o_cell + i] = acc;
}

// ---------------------------------------------------------------------------
// Learned closure: inputs per (g, i) and seeding of the cell QD factors.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_features(const SlabDev *__restrict__ sd, ProbDev pd,
                                                      const Item *__restrict__ tab, const double *__restrict__ T,
                                                      const double *__restrict__ Tprev,
                                                      const double *__restrict__ kappa, const double *__restrict__ fc,
                                                      MlpStats ms, float *__restrict__ X) {
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng;
  const int idx = it.idx + threadIdx.x;
  if (idx >= ng * nx) return;
  const int g = idx / nx, i = idx - g * nx;
  const double *Tc = T + S.o_cell;
  const double Ti = Tc[i];
  const double Tl = i > 0 ? Tc[i - 1] : (S.T_left > 0.0 ? S.T_left : Ti);
  const double Tr = i < nx - 1 ? Tc[i + 1] : Ti;
  const double f[TR_MLP_NFEAT] = {log(Ti),
                                  log(pd.nu_c[S.o_g + g]),
                                  log(kappa[S.o_gi + idx] * pd.dx[S.o_cell + i]),
                                  log(Tl),
                                  log(Tr),
                                  fc[S.o_gi + idx],
                                  Tprev ? log(Ti / Tprev[S.o_cell + i]) : 0.0};
  float *x = X + (S.o_gi + idx) * 8;
#pragma unroll
  for (int k = 0; k < TR_MLP_NFEAT; ++k) x[k] = (float)((f[k] - ms.mean[k]) / ms.std[k]);
  x[7] = 0.0f;
}

// Training targets per (g, i): Y = (s_g,i, r_g,i) with s = 1/2 + (f - f_prev) /
// (2 DF) clipped to [0.01, 0.99] (the sigmoid value that reproduces the
// factor change of the step) and r the log change of the within-block
// spectral shape E_g / E_p between two fine solutions (blocks of `blk`
// consecutive groups); 0 where a share is at or below TR_TINY; clipped to
// [-2, 2] (shares near underflow move by orders of magnitude).
__global__ __launch_bounds__(256) void k_closure_targets(const SlabDev *__restrict__ sd, const Item *__restrict__ tab,
                                                         const double *__restrict__ f, const double *__restrict__ fprev,
                                                         const double *__restrict__ Enew,
                                                         const double *__restrict__ Eprev, int blk,
                                                         float *__restrict__ Y) {
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng;
  const int idx = it.idx + threadIdx.x;
  if (idx >= ng * nx) return;
  const int g = idx / nx, i = idx - g * nx;
  const int g0 = (g / blk) * blk;
  double sn = 0.0, sp = 0.0;
  for (int q = g0; q < min(ng, g0 + blk); ++q) {
    sn += Enew[S.o_gi + (long long)q * nx + i];
    sp += Eprev[S.o_gi + (long long)q * nx + i];
  }
  const double en = Enew[S.o_gi + idx], ep = Eprev[S.o_gi + idx];
  double r = 0.0;
  if (sn > TR_TINY && sp > TR_TINY && en > TR_TINY && ep > TR_TINY) r = log((en / sn) / (ep / sp));
  r = fmin(2.0, fmax(-2.0, r));
  const double sv = 0.5 + (f[S.o_gi + idx] - fprev[S.o_gi + idx]) / (2.0 * TR_MLP_DF);
  Y[2 * (S.o_gi + idx)] = (float)fmin(0.99, fmax(0.01, sv));
  Y[2 * (S.o_gi + idx) + 1] = (float)r;
}

// Prolongation of level `lev` energy densities to the fine groups with the
// closure's shape correction: thread = (slab, coarse group p, cell i); the
// fine groups g of p get E_p w_g / sum w over the block, w = E_prev exp(r_g)
// (r_g = 0 without a prediction); an empty block is split evenly.
__global__ __launch_bounds__(256) void k_prolong(const SlabDev *__restrict__ sd, const Item *__restrict__ tab, int lev,
                                                 const double *__restrict__ Ec, const double *__restrict__ Eprev,
                                                 const float *__restrict__ r, double *__restrict__ Ef) {
  const Item it = tab[blockIdx.x];
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, np = S.lev_ng[lev];
  const int blk = S.ng / np;
  const int idx = it.idx + threadIdx.x;
  if (idx >= np * nx) return;
  const int p = idx / nx, i = idx - p * nx;
  const double Ep = Ec[S.o_lpi[lev] + idx];
  const long long o0 = S.o_gi + (long long)p * blk * nx + i;
  double W = 0.0;
  for (int q = 0; q < blk; ++q) {
    const long long o = o0 + (long long)q * nx;
    W += Eprev[o] * (r ? exp((double)r[2 * o + 1]) : 1.0);
  }
  for (int q = 0; q < blk; ++q) {
    const long long o = o0 + (long long)q * nx;
    const double w = Eprev[o] * (r ? exp((double)r[2 * o + 1]) : 1.0);
    Ef[o] = W > TR_TINY ? Ep * w / W : Ep / blk;
  }
}

// f <- f + DF (2 s_hat - 1) where the result lies in (0, 1) (counted), else
// the old factor stays (counted).
__global__ __launch_bounds__(256) void k_seed_f(const float *__restrict__ out, double *__restrict__ f, long long n,
                                                unsigned long long *__restrict__ counts) {
  __shared__ unsigned int s_ok, s_bad;
  if (threadIdx.x == 0) s_ok = s_bad = 0;
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double cand = f[i] + TR_MLP_DF * (2.0 * (double)out[2 * i] - 1.0);
    if (cand > 0.0 && cand < 1.0) {
      f[i] = cand;
      atomicAdd(&s_ok, 1u);
    } else {
      atomicAdd(&s_bad, 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&counts[0], (unsigned long long)s_ok);
    atomicAdd(&counts[1], (unsigned long long)s_bad);
  }
}

// ---------------------------------------------------------------------------
// A9 in one pass: the s = 0 seeding of the cell factors.  Per (group, cell)
// sample: the closure inputs (as k_mlp_features), the network (bfloat16 MFMA
// with float32 accumulation), the sigmoid of output 0 and the seeded factor
// f + DF (2 s - 1), written where it stays inside (0, 1) and counted (as
// k_seed_f).  The products are taken transposed, C[unit][sample] =
// W^T[unit][k] X[k][sample]: the weights are the A operand (staged in LDS
// once per block) and the activations the B operand, so a layer's
// accumulators feed the next layer directly from registers.  A lane of a
// 32 x 32 accumulator tile holds, for its sample column, the units
// 8 (j / 4) + 4 h + (j % 4) (j < 16, h = lane / 32); read as two 16-wide K
// chunks of 8 values per lane, chunk position 8 h + i then carries unit
// 8 (i / 4) + 4 h + (i % 4) of the chunk, so the next layer's weights are
// staged with K permuted the same way within every 16-wide block.
// Block = TR_CLS_WAVES wavefronts; it loops over the 256-sample items of the
// table (wavefront w takes samples 32 w .. 32 w + 31 of an item).
// ---------------------------------------------------------------------------
#define TR_CLS_WAVES 8
#define TR_CLS_LD 136  // LDS row stride (bf16) of the staged 128-wide weights

__device__ inline int cls_unit(int p) {  // K position within a layer -> unit
  const int q = p >> 4, k = p & 15, h = k >> 3, i = k & 7;
  return 16 * q + 8 * (i >> 2) + 4 * h + (i & 3);
}

__global__ __launch_bounds__(64 * TR_CLS_WAVES) void k_closure_seed(
    const SlabDev *__restrict__ sd, ProbDev pd, const Item *__restrict__ tab, int nitem,
    const double *__restrict__ T, const double *__restrict__ Tprev, const double *__restrict__ kappa,
    double *__restrict__ f, MlpStats ms, const float *__restrict__ params, unsigned long long *__restrict__ counts) {
  using namespace trmlp;
  __shared__ uint16_t W1t[NH * 24];
  __shared__ uint16_t W2p[NH * TR_CLS_LD];
  __shared__ uint16_t W3p[NH * TR_CLS_LD];
  __shared__ uint16_t W4p[32 * TR_CLS_LD];
  __shared__ float bias[3 * NH + NOUT];
  __shared__ unsigned int s_ok, s_bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) s_ok = s_bad = 0;
  for (int i = tid; i < NH * 24; i += nt) {
    const int nn = i / 24, k = i - nn * 24;
    W1t[i] = k < NINP ? to_bf16(params[OW1 + k * NH + nn]) : (uint16_t)0;
  }
  for (int i = tid; i < NH * NH; i += nt) {
    const int nn = i / NH, p = i - nn * NH, u = cls_unit(p);
    W2p[nn * TR_CLS_LD + p] = to_bf16(params[OW2 + u * NH + nn]);
    W3p[nn * TR_CLS_LD + p] = to_bf16(params[OW3 + u * NH + nn]);
  }
  for (int i = tid; i < 32 * NH; i += nt) {
    const int nn = i / NH, p = i - nn * NH;
    W4p[nn * TR_CLS_LD + p] = nn < NOUT ? to_bf16(params[OW4 + cls_unit(p) * NOUT + nn]) : (uint16_t)0;
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
  unsigned int ok = 0, bad = 0;
  for (int q = blockIdx.x; q < nitem; q += gridDim.x) {
    // compiler-only barrier: keeps the staged weights' LDS reads inside the
    // loop (hoisted, the 96 weight fragments of a pass would need 384 VGPRs)
    asm volatile("" ::: "memory");
    const Item it = tab[q];
    const SlabDev &S = sd[it.slab];
    const int nx = S.nx, ng = S.ng;
    const int idx = it.idx + 32 * wv + r;
    const bool valid = idx < ng * nx;
    // inputs of sample r (lanes of both halves compute them; half 1 feeds
    // the zero half of the 16-wide K step)
    bf16x8 x;
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 0;
    double fgi = 0.0;
    if (valid) {
      const int g = idx / nx, i = idx - g * nx;
      const double *Tc = T + S.o_cell;
      const double Ti = Tc[i];
      const double Tl = i > 0 ? Tc[i - 1] : (S.T_left > 0.0 ? S.T_left : Ti);
      const double Tr = i < nx - 1 ? Tc[i + 1] : Ti;
      fgi = f[S.o_gi + idx];
      const double in[TR_MLP_NFEAT] = {log(Ti),
                                       log(pd.nu_c[S.o_g + g]),
                                       log(kappa[S.o_gi + idx] * pd.dx[S.o_cell + i]),
                                       log(Tl),
                                       log(Tr),
                                       fgi,
                                       Tprev ? log(Ti / Tprev[S.o_cell + i]) : 0.0};
      if (h == 0) {
#pragma unroll
        for (int k = 0; k < TR_MLP_NFEAT; ++k) x[k] = (short)to_bf16((float)((in[k] - ms.mean[k]) / ms.std[k]));
      }
    }
    f32x16 acc[4];
    // layer 1: K = 8 features (the upper half of the 16-wide step is zero)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W1t + (t * 32 + r) * 24 + 8 * h);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x, acc[t], 0, 0, 0);
    }
    float o0 = 0.0f;
#pragma unroll
    for (int layer = 0; layer < 3; ++layer) {
      // bias + ReLU of the layer's 128 units -> eight 16-wide K chunks
      bf16x8 bq[8];
      const float *bl = bias + layer * NH;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          tr_u32x4 w;
#pragma unroll
          for (int i = 0; i < 8; i += 2) {
            const int j = 8 * c + i;
            const float v0 = fmaxf(acc[t][j] + bl[32 * t + 8 * (j >> 2) + 4 * h + (j & 3)], 0.0f);
            const float v1 = fmaxf(acc[t][j + 1] + bl[32 * t + 8 * ((j + 1) >> 2) + 4 * h + ((j + 1) & 3)], 0.0f);
            w[i >> 1] = pack_bf16x2(v0, v1);
          }
          bq[2 * t + c] = __builtin_bit_cast(bf16x8, w);
        }
      }
      if (layer < 2) {
        const uint16_t *Wp = layer == 0 ? W2p : W3p;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
#pragma unroll
          for (int kq = 0; kq < 8; ++kq) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(Wp + (t * 32 + r) * TR_CLS_LD + kq * 16 + 8 * h);
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bq[kq], acc[t], 0, 0, 0);
          }
        }
      } else {
        // output layer: rows 0 and 1 of one 32-row tile are the outputs
        f32x16 out;
#pragma unroll
        for (int j = 0; j < 16; ++j) out[j] = 0.0f;
#pragma unroll
        for (int kq = 0; kq < 8; ++kq) {
          const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W4p + r * TR_CLS_LD + kq * 16 + 8 * h);
          out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bq[kq], out, 0, 0, 0);
        }
        o0 = out[0] + bias[3 * NH];  // row 0 of column r on the lanes of half 0
      }
    }
    if (valid && h == 0) {
      const float sg = 1.0f / (1.0f + expf(-o0));
      const double cand = fgi + TR_MLP_DF * (2.0 * (double)sg - 1.0);
      if (cand > 0.0 && cand < 1.0) {
        f[S.o_gi + idx] = cand;
        ++ok;
      } else {
        ++bad;
      }
    }
  }
  atomicAdd(&s_ok, ok);
  atomicAdd(&s_bad, bad);
  __syncthreads();
  if (tid == 0) {
    atomicAdd(&counts[0], (unsigned long long)s_ok);
    atomicAdd(&counts[1], (unsigned long long)s_bad);
  }
}

// ---------------------------------------------------------------------------
// Alg. 1 (paper Sec. 3.1): one transport iteration's multigroup LOQD
// equations and multigroup MEB (Eq. eb-group) on the fine grid, solved
// together by Newton iterations in T with the QD factors fixed (the paper
// leaves the solver of this system open).  At the iterate T^k the group
// emission e_g = 2 sigma_B,g B_g is linearised with its derivative e'_g and
// the absorption c sigma_E,g E_g by the per-group secant derivative D_g of
// sigma_E,g between consecutive iterates (Eq. f-derivative-d applied to each
// group), so the cell MEB gives dT = alpha + beta phi with phi = sum_g c
// sigma_E,g E_g:
//   den = c_v/dt + S' - sum_g c D_g E_g^k,  alpha = (c_v (T^old - T^k)/dt - S) / den,
//   beta = 1 / den,
// and every group's balance gains the emission w_g dT, w_g = e'_g - c D_g E_g^k.
// Eliminating the groups leaves a dense system for phi per slab,
//   (I - sum_g c sigma_E,g A_g^{-1} diag(dx w_g beta)) phi = sum_g c sigma_E,g Y_g,
// (A_g the group's tridiagonal LO matrix, Y_g its solution with the emission
// e_g + w_g alpha), solved by Gaussian elimination with partial pivoting;
// the groups are then solved with e_g + w_g (alpha + beta phi) and T^{k+1} =
// T^k + alpha + beta phi.  At a fixed point dT = 0: the multigroup LOQD and MEB
// equations hold exactly at T.
// ---------------------------------------------------------------------------
__device__ inline bool a1_on(const A1Args &a, int slab) { return a.ctl[slab].active != 0; }

// Edge terms of the eliminated first moment (as in the LO solve): F_e = Ak -
// ca E_R + cb E_L.
__device__ inline void a1_edge(const LevelView &v, int e, double c, double inv_cdt, double &Ak, double &ca,
                               double &cb) {
  double ae, be, sr;
  lv_edge<true>(v, e, ae, be, sr);
  const double h = lv_h(v, e), A = h * inv_cdt;
  const double k = 1.0 / (A + sr * h);
  Ak = k * A * v.Fold[e];
  ca = c * k * ae;
  cb = c * k * be;
}

// Row j (0: E_{1/2}, 1..nx: cells, nx+1: E_{nx+1/2}) of group v's system;
// the cell rows take the emission em (per unit length).  L / R: terms of the
// edges j - 1 and j.
__device__ inline void a1_row(const LevelView &v, int j, double c, double dt, double em, double AkL, double caL,
                              double cbL, double AkR, double caR, double cbR, double &ra, double &rb, double &rc,
                              double &rd) {
  const int nx = v.nx;
  if (j == 0) {
    ra = 0.0;
    rb = cbR - c * v.C[0];
    rc = -caR;
    rd = v.Phi[0] - AkR;
  } else if (j <= nx) {
    const int i = j - 1;
    const double dxi = v.dx[i];
    ra = -cbL;
    rb = dxi / dt + c * v.kap[i] * dxi + cbR + caL;
    rc = -caR;
    rd = dxi * em + dxi / dt * v.Eold[i] - AkR + AkL;
  } else {
    ra = -cbL;
    rb = caL + c * v.C[1];
    rc = 0.0;
    rd = AkL - v.Phi[1];
  }
}

// a1_edge for an interior edge (0 < e < nx) and a1_row for a cell row (1 <=
// j <= nx), without the boundary cases, so that a loop over them has no
// branches between one row's loads and the next.
__device__ inline void a1_edge_in(const LevelView &v, int e, double c, double inv_cdt, double &Ak, double &ca,
                                  double &cb) {
  const double dm = v.dx[e - 1], de = v.dx[e];
  const double sr = (v.sgr[e - 1] * dm + v.sgr[e] * de) / (dm + de);
  const double h = 0.5 * (dm + de), A = h * inv_cdt;
  const double k = 1.0 / (A + sr * h);
  Ak = k * A * v.Fold[e];
  ca = c * k * v.f[e];
  cb = c * k * v.f[e - 1];
}

__device__ inline void a1_row_in(const LevelView &v, int j, double c, double dt, double em, double AkL, double caL,
                                 double cbL, double AkR, double caR, double cbR, double &ra, double &rb, double &rc,
                                 double &rd) {
  const int i = j - 1;
  const double dxi = v.dx[i];
  ra = -cbL;
  rb = dxi / dt + c * v.kap[i] * dxi + cbR + caL;
  rc = -caR;
  rd = dxi * em + dxi / dt * v.Eold[i] - AkR + AkL;
}

// Per cell: alpha, beta and the per-group emission couplings w_g.  The
// arrays are passed as non-aliasing pointers (cell i's column of each [g][i]
// array, stride nx) so that the group loops keep their loads in flight
// across the stores.
__device__ inline void a1_prep_cell(const SlabDev &S, const A1Args &a, long long oc, int nx,
                                    const double *__restrict__ kap, const double *__restrict__ Bv,
                                    const double *__restrict__ dem, const double *__restrict__ kprev,
                                    const double *__restrict__ Ek, double *__restrict__ w) {
  const double Tk = a.T[oc], c = S.c;
  const double dTs = Tk - a.Tprev[oc];
  const bool sec = !a.first && fabs(dTs) > 1e-8 * fabs(Tk);
  double Ssum = 0.0, Sp = 0.0, cDE = 0.0;
#pragma unroll 8
  for (int g = 0; g < S.ng; ++g) {
    const long long o = (long long)g * nx;
    Ssum += 2.0 * kap[o] * Bv[o];
    Sp += dem[o];
    if (sec) cDE += c * (kap[o] - kprev[o]) / dTs * Ek[o];
  }
  const bool use = sec && !(cDE > 0.5 * (S.cv / S.dt + Sp));
  const double den = S.cv / S.dt + Sp - (use ? cDE : 0.0);
  a.alpha[oc] = (S.cv * (a.Told[oc] - Tk) / S.dt - Ssum) / den;
  a.beta[oc] = 1.0 / den;
#pragma unroll 8
  for (int g = 0; g < S.ng; ++g) {
    const long long o = (long long)g * nx;
    w[o] = dem[o] - (use ? c * (kap[o] - kprev[o]) / dTs * Ek[o] : 0.0);
  }
}

__global__ __launch_bounds__(256) void k_a1_prep(const SlabDev *__restrict__ sd, ProbDev pd,
                                                 const Item *__restrict__ tab, A1Args a) {
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int i = it.idx + threadIdx.x;
  if (i >= S.nx) return;
  const long long o = S.o_gi + i;
  a1_prep_cell(S, a, S.o_cell + i, S.nx, a.in.kappa + o, a.in.B + o, a.dem + o, a.kprev + o, a.Ek + o, a.w + o);
}

// Per group: Thomas factors of its matrix (no pivoting: column diagonally
// dominant M-matrix).  Items = (slab, first of 256 groups).
__device__ inline void a1_factor_group(const SlabDev &S, const LevelView &v, int ng, double *__restrict__ ra_,
                                       double *__restrict__ cp_, double *__restrict__ dn_) {
  const int nx = S.nx;
  const double c = S.c, dt = S.dt, icdt = S.inv_cdt;
  double AkL = 0.0, caL = 0.0, cbL = 0.0, AkR, caR, cbR, cpp = 0.0;
  double ra, rb, rc, rd;
  auto put = [&](int j) {  // Thomas factor of row j
    const double dnj = rb - ra * cpp;
    cpp = rc / dnj;
    const long long o = (long long)j * ng;
    ra_[o] = ra;
    cp_[o] = cpp;
    dn_[o] = dnj;
    AkL = AkR;
    caL = caR;
    cbL = cbR;
  };
  a1_edge(v, 0, c, icdt, AkR, caR, cbR);
  a1_row(v, 0, c, dt, 0.0, AkL, caL, cbL, AkR, caR, cbR, ra, rb, rc, rd);
  put(0);
#pragma unroll 4
  for (int j = 1; j < nx; ++j) {
    a1_edge_in(v, j, c, icdt, AkR, caR, cbR);
    a1_row_in(v, j, c, dt, 0.0, AkL, caL, cbL, AkR, caR, cbR, ra, rb, rc, rd);
    put(j);
  }
  a1_edge(v, nx, c, icdt, AkR, caR, cbR);
  a1_row_in(v, nx, c, dt, 0.0, AkL, caL, cbL, AkR, caR, cbR, ra, rb, rc, rd);
  put(nx);
  a1_row(v, nx + 1, c, dt, 0.0, AkL, caL, cbL, AkR, caR, cbR, ra, rb, rc, rd);
  put(nx + 1);
}

__global__ __launch_bounds__(256) void k_a1_factor(const SlabDev *__restrict__ sd, ProbDev pd,
                                                   const Item *__restrict__ tab, A1Args a) {
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int g = it.idx + threadIdx.x;
  if (g >= S.ng) return;
  const LevelView v = make_view<true>(S, pd, 0, a.in, g);
  const long long o = S.o_gi + 2 * S.o_g + g;  // row j of group g at o + j ng
  a1_factor_group(S, v, S.ng, a.ra + o, a.cp + o, a.dn + o);
}

// Per group: the solve with the cell emission 2 kappa B + w (alpha + beta
// phi) (phi null: 0); writes E, the boundary E and, with phi, the fluxes.  A
// block per (slab, group) item (blockDim T >= (nx + 2) / K): thread t builds
// rows j = t K + k from its edges t K - 1 .. t K + K - 1 (rows past nx + 1 are
// identity rows) and solves by the partitioned Thomas + PCR of the LO solver,
// so that the rows' loads are coalesced over the threads; the fluxes take the
// neighbouring row through LDS.
template <int K>
__global__ __launch_bounds__(512) void k_a1_solve_blk(const SlabDev *__restrict__ sd, ProbDev pd,
                                                      const Item *__restrict__ tab, A1Args a, int with_phi) {
  extern __shared__ double lds[];  // tri_lds_doubles(blockDim) doubles (launch argument)
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int g = it.idx, nx = S.nx, t = threadIdx.x;
  const LevelView v = make_view<true>(S, pd, 0, a.in, g);
  const double c = S.c, dt = S.dt, icdt = S.inv_cdt;
  const long long og = S.o_gi + (long long)g * nx;
  double Ak[K + 1], ca[K + 1], cb[K + 1];  // edge t K + k - 1
#pragma unroll
  for (int k = 0; k <= K; ++k) {
    const int e = t * K + k - 1;
    Ak[k] = ca[k] = cb[k] = 0.0;
    if (e >= 0 && e <= nx) a1_edge(v, e, c, icdt, Ak[k], ca[k], cb[k]);
  }
  double ra[K], rb[K], rc[K], rd[K], x[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = t * K + k;
    ra[k] = 0.0;
    rb[k] = 1.0;
    rc[k] = 0.0;
    rd[k] = 0.0;
    if (j <= nx + 1) {
      double em = 0.0;
      if (j >= 1 && j <= nx) {
        const long long oc = S.o_cell + j - 1;
        const double dT = a.alpha[oc] + (with_phi ? a.beta[oc] * a.phi[oc] : 0.0);
        em = 2.0 * a.in.kappa[og + j - 1] * a.in.B[og + j - 1] + a.w[og + j - 1] * dT;
      }
      a1_row(v, j, c, dt, em, Ak[k], ca[k], cb[k], Ak[k + 1], ca[k + 1], cb[k + 1], ra[k], rb[k], rc[k], rd[k]);
    }
  }
  tri_solve_block<K>(ra, rb, rc, rd, x, lds, blockDim.x);
  double *E = a.E + og, *Eb = a.Ebnd + 2 * S.o_g + 2 * g;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = t * K + k;
    if (j == 0)
      Eb[0] = x[k];
    else if (j <= nx)
      E[j - 1] = x[k];
    else if (j == nx + 1)
      Eb[1] = x[k];
  }
  if (a.F && with_phi) {
    __syncthreads();  // the solver's LDS is free again
#pragma unroll
    for (int k = 0; k < K; ++k) lds[t * K + k] = x[k];
    __syncthreads();
    double *F = a.F + S.o_ge + (long long)g * (nx + 1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = t * K + k;  // F_e = Ak - ca u_R + cb u_L, u_L = row e, u_R = row e + 1
      if (e <= nx) F[e] = Ak[k + 1] - ca[k + 1] * lds[e + 1] + cb[k + 1] * lds[e];
    }
  }
}

// Per cell: phi's right-hand side sum_g c kappa_g E_g (fixed group order).
__global__ __launch_bounds__(256) void k_a1_rhs(const SlabDev *__restrict__ sd, const Item *__restrict__ tab,
                                                A1Args a) {
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int i = it.idx + threadIdx.x;
  if (i >= S.nx) return;
  double r = 0.0;
#pragma unroll 8
  for (int g = 0; g < S.ng; ++g) {  // unrolled: several groups' loads in flight, adds in group order
    const long long o = S.o_gi + (long long)g * S.nx + i;
    r += S.c * a.in.kappa[o] * a.E[o];
  }
  a.rhs[S.o_cell + i] = r;
}

// Per (group, column j): column j of A_g^{-1} restricted to the cells (unit
// source in cell j), times c kappa_g,i and dx_j w_g,j beta_j, into P[g][i][j].
// The column slots of P hold the forward-substitution values first.  Items
// = (slab, first of 256 (g, j) pairs).
__device__ inline void a1_cols_column(const SlabDev &S, int ng, int jc, const double *__restrict__ ra_,
                                      const double *__restrict__ cp_, const double *__restrict__ dn_,
                                      const double *__restrict__ kap, double u, double *__restrict__ Pg) {
  const int nx = S.nx;
  // forward: rows r < jc + 1 are zero, row jc + 1 has the unit source
  const int r = jc + 1;
  double d = 1.0 / dn_[(long long)r * ng];
  Pg[(long long)jc * nx] = d;
#pragma unroll 8
  for (int j = r + 1; j <= nx; ++j) {
    const long long o = (long long)j * ng;
    d = -ra_[o] * d / dn_[o];
    Pg[(long long)(j - 1) * nx] = d;
  }
  const long long on = (long long)(nx + 1) * ng;
  double z = -ra_[on] * d / dn_[on];  // row nx + 1 (boundary)
#pragma unroll 8
  for (int j = nx; j >= 1; --j) {
    const long long o = (long long)j * ng;
    const double dj = j >= r ? Pg[(long long)(j - 1) * nx] : 0.0;
    z = dj - cp_[o] * z;
    const int i = j - 1;
    Pg[(long long)i * nx] = S.c * kap[i] * z * u;
  }
}

__global__ __launch_bounds__(256) void k_a1_cols(const SlabDev *__restrict__ sd, ProbDev pd,
                                                 const Item *__restrict__ tab, A1Args a) {
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx, ng = S.ng;
  const int q = it.idx + threadIdx.x;
  if (q >= ng * nx) return;
  const int g = q / nx, jc = q - g * nx;
  const long long o = S.o_gi + 2 * S.o_g + g;  // row j of group g at o + j ng
  const long long oc = S.o_cell + jc, og = S.o_gi + (long long)g * nx;
  const double u = pd.dx[oc] * a.w[og + jc] * a.beta[oc];
  a1_cols_column(S, ng, jc, a.ra + o, a.cp + o, a.dn + o, a.in.kappa + og, u,
                 a.P + a.oP[it.slab] + (long long)g * nx * nx + jc);  // slot i at [i nx]
}

// Per (i, j): M_ij = delta_ij - sum_g P[g][i][j] (fixed group order).
__global__ __launch_bounds__(256) void k_a1_mred(const SlabDev *__restrict__ sd, const Item *__restrict__ tab,
                                                 A1Args a) {
  const Item it = tab[blockIdx.x];
  if (!a1_on(a, it.slab)) return;
  const SlabDev &S = sd[it.slab];
  const int nx = S.nx;
  const int q = it.idx + threadIdx.x;
  if (q >= nx * nx) return;
  const double *P = a.P + a.oP[it.slab] + q;
  double s = 0.0;
#pragma unroll 8
  for (int g = 0; g < S.ng; ++g) s += P[(long long)g * nx * nx];  // several loads in flight, group order
  const int i = q / nx, j = q - i * nx;
  a.M[a.oM[it.slab] + q] = (i == j ? 1.0 : 0.0) - s;
}

// One block per slab: Gaussian elimination with partial pivoting of M phi =
// rhs (row-major in global memory), then back substitution; phi written.
__global__ __launch_bounds__(256) void k_a1_dense(const SlabDev *__restrict__ sd, A1Args a) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ double sl[TR_A1_MAX_CELLS];  // multipliers of the current column
  __shared__ double sx;
  const int slab = blockIdx.x;
  if (!a1_on(a, slab)) return;
  const SlabDev &S = sd[slab];
  const int n = S.nx, t = threadIdx.x, nt = blockDim.x;
  double *M = a.M + a.oM[slab];
  double *b = a.rhs + S.o_cell;
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |M[i][k]|, i >= k (ties: the smallest i)
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < n; i += nt) {
      const double v = fabs(M[(long long)i * n + k]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int h = nt / 2; h > 0; h >>= 1) {
      if (t < h && (sv[t + h] > sv[t] || (sv[t + h] == sv[t] && si[t + h] < si[t]))) {
        sv[t] = sv[t + h];
        si[t] = si[t + h];
      }
      __syncthreads();
    }
    const int p = si[0];
    __syncthreads();
    if (p != k) {
      for (int j = k + t; j < n; j += nt) {
        const double x = M[(long long)k * n + j];
        M[(long long)k * n + j] = M[(long long)p * n + j];
        M[(long long)p * n + j] = x;
      }
      if (t == 0) {
        const double x = b[k];
        b[k] = b[p];
        b[p] = x;
      }
    }
    __syncthreads();
    // multipliers (thread per row), then the trailing update with a thread
    // per column walking the rows (each row access coalesced)
    const double piv = M[(long long)k * n + k];
    const double bk = b[k];
    for (int i = k + 1 + t; i < n; i += nt) {
      const double l = M[(long long)i * n + k] / piv;
      sl[i] = l;
      b[i] -= l * bk;
    }
    __syncthreads();
    for (int j = k + 1 + t; j < n; j += nt) {
      const double mkj = M[(long long)k * n + j];
      double *col = M + j;
      for (int i = k + 1; i < n; ++i) col[(long long)i * n] -= sl[i] * mkj;
    }
    __syncthreads();
  }
  // back substitution by columns: x_i, then every row above drops its term
  double *x = a.phi + S.o_cell;
  for (int i = n - 1; i >= 0; --i) {
    if (t == 0) {
      sx = b[i] / M[(long long)i * n + i];
      x[i] = sx;
    }
    __syncthreads();
    const double xi = sx;
    for (int r = t; r < i; r += nt) b[r] -= M[(long long)r * n + i] * xi;
    __syncthreads();
  }
}

// One block of 1024 threads per slab with the matrix in registers (nx <=
// TR_A1_REG_CELLS): thread t < R n (R = ceil(n / NS) row groups, at most
// 1024 / n) is column j = t mod n of row group q = t / n and holds rows i = q
// NS + s (s < NS) of that column.  Gaussian elimination with partial pivoting
// as in k_a1_dense (at step k the largest |M[i][k]| over the rows not yet
// chosen, ties to the smallest i; multipliers M[i][k] times the pivot's
// reciprocal), with the rows left in place: the pivot row of each step is
// recorded and a chosen row leaves the elimination.  Per step the owners of
// column k copy it to LDS, one wavefront finds the pivot, a thread per row
// forms its multiplier and right side while the pivot row's owners copy it
// to LDS, and every thread of a column j > k updates its rows.  Back
// substitution in reverse step order, a thread per row.
template <int NS>
__global__ __launch_bounds__(1024) void k_a1_dense_reg(const SlabDev *__restrict__ sd, A1Args a) {
  __shared__ double rowp[TR_A1_REG_CELLS];
  __shared__ double colk[TR_A1_REG_CELLS + NS], sl[TR_A1_REG_CELLS + NS];  // + NS: slots past row n - 1
  __shared__ double sb[TR_A1_REG_CELLS];
  __shared__ int prow[TR_A1_REG_CELLS], step_of[TR_A1_REG_CELLS];  // pivot row of a step, step of a row
  const int slab = blockIdx.x;
  if (!a1_on(a, slab)) return;
  const SlabDev &S = sd[slab];
  const int n = S.nx, t = threadIdx.x;
  const int R = (n + NS - 1) / NS;
  const int q = t / n, j = t - q * n;
  const bool own = q < R;  // threads R n .. 1023 hold nothing
  const int r0 = q * NS;   // first row of the group
  const int sn = own ? min(NS, n - r0) : 0;  // slots s < sn hold rows < n
  const double *M = a.M + a.oM[slab];
  double *b = a.rhs + S.o_cell;
  double m[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) m[s] = s < sn ? M[(long long)(r0 + s) * n + j] : 0.0;
  if (t < n) {
    sb[t] = b[t];
    step_of[t] = n;  // not chosen yet
  }
  if (t < TR_A1_REG_CELLS + NS) sl[t] = 0.0;  // rows past n - 1 keep multiplier 0
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (own && j == k) {
#pragma unroll
      for (int s = 0; s < NS; ++s) colk[r0 + s] = m[s];
    }
    __syncthreads();
    if (t < 64) {  // pivot: rows in ascending order per lane, ties to the smaller row
      double best = -1.0;
      int bi = n;
      for (int i = t; i < n; i += 64) {
        const double v = fabs(colk[i]);
        if (step_of[i] == n && v > best) {
          best = v;
          bi = i;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (t == 0) {
        prow[k] = bi;
        step_of[bi] = k;
      }
    }
    __syncthreads();
    const int p = prow[k];
    if (t < n && t != p) {  // multiplier of row t (0 once chosen) and its right side
      const double l = step_of[t] == n ? colk[t] * (1.0 / colk[p]) : 0.0;
      sl[t] = l;
      sb[t] -= l * sb[p];
    }
    if (t == p) sl[t] = 0.0;
    const int dp = p - r0;
    if (own && dp >= 0 && dp < NS) {  // the pivot row
      double vp = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) vp = s == dp ? m[s] : vp;
      rowp[j] = vp;
    }
    __syncthreads();
    if (own && j > k) {
      const double mpj = rowp[j];
#pragma unroll
      for (int s = 0; s < NS; ++s) m[s] -= sl[r0 + s] * mpj;
    }
    __syncthreads();
  }
  // back substitution in reverse step order: x_k from the pivot row of step
  // k, then the rows chosen at earlier steps drop their term
  double *x = a.phi + S.o_cell;
  for (int k = n - 1; k >= 0; --k) {
    if (own && j == k) {
#pragma unroll
      for (int s = 0; s < NS; ++s) colk[r0 + s] = m[s];
    }
    __syncthreads();
    const int p = prow[k];
    const double xk = sb[p] / colk[p];
    if (t == 0) x[k] = xk;
    if (t < n && step_of[t] < k) sb[t] -= colk[t] * xk;
    __syncthreads();
  }
}

// One block per slab (blockDim >= nx): T^{k+1} = T^k + alpha + beta phi
// (floored at T^k / 2), the previous iterate's T kept, and max|dT| / max|T|.
__global__ __launch_bounds__(512) void k_a1_update(const SlabDev *__restrict__ sd, A1Args a, double *Tprev) {
  __shared__ double r0[512], r1[512];
  const int slab = blockIdx.x;
  if (!a1_on(a, slab)) return;
  const SlabDev &S = sd[slab];
  const int i = threadIdx.x;
  double dT = 0.0, Tn = 0.0;
  if (i < S.nx) {
    const long long oc = S.o_cell + i;
    const double Tk = a.T[oc];
    Tn = Tk + a.alpha[oc] + a.beta[oc] * a.phi[oc];
    if (Tn < 0.5 * Tk) Tn = 0.5 * Tk;
    dT = fabs(Tn - Tk);
    Tprev[oc] = Tk;
    a.Tout[oc] = Tn;
  }
  r0[i] = dT;
  r1[i] = fabs(Tn);
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (i < h) {
      r0[i] = fmax(r0[i], r0[i + h]);
      r1[i] = fmax(r1[i], r1[i + h]);
    }
    __syncthreads();
  }
  if (i == 0) a.err[slab] = r1[0] > 0.0 ? r0[0] / r1[0] : 0.0;
}

// One block per slab: max|T - Ts|, max|T|, max|Es - Esp|, max|Es| (outer
// test of Alg. 1) into out[4 slab ..]; Esum = sum_g E_g per cell.
__global__ __launch_bounds__(512) void k_a1_outer(const SlabDev *__restrict__ sd, const Ctl *ctl, const double *T,
                                                  const double *Ts, const double *E, double *Esum,
                                                  const double *Esp, double *out) {
  __shared__ double r[4][512];
  const int slab = blockIdx.x;
  if (ctl[slab].active == 0) return;
  const SlabDev &S = sd[slab];
  const int i = threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < S.nx) {
    const long long oc = S.o_cell + i;
    double e = 0.0;
#pragma unroll 8
    for (int g = 0; g < S.ng; ++g) e += E[S.o_gi + (long long)g * S.nx + i];  // loads in flight, group order
    Esum[oc] = e;
    v[0] = fabs(T[oc] - Ts[oc]);
    v[1] = fabs(T[oc]);
    v[2] = fabs(e - Esp[oc]);
    v[3] = fabs(e);
  }
  for (int k = 0; k < 4; ++k) r[k][i] = v[k];
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (i < h)
      for (int k = 0; k < 4; ++k) r[k][i] = fmax(r[k][i], r[k][i + h]);
    __syncthreads();
  }
  if (i == 0)
    for (int k = 0; k < 4; ++k) out[4 * slab + k] = r[k][0];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline dim3 blocks(int n) { return dim3((unsigned)n); }

void launch_opacity(const LaunchEnv &env, const Table &tab, int run, const Ctl *ctl, int pmode, int lcyc,
                    const double *T, double *kappa, double *B, double *dSpart, bool spec, const double *Eg,
                    double *sgr, double *dem) {
  if (tab.n == 0) return;
#define TR_OP(R, SP)                                                                                                 \
  hipLaunchKernelGGL((k_opacity<R, SP>), blocks(tab.n), dim3(256), 0, env.stream, env.sd, env.pd, tab.d, ctl, pmode, \
                     lcyc, T, kappa, B, dSpart, Eg, sgr, dem)
  if (spec) {
    if (run == 1) TR_OP(1, true); else TR_OP(4, true);
  } else {
    if (run == 1) TR_OP(1, false); else TR_OP(4, false);
  }
#undef TR_OP
}

void launch_dS_sum(const LaunchEnv &env, const Table &tab, const Ctl *ctl, int pmode, int lcyc, const double *dSpart,
                   double *dS) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_dS_sum, blocks(tab.n), dim3(256), 0, env.stream, env.sd, tab.d, ctl, pmode, lcyc, dSpart, dS);
}

void launch_sweep(const LaunchEnv &env, const Table &tab, int K, int split, bool f32, bool nt_hint, const Ctl *ctl,
                  int pmode, int lcyc, const double *kappa, const double *B, const void *Ip, void *Io, double *mom,
                  double *bnd, hipEvent_t ev0, hipEvent_t ev1) {
  if (tab.n == 0) return;
  const int waves = 2 * tab.n;
  const int nb = split == 1 ? (waves + 3) / 4 : waves;
  const int nt = split == 1 ? 256 : 64 * split;
  const size_t lds = (size_t)sweep_lds_doubles(K, split) * sizeof(double);
#define TR_SWEEP_KN(KK, TT, NN)                                                                                      \
  do {                                                                                                                 \
    if (ev0)                                                                                                           \
      hipExtLaunchKernelGGL((k_sweep<KK, TT, NN>), blocks(nb), dim3(nt), lds, env.stream, ev0, ev1, 0, env.sd,       \
                            env.pd, tab.d, tab.n, split, ctl, pmode, lcyc, kappa, B, static_cast<const TT *>(Ip),   \
                            static_cast<TT *>(Io), mom, bnd);                                                        \
    else                                                                                                               \
      hipLaunchKernelGGL((k_sweep<KK, TT, NN>), blocks(nb), dim3(nt), lds, env.stream, env.sd, env.pd, tab.d, tab.n, \
                         split, ctl, pmode, lcyc, kappa, B, static_cast<const TT *>(Ip), static_cast<TT *>(Io), mom,    \
                         bnd);                                                                                         \
  } while (0)
#define TR_SWEEP_K(KK, TT)                \
  do {                                    \
    if (stream_hint)                      \
      TR_SWEEP_KN(KK, TT, true);          \
    else                                  \
      TR_SWEEP_KN(KK, TT, false);         \
  } while (0)
  const bool stream_hint = nt_hint;
  if (f32) {
    switch (K) {
      case 1: TR_SWEEP_K(1, float); break;
      case 2: TR_SWEEP_K(2, float); break;
      case 8: TR_SWEEP_K(8, float); break;
      default: TR_SWEEP_K(4, float); break;
    }
  } else {
    switch (K) {
      case 1: TR_SWEEP_K(1, double); break;
      case 2: TR_SWEEP_K(2, double); break;
      case 8: TR_SWEEP_K(8, double); break;
      default: TR_SWEEP_K(4, double); break;
    }
  }
#undef TR_SWEEP_KN
#undef TR_SWEEP_K
}

void launch_moments(const LaunchEnv &env, const Table &tab, const Ctl *ctl, int pmode, int lcyc, const double *mom,
                    const double *bnd, double *f, double *fbnd, double *C, double *Phi) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_moments, blocks(tab.n), dim3(256), 0, env.stream, env.sd, env.pd, tab.d, ctl, pmode, lcyc, mom,
                     bnd, f, fbnd, C, Phi);
}


void launch_lo(const LaunchEnv &env, const Table &tab, int threads, const Ctl *ctl, int pmode, int lcyc, int level,
               const LoIn &in, const LoSol &sol) {
  if (tab.n == 0) return;
  if (level == 0 && in.mom)
    hipLaunchKernelGGL((k_lo<TR_LO_K, true, true>), blocks(tab.n), dim3(threads), tri_lds_doubles(threads) * sizeof(double), env.stream, env.sd, env.pd,
                       tab.d, ctl, pmode, lcyc, level, in, sol);
  else if (level == 0)
    hipLaunchKernelGGL((k_lo<TR_LO_K, true, false>), blocks(tab.n), dim3(threads), tri_lds_doubles(threads) * sizeof(double), env.stream, env.sd, env.pd, tab.d, ctl,
                       pmode, lcyc, level, in, sol);
  else
    hipLaunchKernelGGL((k_lo<TR_LO_K, false, false>), blocks(tab.n), dim3(threads), tri_lds_doubles(threads) * sizeof(double), env.stream, env.sd, env.pd, tab.d, ctl,
                       pmode, lcyc, level, in, sol);
}

template <bool FINE, bool OLD, int MODE>
void launch_restrict_t(const LaunchEnv &env, const RestrictTables &rt, const Ctl *ctl, int pmode, int lcyc, int from,
                       int to, const LoIn &in, const LoSol &sol, const LoOut &out, double *red, const double *T,
                       double *dsop) {
  if (rt.single.n)
    hipLaunchKernelGGL((k_restrict<FINE, OLD, MODE>), blocks(rt.single.n), dim3(256), 0, env.stream, env.sd, env.pd,
                       rt.single.d, ctl, pmode, lcyc, from, to, in, sol, out, T, dsop);
  if (rt.part.n)
    hipLaunchKernelGGL((k_restrict_part<FINE, OLD, MODE>), blocks(rt.part.n), dim3(256), 0, env.stream, env.sd,
                       env.pd, rt.part.d, ctl, pmode, lcyc, from, to, in, sol, red, T, dsop);
  if (rt.fin.n)
    hipLaunchKernelGGL((k_restrict_final<OLD, MODE>), blocks(rt.fin.n), dim3(256), 0, env.stream, env.sd, env.pd,
                       rt.fin.d, ctl, pmode, lcyc, from, to, out, red);
}

void launch_restrict(const LaunchEnv &env, const RestrictTables &rt, const Ctl *ctl, int pmode, int lcyc, int from,
                     int to, const LoIn &in, const LoSol &sol, const LoOut &out, double *red, bool old, int mode,
                     const double *T, double *dsop) {
  const bool fine = from == 0;
#define TR_RL(F, O, M) launch_restrict_t<F, O, M>(env, rt, ctl, pmode, lcyc, from, to, in, sol, out, red, T, dsop)
  if (fine) {
    if (mode == RM_OPAC) {
      if (old) TR_RL(true, true, RM_OPAC); else TR_RL(true, false, RM_OPAC);
    } else {
      if (old) TR_RL(true, true, RM_PLAIN); else TR_RL(true, false, RM_PLAIN);
    }
  } else {
    if (mode == RM_DSF) {
      if (old) TR_RL(false, true, RM_DSF); else TR_RL(false, false, RM_DSF);
    } else {
      if (old) TR_RL(false, true, RM_PLAIN); else TR_RL(false, false, RM_PLAIN);
    }
  }
#undef TR_RL
}

void launch_grey(const LaunchEnv &env, const Table &tab, int threads, Ctl *ctl, int pmode, int lcyc,
                 const GreyArgs &ga) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_grey<TR_GREY_K>, blocks(tab.n), dim3(threads), tri_lds_doubles(threads) * sizeof(double), env.stream, env.sd, env.pd, tab.d, ctl, pmode,
                     lcyc, ga);
}

void launch_outer_end(const LaunchEnv &env, Ctl *ctl, int nslab, int max_outer, int *out, Ctl *hout, int *serial) {
  hipLaunchKernelGGL(k_outer_end, dim3(1), dim3(256), 0, env.stream, ctl, nslab, max_outer, out, hout, serial);
}

void launch_step_start(const LaunchEnv &env, const double *T, const double *Egrey, const double *E, const double *F,
                       long long n_cell, long long n_gi, long long n_ge, double *Told, double *Ts, double *Tcyc,
                       double *Tstar, double *Es, double *Ecyc, double *Eold, double *Fold, const Ctl *ctl_in,
                       Ctl *ctl, int nslab, const Table &tab_g, const double *C, double *Phi, const Table &tab_op,
                       int run, double *kappa, double *B, double *dSpart, bool spec, double *sgr) {
  const long long n_ctl = (long long)nslab * (long long)(sizeof(Ctl) / sizeof(int));
  const long long n = std::max(std::max(n_cell, n_ctl), std::max(n_gi, n_ge));
  const unsigned copy_blocks = (unsigned)((n + 255) / 256), phi_end = copy_blocks + (unsigned)tab_g.n;
  const StepCopies a{T,       Egrey,  E,       F,      Told,        Ts,
                     Tcyc,    Tstar,  Es,      Ecyc,   Eold,        Fold,
                     n_cell,  n_gi,   n_ge,    reinterpret_cast<const int *>(ctl_in), reinterpret_cast<int *>(ctl), n_ctl,
                     copy_blocks, phi_end, env.sd, env.pd, tab_g.d, C, Phi, tab_op.d, kappa, B, dSpart, sgr};
  const unsigned nb = phi_end + (unsigned)tab_op.n;
  if (nb == 0) return;
  if (spec) {
    if (run == 1)
      hipLaunchKernelGGL((k_step_start<1, true>), dim3(nb), dim3(256), 0, env.stream, a);
    else
      hipLaunchKernelGGL((k_step_start<4, true>), dim3(nb), dim3(256), 0, env.stream, a);
  } else {
    if (run == 1)
      hipLaunchKernelGGL((k_step_start<1, false>), dim3(nb), dim3(256), 0, env.stream, a);
    else
      hipLaunchKernelGGL((k_step_start<4, false>), dim3(nb), dim3(256), 0, env.stream, a);
  }
}

void launch_copy(const LaunchEnv &env, const double *src, double *dst, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, env.stream, src, dst, n);
}

void launch_fill(const LaunchEnv &env, double *dst, double v, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, env.stream, dst, v, n);
}

void launch_init_state(const LaunchEnv &env, const Table &tab, bool f32, const double *Bt, void *I, double *E,
                       double *F, double *Ebnd, double *mom, double *bnd) {
  if (tab.n == 0) return;
  if (f32)
    hipLaunchKernelGGL(k_init_state<float>, blocks(tab.n), dim3(256), 0, env.stream, env.sd, env.pd, tab.d, Bt,
                       static_cast<float *>(I), E, F, Ebnd, mom, bnd);
  else
    hipLaunchKernelGGL(k_init_state<double>, blocks(tab.n), dim3(256), 0, env.stream, env.sd, env.pd, tab.d, Bt,
                       static_cast<double *>(I), E, F, Ebnd, mom, bnd);
}

void launch_group_sum(const LaunchEnv &env, const Table &tab, const double *E, double *out) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_group_sum, blocks(tab.n), dim3(256), 0, env.stream, env.sd, tab.d, E, out);
}

void launch_mlp_features(const LaunchEnv &env, const Table &tab, const double *T, const double *Tprev,
                         const double *kappa, const double *f, const MlpStats &ms, float *X) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_mlp_features, blocks(tab.n), dim3(256), 0, env.stream, env.sd, env.pd, tab.d, T, Tprev, kappa,
                     f, ms, X);
}

void launch_closure_targets(const LaunchEnv &env, const Table &tab, const double *f, const double *fprev,
                            const double *Enew, const double *Eprev, int blk, float *Y) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_closure_targets, blocks(tab.n), dim3(256), 0, env.stream, env.sd, tab.d, f, fprev, Enew, Eprev,
                     blk, Y);
}

void launch_prolong(const LaunchEnv &env, const Table &tab, int lev, const double *Ec, const double *Eprev,
                    const float *r, double *Ef) {
  if (tab.n == 0) return;
  hipLaunchKernelGGL(k_prolong, blocks(tab.n), dim3(256), 0, env.stream, env.sd, tab.d, lev, Ec, Eprev, r, Ef);
}

void launch_closure_seed(const LaunchEnv &env, const Table &tab, const double *T, const double *Tprev,
                         const double *kappa, double *f, const MlpStats &ms, const float *params,
                         unsigned long long *counts) {
  if (tab.n == 0) return;
  // at most one block per CU: every block stages the weights once
  const unsigned nb = (unsigned)std::min(tab.n, 256);
  hipLaunchKernelGGL(k_closure_seed, dim3(nb), dim3(64 * TR_CLS_WAVES), 0, env.stream, env.sd, env.pd, tab.d, tab.n,
                     T, Tprev, kappa, f, ms, params, counts);
}

void launch_seed_f(const LaunchEnv &env, const float *out, double *f, long long n, unsigned long long *counts) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_seed_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, env.stream, out, f, n, counts);
}

// Alg. 1 launchers (items: t_cell = (slab, first of 256 cells), t_g = (slab,
// first of 256 groups), t_gi = (slab, first of 256 (g, i) pairs), t_mm =
// (slab, first of 256 (i, j) pairs)).
void launch_a1_prep(const LaunchEnv &env, const Table &t_cell, const A1Args &a) {
  if (t_cell.n) hipLaunchKernelGGL(k_a1_prep, blocks(t_cell.n), dim3(256), 0, env.stream, env.sd, env.pd, t_cell.d, a);
}
void launch_a1_factor(const LaunchEnv &env, const Table &t_g, const A1Args &a) {
  if (t_g.n) hipLaunchKernelGGL(k_a1_factor, blocks(t_g.n), dim3(256), 0, env.stream, env.sd, env.pd, t_g.d, a);
}
void launch_a1_solve_blk(const LaunchEnv &env, const Table &t_sg, int threads, const A1Args &a, bool with_phi) {
  if (t_sg.n == 0) return;
  hipLaunchKernelGGL(k_a1_solve_blk<TR_LO_K>, blocks(t_sg.n), dim3(threads), tri_lds_doubles(threads) * sizeof(double), env.stream, env.sd, env.pd,
                     t_sg.d, a, with_phi ? 1 : 0);
}
void launch_a1_rhs(const LaunchEnv &env, const Table &t_cell, const A1Args &a) {
  if (t_cell.n) hipLaunchKernelGGL(k_a1_rhs, blocks(t_cell.n), dim3(256), 0, env.stream, env.sd, t_cell.d, a);
}
void launch_a1_cols(const LaunchEnv &env, const Table &t_gi, const A1Args &a) {
  if (t_gi.n) hipLaunchKernelGGL(k_a1_cols, blocks(t_gi.n), dim3(256), 0, env.stream, env.sd, env.pd, t_gi.d, a);
}
void launch_a1_mred(const LaunchEnv &env, const Table &t_mm, const A1Args &a) {
  if (t_mm.n) hipLaunchKernelGGL(k_a1_mred, blocks(t_mm.n), dim3(256), 0, env.stream, env.sd, t_mm.d, a);
}
void launch_a1_dense(const LaunchEnv &env, int nslab, int max_nx, const A1Args &a) {
  // registers for every slab of at most TR_A1_REG_CELLS cells (slots per
  // thread from the largest: ceil(n / (1024 / n)) rows), else the
  // global-memory elimination
  const int ns = max_nx > 0 ? (max_nx + 1024 / max_nx - 1) / (1024 / max_nx) : 1;
  if (max_nx > TR_A1_REG_CELLS)
    hipLaunchKernelGGL(k_a1_dense, dim3((unsigned)nslab), dim3(256), 0, env.stream, env.sd, a);
  else if (ns <= 8)
    hipLaunchKernelGGL(k_a1_dense_reg<8>, dim3((unsigned)nslab), dim3(1024), 0, env.stream, env.sd, a);
  else if (ns <= 16)
    hipLaunchKernelGGL(k_a1_dense_reg<16>, dim3((unsigned)nslab), dim3(1024), 0, env.stream, env.sd, a);
  else if (ns <= 24)
    hipLaunchKernelGGL(k_a1_dense_reg<24>, dim3((unsigned)nslab), dim3(1024), 0, env.stream, env.sd, a);
  else if (ns <= 32)
    hipLaunchKernelGGL(k_a1_dense_reg<32>, dim3((unsigned)nslab), dim3(1024), 0, env.stream, env.sd, a);
  else
    hipLaunchKernelGGL(k_a1_dense_reg<TR_A1_REG_SLOTS>, dim3((unsigned)nslab), dim3(1024), 0, env.stream,
                       env.sd, a);
}
void launch_a1_update(const LaunchEnv &env, int nslab, const A1Args &a, double *Tprev) {
  hipLaunchKernelGGL(k_a1_update, dim3((unsigned)nslab), dim3(512), 0, env.stream, env.sd, a, Tprev);
}
void launch_a1_outer(const LaunchEnv &env, int nslab, const Ctl *ctl, const double *T, const double *Ts,
                     const double *E, double *Esum, const double *Esp, double *out) {
  hipLaunchKernelGGL(k_a1_outer, dim3((unsigned)nslab), dim3(512), 0, env.stream, env.sd, ctl, T, Ts, E, Esum, Esp,
                     out);
}
