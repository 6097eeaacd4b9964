/*
 * tr.h - C ABI of the MI355X (gfx950) library for the multilevel quasidiffusion
 * (MLQD) method with multigrid in photon frequency for time-dependent
 * multigroup thermal radiative transfer in 1-D slabs (Anistratov, arXiv
 * 2011.05427).
 *
 * Conventions (every entry point):
 *  - Arrays named in a call are DEVICE pointers owned by the caller unless a
 *    comment says "host".  The library never frees caller memory.
 *  - Work is enqueued asynchronously on the given stream (0 = default stream);
 *    the caller synchronises.  tr_step and tr_run wait on the host until the
 *    device has published the number of slabs still iterating: the
 *    iteration's end kernel writes it, with an iteration serial number, into
 *    coherent pinned host memory and the host spins on that serial (no
 *    stream synchronisation); their outputs (T, E, F, I, factors) are ready
 *    only in the order of the given stream: work queued there afterwards
 *    sees them, a reader on another stream or on the host synchronises the
 *    stream first.  tr_alg1_step synchronises the stream.
 *  - Every call returns TR_OK (0) or a negative TR_E* code; tr_error_string()
 *    gives a message.  Nothing throws across the ABI.
 *  - One context serves one stream at a time; calls on one context are not
 *    thread-safe.
 *  - Floating point is IEEE binary64 throughout, except the corner intensities
 *    of a context created with TR_PREC_F32_STORAGE (binary32 storage) and the
 *    closure network calls (float32 parameters, bfloat16 products).
 *
 * Batched layout ("pooled" arrays).  The library works in the canonical
 * layout below (the one the CPU oracle and the tests use): intensities
 * [g][m][i][corner] keep a corner pair in one 16-byte load and every
 * (group, direction) row contiguous for the sweep's coalesced passes, so no
 * pack/unpack between an internal and a user layout exists.  A context holds
 * n_slab independent slab problems.  Every per-slab array is stored slab after slab in creation order;
 * tr_layout() returns, per slab, the element offset of its part in each kind
 * of pooled array.  Within one slab (nx cells, ng groups, nmu directions, cell
 * i, edge e = 0..nx at x_edges[e], group g, direction m, corner k = 0 (left,
 * x_{i-1/2}) / 1 (right, x_{i+1/2})):
 *     cell     [nx]                T, grey E
 *     I        [ng][nmu][nx][2]    corner intensities      (kind TR_K_I)
 *     gi       [ng][nx]            kappa, B, E_g, f        (kind TR_K_GI)
 *     ge       [ng][nx+1]          F_g at edges            (kind TR_K_GE)
 *     g2       [ng][2]             boundary values (x=0, x=X)
 *     level-l  [n_l][nx], [n_l][nx+1], [n_l][2] for frequency level l
 *              (level 0 is the fine grid, the last level is grey, n = 1).
 */
#ifndef TR_H
#define TR_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TR_OK = 0,
  TR_EINVAL = -1,  /* bad argument or shape */
  TR_ENOMEM = -2,  /* device allocation failed */
  TR_EHIP = -3,    /* a HIP runtime call failed */
  TR_ENOCONV = -4, /* a slab exceeded max_outer transport iterations */
  TR_ENAN = -5     /* a non-finite temperature or energy appeared */
};

enum { TR_CYCLE_V = 0, TR_CYCLE_W = 1, TR_CYCLE_F = 2 };
enum { TR_MAX_LEVELS = 8 };

/* Array kinds for tr_layout(). */
enum {
  TR_K_CELL = 0, /* [nx]               */
  TR_K_EDGE = 1, /* [nx+1]             */
  TR_K_I = 2,    /* [ng][nmu][nx][2]   */
  TR_K_GI = 3,   /* [ng][nx]           */
  TR_K_GE = 4,   /* [ng][nx+1]         */
  TR_K_G2 = 5,   /* [ng][2]            */
  TR_K_G = 6,    /* [ng]               */
  TR_K_LEV_PI = 8,  /* + level: [n_l][nx]   */
  TR_K_LEV_PE = 16, /* + level: [n_l][nx+1] */
  TR_K_LEV_P2 = 24  /* + level: [n_l][2]    */
};

/*
 * One slab problem (all pointers HOST, copied at tr_create).  Paper Sec. 2
 * (Eqs. rt-nu, eb-nu, rt-nu-bc and the multigroup Eqs. rt, rt-bc, rt-ic),
 * eps = cv T, and the spectral opacity sigma(nu, T) = C_cell / nu^3 (1 -
 * exp(-nu / T)) of Sec. 6, entering the group equations either
 *  - TR_OPAC_POINT: as the point law kappa_g(T) = C_cell / nu_c^3 (1 -
 *    exp(-nu_c / T)) at the group centre nu_c, sigma_E = sigma_B = sigma_R =
 *    kappa_g; or
 *  - TR_OPAC_SPECTRAL: as the paper's group averages (Sec. 2 after Eq. rt,
 *    Sec. 3.1 with Eq. mloqd-2): sigma_B,g(T) Planck-weighted at T (only the
 *    emission sigma_B,g B_g enters; closed form), sigma_E,g(T, T_r)
 *    Planck-weighted at the radiation temperature T_r = (E / a_R)^(1/4) of the
 *    cell's latest grey energy density E, sigma_R,g(T, T_r) the dB/dT-weighted
 *    harmonic mean at T_r (Gauss-Legendre panels in nu / T_r).  nu_center is
 *    not used.
 */
enum { TR_OPAC_POINT = 0, TR_OPAC_SPECTRAL = 1 };
typedef struct tr_problem {
  int nx;                  /* cells, >= 2 */
  int ng;                  /* fine groups, >= 1 */
  int nmu;                 /* directions, even, mu ascending, symmetric */
  const double *x_edges;   /* [nx+1] increasing */
  const double *nu_edges;  /* [ng+1] group edges for the Planck integrals;
                              nu_edges[0] may be 0 and nu_edges[ng] +inf */
  const double *nu_center; /* [ng] opacity evaluation point of each group */
  const double *mu;        /* [nmu] direction cosines, ascending */
  const double *w;         /* [nmu] quadrature weights (sum 2) */
  const double *C_cell;    /* [nx] opacity constant per cell */
  double T_left, T_right;  /* isotropic incoming Planck radiation at this
                              temperature at x=0 / x=X; <= 0 means vacuum */
  double cv;               /* material heat capacity, eps = cv T */
  double dt;               /* time step */
  double c, aR;            /* speed of light, radiation constant */
  int n_levels;            /* frequency grids incl. fine and grey, 2..8 */
  const int *level_ng;     /* [n_levels] groups per grid: ng, ..., 1; each
                              divides the previous (uniform coarsening) */
  int opacity;             /* TR_OPAC_POINT or TR_OPAC_SPECTRAL */
} tr_problem;

/* Iteration settings shared by all slabs of a context (paper Alg. 3). */
typedef struct tr_solver_cfg {
  int cycle;        /* TR_CYCLE_V / W / F: schedule of grids visited after each
                       grey solve (V none, W the middle grid, F every
                       intermediate grid from coarse to fine) */
  int lmax;         /* maximum cycles per transport iteration (>= 1) */
  double eps;       /* outer tolerance on T and grey E (relative, inf-norm) */
  double eps_inner; /* inner tolerance */
  int max_outer;    /* transport iterations before TR_ENOCONV */
  int secant;       /* 1: diagonal secant Frechet derivative of the grey
                       sigma_E (Eq. f-derivative-d); 0: D = 0 */
  int timing;       /* 1: tr_step brackets its kernel groups with HIP events
                       and accumulates their durations in tr_stats.t_ms */
  int precision;    /* TR_PREC_F64: corner intensities stored in binary64;
                       TR_PREC_F32_STORAGE: stored in binary32 (I arrays are
                       float), every sweep operation and all moments still in
                       binary64 registers */
} tr_solver_cfg;

enum { TR_PREC_F64 = 0, TR_PREC_F32_STORAGE = 1 };

typedef struct tr_ctx tr_ctx;

/* Creates a context for n_slab problems (host arrays) and allocates its
 * device workspace.  Errors: TR_EINVAL (shapes, levels not dividing, nmu odd,
 * non-symmetric mu), TR_ENOMEM, TR_EHIP. */
int tr_create(tr_ctx **out, const tr_problem *probs, int n_slab, const tr_solver_cfg *cfg);
int tr_destroy(tr_ctx *ctx);
const char *tr_error_string(int code);

/* Element offset of slab `slab` inside pooled arrays of `kind`, and the total
 * element count of that kind (host outputs).  Errors: TR_EINVAL. */
int tr_layout(const tr_ctx *ctx, int kind, int slab, long long *offset, long long *total);

/* Overrides the isotropic incoming intensity per group of one slab (host
 * arrays [ng]; NULL keeps the current side). */
int tr_set_incoming(tr_ctx *ctx, int slab, const double *inc_left, const double *inc_right);

/*
 * A1 (paper Sec. 2 group opacities and Planck function).  For every slab,
 * cell and group, at T_i:
 *  - point slabs: kappa[g][i] = kappa_g(T_i), B[g][i] = group Planck integral
 *      B_g = (aR c T^4 / 2) (15/pi^4) int_{nu_g/T}^{nu_{g+1}/T} t^3/(e^t-1) dt;
 *  - spectral slabs: kappa[g][i] = sigma_E,g(T_i, T_r,i), B[g][i] =
 *    sigma_B,g B_g / sigma_E,g (so that kappa B is the group emission), and
 *    sigR[g][i] = sigma_R,g(T_i, T_r,i), with T_r = (Egrey / aR)^(1/4)
 *    (Egrey NULL: T_r = T);
 * and dS[i] = d/dT sum_g 2 sigma_B,g B_g at T_i.  The sweep and the LO
 * solves take kappa as the absorption opacity and kappa B as the emission.
 * T, Egrey: cell (pooled); kappa, B, sigR: gi (pooled); dS: cell (pooled,
 * nullable); sigR is written for spectral slabs only (nullable when no slab
 * is spectral).  Errors: TR_EINVAL (sigR NULL with a spectral slab).
 */
int tr_opacity(tr_ctx *ctx, const double *T, const double *Egrey, double *kappa, double *B, double *sigR,
               double *dS, hipStream_t stream);

/*
 * A2 + partial A3: one transport sweep (paper Sec. 5: implicit Euler, simple
 * corner balance) of every (group, direction) of every slab with opacity and
 * Planck tables kappa, B (gi), previous-time-level corner intensities I_prev
 * (I), writing I_out (I) and the half-range partial moments
 *   mom[h][g][i][2] = (sum_{m in h} w Ibar, sum_{m in h} w mu^2 Ibar),
 *   bnd[h][g][3]    = outgoing edge sums (sum w psi, sum w mu psi,
 *                     sum w mu^2 psi) of half h at its outflow boundary,
 * h = 0 for mu > 0, 1 for mu < 0.  mom has 4 * gi elements per slab, bnd
 * 6 * ng (offsets: 4 * gi offset, 6 * g offset).  I_prev and I_out must not
 * alias.  With TR_PREC_F32_STORAGE, I_prev and I_out point to float arrays.
 */
int tr_sweep(tr_ctx *ctx, const double *kappa, const double *B, const double *I_prev, double *I_out,
             double *mom, double *bnd, hipStream_t stream);

/*
 * A3: QD factors from sweep partials (paper Eqs. f_g, c_g, mloqd-bcs):
 * f[g][i] = chi/phi (gi), fbnd[g][2] edge factors, C[g][2] = (C^-, C^+),
 * Phi[g][2] = F_in - c C E_in (g2).  Isotropic quadrature values replace
 * 0/0 ratios.
 */
int tr_moments(tr_ctx *ctx, const double *mom, const double *bnd, double *f, double *fbnd, double *C,
               double *Phi, hipStream_t stream);

/* Coefficients of one frequency level (all device, pooled level-l arrays, or
 * for level 0 the fine-grid tables). */
typedef struct tr_lo_coeffs {
  /* level 0 (fine): */
  const double *kappa, *B;   /* gi, tables at the level's temperature */
  const double *f, *fbnd;    /* gi, g2 QD factors */
  const double *sigRc;       /* gi, cell values of sigma_R,g (spectral
                                slabs); NULL: kappa (point law) */
  /* levels >= 1: */
  const double *sigE, *emis; /* [n][nx] absorption, emission e = sum 2 kappa B */
  const double *a, *b;       /* [n][nx+1] coefficients of E right / left of edge */
  const double *sigR;        /* [n][nx+1] edge opacity */
  /* all levels: */
  const double *C, *Phi;     /* [n][2] boundary factors / inhomogeneous part */
  const double *Eold, *Fold; /* [n][nx], [n][nx+1] previous time level */
} tr_lo_coeffs;

typedef struct tr_lo_fields {
  double *E;    /* [n][nx]   */
  double *F;    /* [n][nx+1] */
  double *Ebnd; /* [n][2]    */
} tr_lo_fields;

/* Writable level coefficients (output of tr_restrict). */
typedef struct tr_lo_out {
  double *sigE, *emis, *a, *b, *sigR, *C, *Phi, *Eold, *Fold;
  double *Esum; /* [n][nx] sum of the finer E over each group (E* of the MEB) */
} tr_lo_out;

/*
 * A4 / A6: discrete LOQD equations of every group of level `level` (paper
 * Eqs. mloqd1-d, mloqd2-d; coarse Eqs. mloqd1-d-gamma, mloqd2-d-gamma; the
 * boundary conditions Eq. mloqd-bcs closed on boundary half cells).  The
 * tridiagonal system in (E_{1/2}, E_1..E_nx, E_{nx+1/2}) is solved per group.
 */
int tr_lo_solve(tr_ctx *ctx, int level, const tr_lo_coeffs *in, const tr_lo_fields *out, hipStream_t stream);

/*
 * A5: restriction of level `from` (coefficients + its solution) to level
 * `to` > from (paper Eqs. coeff-gamma, g-notation, eta-gamma, coeff-Gamma,
 * eta-Gamma): E-weighted sigma_E, right/left E-weighted a, b, |F|-weighted
 * sigma_R with the upwind-split compensation eta, E_boundary-weighted C, and
 * sums of emission, Phi and old-time values.  For from = 0 the fine
 * coefficients come from kappa/B (at the stage temperature) and f, fbnd.
 */
int tr_restrict(tr_ctx *ctx, int from, int to, const tr_lo_coeffs *in, const tr_lo_fields *sol,
                const tr_lo_out *out, hipStream_t stream);

/*
 * A7: grey LOQD + MEB, one Newton iteration (paper Eq. eb-Gamma-d, Newton
 * with the diagonal Frechet derivative D of the grey sigma_E, Eq.
 * f-derivative-d).  grey: level-last coefficients; Tstar: stage temperature;
 * Told: previous time level; dS: d/dT sum 2 kappa B at Tstar; Estar: stage
 * spectrum total; D: secant derivative (cell arrays).  Writes T_out = Tstar +
 * alpha + beta E (floored at Tstar/2) and the grey fields.
 */
int tr_grey_solve(tr_ctx *ctx, const tr_lo_coeffs *grey, const double *Tstar, const double *Told,
                  const double *dS, const double *Estar, const double *D, double *T_out,
                  const tr_lo_fields *out, hipStream_t stream);

/* Caller-owned step state (device, pooled). */
typedef struct tr_state {
  double *T;       /* cell: material temperature */
  const double *I_prev; /* I: corner intensities of the previous time level
                           (float with TR_PREC_F32_STORAGE) */
  double *I_out;   /* I: written by every sweep; holds I^j after the step */
  double *E, *F, *Ebnd; /* gi, ge, g2: fine LO solution (old-time values in,
                           new values out) */
  double *f, *fbnd, *C; /* gi, g2, g2: QD factors of the last sweep */
  double *Egrey;   /* cell: grey energy density of the last grey solve */
} tr_state;

/* Fills a state with the initial condition T = T0, I^0 = B_g(T0) in every
 * corner and direction, E = (1/c) sum w I^0, F = 0 and the factors of I^0
 * (written to I_out; the caller uses I_out as I_prev of the first step). */
int tr_state_init(tr_ctx *ctx, const tr_state *st, double T0, hipStream_t stream);

enum { TR_T_OPACITY = 0, TR_T_SWEEP = 1, TR_T_MOMENTS = 2, TR_T_LO_FINE = 3, TR_T_RESTRICT = 4,
       TR_T_LO_COARSE = 5, TR_T_GREY = 6, TR_T_N = 8 };

typedef struct tr_stats {
  long long n_ti;  /* transport sweeps */
  long long n_c;   /* cycles */
  long long n_lo;  /* group LO solves (grey counted 1) */
  long long n_floor; /* temperature floor activations */
  int n_outer;     /* transport iterations of the last step incl. s = 0 */
  int cycles[64];  /* cycles per transport iteration of the last step */
  double t_ms[TR_T_N];     /* with cfg.timing: summed kernel time per group
                              (TR_T_*), over launches that did work; with
                              tr_set_sweep_timing only t_ms[TR_T_SWEEP].
                              Inside tr_step the QD factors after a sweep are
                              formed by the first fine LO solve (time under
                              TR_T_LO_FINE; TR_T_MOMENTS stays 0) */
  long long n_launch[TR_T_N]; /* timed launch groups per TR_T_* (sweep: kernel
                                 launches, one per non-empty slab-size bucket
                                 and transport iteration) */
  long long n_seeded;   /* cell factors replaced by the closure */
  long long n_fallback; /* closure predictions rejected (outside (0, 1)) */
} tr_stats;

/*
 * A8: one backward-Euler step of paper Alg. 3 for every slab (V/W/F cycles,
 * grid skipping, inner/outer infinity-norm tests, lmax cap).  replay (host,
 * nullable): per slab, a row of 64 ints = cycles per transport iteration
 * (0 terminates; a row starting with 0 leaves that slab free-running),
 * executed instead of the convergence tests.  stats (host,
 * nullable): [n_slab] counters accumulated over calls.  The step runs on
 * `stream` after the work already queued there (its graphs are captured on a
 * stream of the library's own and launched on `stream`); the call returns
 * once the host has seen every slab
 * stop (the stats are final), while the last copy into st->T may still be
 * in flight: work queued on `stream` afterwards sees the results, the host
 * synchronises `stream` before reading device memory directly.
 * Errors: TR_ENOCONV, TR_ENAN, TR_EHIP.
 */
int tr_step(tr_ctx *ctx, const tr_state *st, const int *replay, tr_stats *stats, hipStream_t stream);

/*
 * A8: nsteps consecutive free-running steps (as nsteps calls of tr_step
 * without replay, with no return to the caller in between).  Step k uses the
 * state with I_prev and I_out exchanged k times, as a caller of tr_step
 * exchanges them after each step (so both buffers must be writable); after
 * the call the caller exchanges its two pointers once more when nsteps is
 * odd.  Every step runs on `stream`.  stats (host, nullable)
 * as in tr_step, accumulated over the steps.  The call stops at the first failing
 * step and returns its error; *done (host, nullable) receives the number of
 * steps completed.  Errors: TR_EINVAL (nsteps < 0) and those of tr_step.
 */
int tr_run(tr_ctx *ctx, const tr_state *st, int nsteps, tr_stats *stats, int *done, hipStream_t stream);

/*
 * Alg. 1 (paper Sec. 3.1): one backward-Euler step of every slab by the
 * two-level QD method on the single fine frequency grid.  Transport
 * iterations s = 0, 1, ... (no sweep at s = 0): opacities at T^(s), sweep,
 * QD factors, then the multigroup LOQD equations (Eqs. mloqd1-d, mloqd2-d)
 * and the multigroup MEB (Eq. eb-group) solved together for T^(s+1), E_g,
 * F_g; stop from s = 1 on when the infinity-norm changes of T and of the
 * total energy density sum_g E_g are at most eps (tr_solver_cfg) of their
 * norms.  The paper leaves the solver of the coupled system open: here
 * Newton iterations in T with the group emission linearised, a per-group
 * secant derivative of sigma_E,g (Eq. f-derivative-d per group) and the
 * cell MEB eliminated, so that the groups couple through phi = sum_g c
 * sigma_E,g E_g; per slab the dense nx x nx system for phi is formed from
 * the groups' tridiagonal factors and solved by Gaussian elimination with
 * partial pivoting, all on the device; each Newton step ends when the
 * relative temperature change reaches rounding.  State as for tr_step
 * (I_prev in, I_out: the last sweep; E, F, Ebnd, f, fbnd, C, T, Egrey =
 * sum_g E_g out).  stats (host, nullable): n_ti sweeps, n_c Newton
 * iterations, n_lo group solves (two per group and Newton iteration),
 * cycles[s] Newton iterations of transport iteration s.  The context's
 * workspace for it (about 8 ng nx^2 + 100 ng nx bytes per slab) is
 * allocated at the first call; the host synchronises the stream after
 * every Newton iteration.  Errors: TR_EINVAL (a slab with more than 512
 * cells), TR_ENOCONV (no convergence in max_outer transport or 60 Newton
 * iterations), TR_ENAN, TR_EHIP, TR_ENOMEM.
 */
int tr_alg1_step(tr_ctx *ctx, const tr_state *st, tr_stats *stats, hipStream_t stream);

/*
 * A8: cycle and lmax of the following tr_step calls (the context's grids stay:
 * V visits none of the intermediate grids, W the second grid, F every
 * intermediate grid from coarse to fine).  Which cycle, hierarchy and lmax
 * cost least depends on the stage of the TRT process and on the time step
 * (Sec. 6 and 7); this lets a caller choose them step by step.  Every
 * intermediate grid's restriction tables and buffers are made at tr_create,
 * so a change needs no new device memory; a schedule's graphs are captured
 * at its first step and kept.  Host only, takes effect
 * at the next tr_step.  Errors: TR_EINVAL (cycle not TR_CYCLE_*, lmax outside
 * 1..64).
 */
int tr_set_schedule(tr_ctx *ctx, int cycle, int lmax);

/*
 * A8 with the hierarchy chosen per step: the following tr_step calls visit,
 * after each grey solve, the context grids grids[0..n-1] (host, indices of
 * the context's intermediate grids 1..n_levels-2, distinct, in the order
 * given) and run at most lmax cycles per transport iteration.  This selects
 * the grid hierarchy of Alg. 3 (fine grid, the listed grids, grey) and its
 * schedule S per time step: n = 0 is the two-grid V cycle, one grid a W
 * cycle through that grid, the intermediate grids from coarse to fine an F
 * cycle over that sub-hierarchy.  Which hierarchy costs least depends on the
 * stage of the TRT process and the time step (Sec. 6 and 7).  The context
 * builds every intermediate grid's restriction tables at tr_create, so a
 * change needs no device memory; its graphs are captured at the first step
 * and kept.  Host only.  Errors: TR_EINVAL (n or an index out of range, a
 * repeated grid, lmax outside 1..64).
 */
int tr_set_grids(tr_ctx *ctx, int n, const int *grids, int lmax);

/*
 * Sweep kernel timing inside tr_step.  on = 1: the transport sweeps of
 * iterations s >= 1 are launched outside the replayed graphs, each launch
 * recording its own start and end on HIP events, and their kernel time is
 * added to tr_stats.t_ms[TR_T_SWEEP] (launches in n_launch[TR_T_SWEEP]).
 * Each is queued behind the previous iteration before the host waits for
 * it, so one more launch at the end of a step finds no slab active (it
 * does nothing and is not counted).  on = 0 (default):
 * sweeps stay inside the graphs, untimed.  Errors: TR_EINVAL (on not 0/1).
 */
int tr_set_sweep_timing(tr_ctx *ctx, int on);

/*
 * Batched launch tiles.  Sweep work is grouped by slab size into 6 buckets
 * (nx <= 64, 128, 256, 512, 1024, larger), ordered longest slab first.  A
 * bucket's tile is (K, split): its wavefronts own K in {1, 2, 4, 8} cells per
 * lane and pass, and split in {1, 2, 4} wavefronts share the directions of
 * one (group, half range) (more wavefronts in flight for small problems).
 * tr_autotune times the 12 tiles on each non-empty bucket (reps launches
 * each, on the given I buffers and the context's current opacity tables) and
 * keeps the fastest; K_out, split_out (host [6]) and us_out (host [6][12],
 * microseconds per launch, tile q = (K index q / 3, split index q % 3)) report
 * the result (each nullable).  tr_set_tiles applies a cached choice (split
 * nullable: 1); tr_get_tiles reads the current one and the items per bucket
 * (host [6] each; split, items nullable).  Tiles change only the association
 * of the sweep's prefix scan and of its direction sums (results at roundoff).
 * Errors: TR_EINVAL (K or split outside the sets above).
 */
int tr_autotune(tr_ctx *ctx, const double *I_prev, double *I_out, int reps, int *K_out, int *split_out,
                double *us_out, hipStream_t stream);
int tr_set_tiles(tr_ctx *ctx, const int *K, const int *split);
int tr_get_tiles(const tr_ctx *ctx, int *K, int *split, int *items);

/*
 * Learned closure (not part of the paper's method; the plain sweeps still
 * decide convergence).  A multilayer perceptron 7 -> 128 -> 128 -> 128 -> 2 with ReLU
 * hidden layers; output 0 through a logistic sigmoid s predicts the change of
 * the group Eddington factor over a time step, f_seed = f + 0.05 (2 s - 1);
 * output 1 is a prolongation correction (log change of the within-block
 * spectral shape).  Products run in bfloat16 on MFMA with float32
 * accumulation.  Parameters: float32 vector of tr_mlp_nparam() entries,
 * row-major W1 [8][128] (input row 7 unused), b1 [128], W2 [128][128], b2, W3
 * [128][128], b3, W4 [128][2], b4 [2].  Inputs X [n][8] float32 standardised
 * features (column 7 ignored); targets Y [n][2] float32.  `work` is
 * caller-owned device scratch of tr_mlp_work_bytes(n)
 * (tr_mlp_train_work_bytes(batch) for training).
 */
int tr_mlp_nparam(void);
size_t tr_mlp_work_bytes(long long n);
size_t tr_mlp_train_work_bytes(int batch);
/* out [n][2] = (sigmoid(o_0), o_1). */
int tr_mlp_forward(const float *params, const float *X, long long n, float *out, void *work, hipStream_t stream);
/* grad [nparam] of the mean-squared loss (1/n) sum (fhat-f)^2 + (rhat-r)^2 and
 * the loss (device float). */
int tr_mlp_grad(const float *params, const float *X, const float *Y, long long n, float *grad, float *loss,
                void *work, hipStream_t stream);
/*
 * tr_mlp_grad without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  It allocates nothing: its pass work lives in a
 * file-scope device array of the library (10.4 MiB, held by every GPU the
 * library runs on until the process ends), sized for at most
 * TR_MLP_NOALLOC_MAX_N samples.  The array's address on the current device
 * (the device of `stream`, which must be current) is looked up on the first
 * call on that device.  Results equal tr_mlp_grad's bit for bit.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and give wrong gradients; the caller orders them.
 * No state carries over between calls (each writes every word it reads).
 * Errors: TR_EINVAL (a null pointer, n < 1 or n > TR_MLP_NOALLOC_MAX_N),
 * TR_EHIP.
 */
enum { TR_MLP_NOALLOC_MAX_N = 4096 };
int tr_mlp_grad_noalloc(const float *params, const float *X, const float *Y, long long n, float *grad, float *loss,
                        hipStream_t stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected, t >= 1). */
int tr_mlp_adam(float *params, float *m, float *v, const float *grad, int t, float lr, hipStream_t stream);
/* One epoch of minibatch Adam in the order given by perm [n] (device ints);
 * *t counts Adam steps (host), loss_sum (device float) accumulates the batch
 * losses. */
int tr_mlp_train_epoch(float *params, float *m, float *v, int *t, float lr, const float *X, const float *Y,
                       long long n, const int *perm, int batch, void *work, float *loss_sum, hipStream_t stream);

/*
 * Closure inputs for every slab, group and cell (sample g * nx + i of each
 * slab, pooled like gi): log T_i, log nu_g, log(kappa_g,i dx_i), log T_{i-1},
 * log T_{i+1} (left neighbour of cell 0: T_left when positive, else T_0;
 * right neighbour of the last cell: itself), the factor f_g,i, and
 * log(T_i / T_prev_i) (T_prev: cell array of the previous time step's start,
 * nullable = no change), standardised with mean/std (host [7] each).
 * X: [gi total][8] float32 (column 7 zero).
 */
int tr_mlp_features(tr_ctx *ctx, const double *T, const double *T_prev, const double *kappa, const double *f,
                    const float *mean, const float *std, float *X, hipStream_t stream);

/*
 * Training targets from two consecutive converged steps (gi arrays): Y [gi][2]
 * float32 = (s_g,i, r_g,i), s = 1/2 + (f - f_prev) / 0.1 clipped to
 * [0.01, 0.99] (the sigmoid value that reproduces the factor change), r =
 * log((E_g/E_p) / (E'_g/E'_p)) the change of the within-block spectral shape,
 * E_p the sum over the `block` consecutive groups containing g (0 where a
 * share is at or below 1e-290), clipped to [-2, 2].
 */
int tr_closure_targets(tr_ctx *ctx, const double *f, const double *f_prev, const double *E_new, const double *E_prev,
                       int block, float *Y, hipStream_t stream);

/*
 * Prolongation with the learned shape correction (the paper's method moves
 * coarse-grid information back to the fine grid through T only; prolongation
 * between frequency grids appears there as a general multigrid operator).
 * For every slab, coarse group p of level `level` (>= 1) and cell i, the fine
 * groups g of p get E_fine = E_p,i w_g,i / sum_{g' in p} w_g',i with
 * w = E_prev exp(r), r the closure's second output (r: [gi][2] float32 as
 * written by tr_mlp_forward on tr_mlp_features rows; column 1 is read; NULL
 * means r = 0); a block whose weights sum to 1e-290 or less is split evenly.
 * E_coarse: pooled like kind TR_K_LEV_PI + level; E_prev, E_fine: gi arrays
 * (distinct).  Prolonged groups of a block sum to E_p.
 * Errors: TR_EINVAL (level out of range, ng not a multiple of the level).
 */
int tr_prolong(tr_ctx *ctx, int level, const double *E_coarse, const double *E_prev, const float *r, double *E_fine,
               hipStream_t stream);

/*
 * Attaches a trained closure to the context (params: device, kept by the
 * caller; mean/std: host [7]; NULL params detaches).  While attached, tr_step
 * adds the network's predicted factor change to the previous step's cell QD
 * factors at the start of every step (transport iteration s = 0); a seeded
 * factor outside (0, 1) keeps the old one.  The temperature history the
 * inputs use restarts with tr_state_init.  All later transport iterations
 * sweep and test convergence exactly as without the closure.
 */
int tr_set_closure(tr_ctx *ctx, const float *params, const float *mean, const float *std);

/*
 * A9 (extension): the seeding step of the attached closure on its own, the
 * kernel tr_step runs at s = 0.  For every (group, cell) of every slab it
 * forms the network's inputs from T, T_prev (the previous step's start
 * temperature; NULL: none), kappa (gi tables at T) and the factors f (gi),
 * evaluates the network (bfloat16 products, float32 accumulation) and sets
 * f <- f + 0.05 (2 s - 1), s the sigmoid of output 0, where that lies in
 * (0, 1); elsewhere f is kept.  counts (device, 2 values, accumulated):
 * factors seeded, factors kept.  All pointers are device pointers owned by the
 * caller.  Errors: TR_EINVAL (no closure attached, a null pointer other
 * than T_prev).
 */
int tr_closure_seed(tr_ctx *ctx, const double *T, const double *T_prev, const double *kappa, double *f,
                    unsigned long long *counts, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* TR_H */
