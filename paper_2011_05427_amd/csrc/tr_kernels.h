// Kernel argument structures and host launchers (internal to the library).
#pragma once

#include "tr_common.h"

#define TR_LO_K 4    // rows per thread of the group LO solves (one block of up to 512 threads per system)
#define TR_GREY_K 4  // rows per thread of the grey solve (one block of up to 512 threads per slab)

enum { PRED_ALL = 0, PRED_CYCLE = 1, PRED_DONECYC = 2, PRED_SWEEP = 3, PRED_ACTIVE = 4 };

// Coefficients of a level (fine: kappa/B/f/fbnd; coarse: level arrays).
struct LoIn {
  const double *kappa, *B, *f, *fbnd;
  const double *sgr;  // fine level: cell sigma_R table (spectral slabs); null: kappa
  const double *sigE, *emis, *a, *b, *sigR;
  const double *C, *Phi, *Eold, *Fold;
  // fine level, first cycle of an iteration with a sweep: the QD factors are
  // formed from the sweep's half-range partials (mom, bnd) inside the solve
  // and written to f_out, fbnd_out, C_out, Phi_out (all null otherwise)
  const double *mom, *bnd;
  double *f_out, *fbnd_out, *C_out, *Phi_out;
};

struct LoSol {
  double *E, *F, *Ebnd;
};

struct LoOut {
  double *sigE, *emis, *a, *b, *sigR, *C, *Phi, *Eold, *Fold, *Esum;
  // restriction to the grey level in a step: also reduce the 64-group chunk
  // partials of dS into the cell array (both null otherwise)
  const double *dSpart;
  double *dS;
};

struct GreyArgs {
  LoIn grey;             // grey-level coefficient arrays
  const double *Estar;   // grey-level Esum (stage spectrum total)
  LoSol sol;             // grey-level fields
  const double *Tstar;   // cell: stage temperature
  double *Tout;          // cell: new temperature (may equal Tstar)
  const double *Told;    // cell: previous time level
  const double *dS;      // cell: d/dT of the emission sum_g 2 kappa_g B_g at Tstar
  const double *D;       // cell: explicit Frechet derivative (nullable)
  double *Tprev, *sigprev;         // secant memory (step mode)
  double *Egrey;                   // cell: grey E output (nullable)
  double *Tcyc, *Ecyc, *Ts, *Es;   // convergence references (step mode)
  const Ctl *ctl_dummy;             // any valid control record (read, unused, without control)
  int stage_mask;                   // bit l: grid l is visited after each grey solve (LO solves counted)
  int secant, end_cycle, lmax;
  double eps, eps_inner;
};

struct LaunchEnv {
  const SlabDev *sd;
  ProbDev pd;
  hipStream_t stream;
};

struct Table {
  const Item *d;
  int n;
};

// run = 1 or 4 groups per thread; tab items = (slab, chunk * ncb + cell block)
// with ncb = ceil(nx / (4 run)).  spec: slabs with the spectral opacity model
// get the group averages at (T, T_r from Eg; Eg null: T_r = T) and their
// sigma_R in sgr; without spec every slab gets the point law and the group
// Planck integrals (the initial state and the incoming radiation use B_g).
void launch_opacity(const LaunchEnv &env, const Table &tab, int run, const Ctl *ctl, int pmode, int lcyc,
                    const double *T, double *kappa, double *B, double *dSpart, bool spec = false,
                    const double *Eg = nullptr, double *sgr = nullptr, double *dem = nullptr);
// dS per cell from the chunk partials; tab items = (slab, first of 64 cells).
void launch_dS_sum(const LaunchEnv &env, const Table &tab, const Ctl *ctl, int pmode, int lcyc, const double *dSpart,
                   double *dS);
// Sweep tiles: K cells per lane and pass (K in {1, 2, 4, 8}); split in
// {1, 2, 4} wavefronts share the directions of one (group, half range).
// f32: corner intensities stored as float (binary64 arithmetic inside).
// With ev0 / ev1 the launch records the kernel's own start and end on them.
// nt_hint: stream the intensities past the caches (arrays larger than the
// last-level cache; see Pair).
void launch_sweep(const LaunchEnv &env, const Table &tab, int K, int split, bool f32, bool nt_hint, const Ctl *ctl,
                  int pmode, int lcyc, const double *kappa, const double *B, const void *Ip, void *Io, double *mom,
                  double *bnd, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_moments(const LaunchEnv &env, const Table &tab, const Ctl *ctl, int pmode, int lcyc, const double *mom,
                    const double *bnd, double *f, double *fbnd, double *C, double *Phi);
void launch_lo(const LaunchEnv &env, const Table &tab, int threads, const Ctl *ctl, int pmode, int lcyc, int level,
               const LoIn &in, const LoSol &sol);
// Restriction work: coarse groups of r <= 16 finer groups are done in one pass
// (except on wide slabs restricted to very few coarse groups, see
// restrict_cpb); larger r in a chunk pass plus a final pass over blocks of
// TR_RFIN_E edges.
// old: also restrict the old-time E and F (out.Eold / out.Fold are written
// only then).  mode 1 (fine to a stage level): kappa and B are computed at
// the cell temperatures T instead of read, in tiles of 63 edges (tables from
// build with restrict_tile(1)), and the stage dS partials of every cell go to
// dsop (S.dsnp[to] rows of nx per slab at S.o_dsop); mode 2 (stage level to
// grey): those partials are added into out.dS.
inline int restrict_tile(int mode) { return mode == 1 ? 63 : 64; }
// In the chunk pass a block of 4 wavefronts covers 64 edges and 4 rcw finer
// groups (rcw per wavefront), giving cpb chunk records per coarse group.  On
// slabs of 16 or more edge tiles rcw starts at 16 (or r / 4 if smaller: one
// record per coarse group), a rule of the slab alone; it then grows (fewer records to write and re-read)
// while a slab's pass keeps at least `target` blocks (4096 over the slabs of
// a context), and so that cpb <= 64.
#define TR_RFIN_E 11
__host__ __device__ inline int restrict_rcw(int r, int nto, int ne, int target) {
  const int ntile = (ne + 63) / 64;
  int rcw = 1;
  if (ntile >= 16)  // wide slabs: at least 16 finer groups per wavefront where r allows
    while (rcw < 16 && 4 * rcw < r) rcw *= 2;
  while (rcw < 32 && 4 * rcw < r && (long long)nto * ((r + 8 * rcw - 1) / (8 * rcw)) * ntile >= target) rcw *= 2;
  while ((r + 4 * rcw - 1) / (4 * rcw) > 64) rcw *= 2;
  return rcw;
}
// One pass unless the single pass would run few long wavefronts: a wide slab
// (8 or more edge tiles) restricted to very few coarse groups (under 256
// wavefront items) takes the chunk pass from r = 8 up.
__host__ __device__ inline bool restrict_single(int r, int nto, int ne) {
  const int ntile = (ne + 63) / 64;
  return r <= 16 && !(r >= 8 && ntile >= 8 && (long long)nto * ntile < 256);
}
__host__ __device__ inline int restrict_cpb(int r, int nto, int ne, int target) {
  if (restrict_single(r, nto, ne)) return 1;
  const int rcw = restrict_rcw(r, nto, ne, target);
  return (r + 4 * rcw - 1) / (4 * rcw);
}
// Edges per block of the final pass: TR_RFIN_E, or a quarter of it (rounded
// down) when 16 or more chunk records per edge are split over four parts.
__host__ __device__ inline int restrict_fin_edges(int cpb) { return cpb >= 16 ? TR_RFIN_E / 4 : TR_RFIN_E; }

struct RestrictTables {
  Table single, part, fin;
};
void launch_restrict(const LaunchEnv &env, const RestrictTables &rt, const Ctl *ctl, int pmode, int lcyc, int from,
                     int to, const LoIn &in, const LoSol &sol, const LoOut &out, double *red, bool old,
                     int mode = 0, const double *T = nullptr, double *dsop = nullptr);
void launch_grey(const LaunchEnv &env, const Table &tab, int threads, Ctl *ctl, int pmode, int lcyc,
                 const GreyArgs &ga);
// End of a transport iteration (start of s + 1 where the inner iteration is
// done) and the count of slabs still active into out[0] (out[1]: slabs in
// the middle of an inner iteration), one launch; with no slab left active
// the control records are copied to hout.  Then *serial (device) is
// incremented and written to out[2], after the other host writes.
void launch_outer_end(const LaunchEnv &env, Ctl *ctl, int nslab, int max_outer, int *out, Ctl *hout, int *serial);
// Step-start copies of T, Egrey, E, F into the step's reference arrays, of
// the nslab control records from (coherent pinned) host memory ctl_in, Phi
// from C and the incoming intensities (tab_g items = (slab, first of 256
// groups)), and the opacity tables kappa, B, dSpart at T (tab_op and run as
// for launch_opacity, every slab), in one launch.
void launch_step_start(const LaunchEnv &env, const double *T, const double *Egrey, const double *E, const double *F,
                       long long n_cell, long long n_gi, long long n_ge, double *Told, double *Ts, double *Tcyc,
                       double *Tstar, double *Es, double *Ecyc, double *Eold, double *Fold, const Ctl *ctl_in,
                       Ctl *ctl, int nslab, const Table &tab_g, const double *C, double *Phi, const Table &tab_op,
                       int run, double *kappa, double *B, double *dSpart, bool spec = false,
                       double *sgr = nullptr);
void launch_copy(const LaunchEnv &env, const double *src, double *dst, long long n);
void launch_fill(const LaunchEnv &env, double *dst, double v, long long n);
void launch_init_state(const LaunchEnv &env, const Table &tab, bool f32, const double *Bt, void *I, double *E,
                       double *F, double *Ebnd, double *mom, double *bnd);
void launch_group_sum(const LaunchEnv &env, const Table &tab, const double *E, double *out);
#define TR_MLP_NFEAT 7   // closure inputs per sample (8 columns, the last zero)
#define TR_MLP_DF 0.05   // scale of the predicted factor change per time step
struct MlpStats {
  double mean[TR_MLP_NFEAT], std[TR_MLP_NFEAT];
};
void launch_mlp_features(const LaunchEnv &env, const Table &tab, const double *T, const double *Tprev,
                         const double *kappa, const double *f, const MlpStats &ms, float *X);
void launch_closure_targets(const LaunchEnv &env, const Table &tab, const double *f, const double *fprev,
                            const double *Enew, const double *Eprev, int blk, float *Y);
// tab items = (slab, first (p, i) of 256) over the level's n_p nx cells.
void launch_prolong(const LaunchEnv &env, const Table &tab, int lev, const double *Ec, const double *Eprev,
                    const float *r, double *Ef);
void launch_seed_f(const LaunchEnv &env, const float *out, double *f, long long n, unsigned long long *counts);
// A9 fused: inputs, network and seeding of f in one kernel (tab = the (slab,
// first of 256 (g, i)) items); counts[0] += seeded, counts[1] += kept.
void launch_closure_seed(const LaunchEnv &env, const Table &tab, const double *T, const double *Tprev,
                         const double *kappa, double *f, const MlpStats &ms, const float *params,
                         unsigned long long *counts);

// Alg. 1 (single-grid multigroup LOQD + MEB by Newton in T; see the kernels).
#define TR_A1_MAX_CELLS 512  // cells per slab of the Alg. 1 dense solve
// The dense solve holds the matrix in registers up to TR_A1_REG_CELLS cells
// (1024 threads, at most TR_A1_REG_SLOTS rows per thread: R = 1024 / nx row
// groups need ceil(nx / R) <= 40 slots, true for nx <= 200).
#define TR_A1_REG_CELLS 200
#define TR_A1_REG_SLOTS 40
struct A1Args {
  LoIn in;                 // fine tables at T^k, QD factors, old-time values
  const double *dem;       // gi: d/dT of the group emission at T^k
  const double *T, *Told, *Tprev, *kprev;  // cell, cell, cell, gi (previous iterate)
  const double *Ek;        // gi: E of the previous iterate
  double *alpha, *beta;    // cell
  double *w;               // gi
  double *ra, *cp, *dn;     // Thomas factors, per slab at o_gi + 2 o_g, row j of group g at j ng + g
  double *P;               // per slab ng nx nx partial products (at oP)
  double *M, *rhs, *phi;   // per slab nx nx (at oM); cell; cell
  const long long *oM, *oP;
  const Ctl *ctl;          // slab iterates while ctl[slab].active
  int first;               // first Newton iteration of the transport iteration (D = 0)
  double *E, *F, *Ebnd;    // group solution (state)
  double *Tout, *err;      // new T; per slab max|dT| / max|T|
};

void launch_a1_prep(const LaunchEnv &env, const Table &t_cell, const A1Args &a);
void launch_a1_factor(const LaunchEnv &env, const Table &t_g, const A1Args &a);
// Per-group solves of Alg. 1: items (slab, group), threads >= (nx + 2) /
// TR_LO_K of every slab (at most 512), 64 bytes of LDS per thread.
void launch_a1_solve_blk(const LaunchEnv &env, const Table &t_sg, int threads, const A1Args &a, bool with_phi);
void launch_a1_rhs(const LaunchEnv &env, const Table &t_cell, const A1Args &a);
void launch_a1_cols(const LaunchEnv &env, const Table &t_gi, const A1Args &a);
void launch_a1_mred(const LaunchEnv &env, const Table &t_mm, const A1Args &a);
void launch_a1_dense(const LaunchEnv &env, int nslab, int max_nx, const A1Args &a);
void launch_a1_update(const LaunchEnv &env, int nslab, const A1Args &a, double *Tprev);
void launch_a1_outer(const LaunchEnv &env, int nslab, const Ctl *ctl, const double *T, const double *Ts,
                     const double *E, double *Esum, const double *Esp, double *out);
