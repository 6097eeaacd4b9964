// C ABI of the MLQD library: context set-up, pooled layout, stage entry points
// and the host orchestration of one time step (paper Alg. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "tr.h"
#include "tr_kernels.h"

// Instantiated graph sets kept per context (state buffers x schedule); the
// oldest is destroyed beyond this.
#define TR_GRAPH_CACHE 12

#define TR_NBUCKET 6
#define TR_LLC_BYTES (256LL << 20)  // last-level (Infinity) cache of the device

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct tr_ctx {
  int nslab = 0;
  tr_solver_cfg cfg{};
  int nlev = 0;
  std::vector<int> sched;
  int grey_threads = 64;  // block size of the grey solve
  int opac_run = 4;       // groups per thread of the opacity kernel (1 or 4)
  // some slab has the spectral opacity model: the opacity launches evaluate
  // the group averages (radiation temperature from the grey E) and write the
  // sigma_R table; grey stages take tables at T~ and the plain restriction
  bool spectral = false;
  // the sweep streams its intensities past the caches (non-temporal hint)
  // when the previous and new arrays together exceed the last-level cache
  bool sweep_nt = false;
  std::vector<SlabDev> hs;  // host copies of the slab descriptors
  std::vector<double> h_inc;
  // totals per kind
  long long n_cell = 0, n_edge = 0, n_I = 0, n_gi = 0, n_ge = 0, n_g = 0, n_nu = 0, n_mu = 0, n_chunk = 0, n_red = 0;
  long long n_lpi[TR_MAXLEV] = {}, n_lpe[TR_MAXLEV] = {}, n_lp2[TR_MAXLEV] = {};
  std::vector<void *> allocs;
  SlabDev *d_sd = nullptr;
  ProbDev pd{};
  double *d_inc = nullptr;
  // workspace
  double *sigR = nullptr;  // cell sigma_R table (spectral); = kappa otherwise
  double *kappa = nullptr, *B = nullptr, *dSpart = nullptr, *dS = nullptr, *mom = nullptr, *bnd = nullptr, *Phi = nullptr;
  double *Eold = nullptr, *Fold = nullptr, *red = nullptr;
  double *Told = nullptr, *Ts = nullptr, *Tcyc = nullptr, *Tstar = nullptr, *Tprev = nullptr, *sigprev = nullptr;
  double *Ecyc = nullptr, *Es = nullptr;
  struct Lev {
    double *sigE, *emis, *a, *b, *sigR, *C, *Phi, *Eold, *Fold, *E, *F, *Ebnd, *Esum;
  } lev[TR_MAXLEV]{};
  Ctl *d_ctl = nullptr;
  int *h_count = nullptr;  // pinned, coherent: [active slabs, slabs in mid-iteration, iteration serial]
  int *d_serial = nullptr;  // iterations ended so far (device)
  Ctl *h_ctl_out = nullptr;  // pinned, coherent: control records once every slab stopped
  Ctl *h_ctl_in = nullptr;   // pinned: control records uploaded at the step start
  // work tables
  Table t_opac{}, t_dS{}, t_cell{}, t_gi{}, t_g{}, t_grey{};
  // sweep work per slab-size bucket (nx <= 64, 128, 256, 512, 1024, more),
  // longest slabs first; K = cells per lane of each bucket's launch
  Table t_sweep_b[TR_NBUCKET]{};
  int sweep_K[TR_NBUCKET] = {1, 2, 4, 4, 4, 4};
  int sweep_S[TR_NBUCKET] = {1, 1, 1, 1, 1, 1};  // wavefronts sharing a (group, half range)
  // group LO solves per level, by block size 64 << kb (kb = 0..3): a slab's
  // systems take the smallest block that covers them with 4 rows per thread
  Table t_lo[4][TR_MAXLEV]{};
  std::map<std::pair<int, int>, RestrictTables> t_red;
  // stage restrictions fine -> level computing kappa / B themselves (tiles of
  // 63 edges) and their dS partials
  std::map<int, RestrictTables> t_red_op;
  double *dsop = nullptr;
  long long n_dsop = 0;
  std::map<int, Table> t_pro;  // prolongation work per level
  // optional event timing of kernel groups inside tr_step
  struct TimedGroup {
    int cat, cycle, e0, e1;
  };
  std::vector<hipEvent_t> events;
  int ev_used = 0;
  std::vector<TimedGroup> groups;
  // graph replay of one transport iteration (the launch sequence depends on
  // the state pointers, the number of cycles launched, the cycle and lmax)
  struct GraphEntry {
    std::vector<const void *> key;
    // s = 0 (no sweep); s >= 1 with the sweep; s >= 1 without it (the sweep
    // launched separately with its start / end events)
    hipGraphExec_t first = nullptr, next = nullptr, rest = nullptr;
    // s >= 1 with its first cycle only, and the remaining cycles of an
    // iteration (no sweep): the last iteration of a step usually needs one
    hipGraphExec_t next1 = nullptr, tail = nullptr;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t gs = nullptr;  // library stream for graph capture (replays run on the caller's stream)
  // start / end events of the sweep launches of tr_step (one pair per
  // slab-size bucket): the sweep's kernel time is measured in every step
  hipEvent_t ev_sw[TR_NBUCKET][2] = {};
  int sweep_events = 0;  // tr_set_sweep_timing
  int last_iters = 0;    // transport iterations (incl. s = 0) of the previous step's slowest slab
  // learned closure (seeding of the s = 0 cell factors)
  const float *mlp_params = nullptr;
  MlpStats mlp_stats{};
  unsigned long long *d_seed_counts = nullptr;
  double *T_hist = nullptr;  // temperature at the start of the previous closure step
  int have_hist = 0;
  // Alg. 1 (single-grid solve of the multigroup LOQD + MEB), allocated at
  // its first use
  struct A1Work {
    bool ready = false;
    double *dem, *kprev, *w, *ra, *cp, *dn, *P, *M, *rhs, *phi, *alpha, *beta, *Tprev, *Ts, *Esum, *Esp, *Er;
    double *err, *outer, *h_err, *h_outer;  // device and pinned host copies (per slab)
    long long *oM, *oP;
    Table t_mm, t_sg;  // (slab, 256-entry block of M) and (slab, group) items
    int sg_threads = 64;  // block of the per-group solves
  } a1{};
};

namespace {

int hip_err(hipError_t e) { return e == hipSuccess ? TR_OK : TR_EHIP; }

template <class T>
int dalloc(tr_ctx *c, T **p, long long n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  void *q = nullptr;
  if (hipMalloc(&q, sizeof(T) * (size_t)n) != hipSuccess) return TR_ENOMEM;
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return TR_OK;
}

int upload_table(tr_ctx *c, const std::vector<Item> &h, Table &t) {
  t.n = (int)h.size();
  t.d = nullptr;
  if (h.empty()) return TR_OK;
  Item *d = nullptr;
  int rc = dalloc(c, &d, (long long)h.size());
  if (rc) return rc;
  if (hipMemcpy(d, h.data(), sizeof(Item) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return TR_EHIP;
  t.d = d;
  return TR_OK;
}

// Head coefficients c_k = B_k / (k! (k + 3)) of int_0^x t^3/(e^t - 1) dt.
// Odd Bernoulli numbers vanish beyond B_1 = -1/2; the even ones follow from
// B_2j / (2j)! = (-1)^(j+1) 2 zeta(2j) / (2 pi)^(2j), with zeta(2) = pi^2/6
// and zeta(s >= 4) summed directly with an Euler-Maclaurin tail.
std::vector<int> schedule_for(int cycle, int nlev) {
  std::vector<int> s;
  if (cycle == TR_CYCLE_V || nlev <= 2) return s;
  if (cycle == TR_CYCLE_W) {
    s.push_back(1);
    return s;
  }
  for (int l = nlev - 2; l >= 1; --l) s.push_back(l);
  return s;
}

// Block size class of a slab's LO systems (4 rows per thread): 64 << kb
// threads, the smallest that covers nx + 2 rows.  The padding rows of a
// larger block do not change the arithmetic of the system's rows.
int lo_block(int nx) {
  const int need = (nx + 2 + TR_LO_K - 1) / TR_LO_K;
  int kb = 0;
  while ((64 << kb) < need) ++kb;
  return kb;
}

// Work tables of the restriction from -> to; mode 1 = the stage restriction
// fine -> level computing the tables itself (tiles of 63 edges).
int build_restrict_tables(tr_ctx *c, int from, int to, int mode = 0) {
  auto key = std::make_pair(from, to);
  if (mode == 0 ? c->t_red.count(key) != 0 : c->t_red_op.count(to) != 0) return TR_OK;
  const int TE = restrict_tile(mode);
  std::vector<Item> single, part, fin;
  for (int s = 0; s < c->nslab; ++s) {
    const SlabDev &S = c->hs[s];
    const int ne = S.nx + 1;
    const int nf = S.lev_ng[from], nt = S.lev_ng[to];
    const int r = nf / nt;
    const int cpb = restrict_cpb(r, nt, ne, S.rtarget);
    if (restrict_single(r, nt, ne)) {
      // four wavefront items (coarse group, tile of edges) per block
      const int nwi = nt * ((ne + TE - 1) / TE);
      for (int q = 0; 4 * q < nwi; ++q) single.push_back({s, q});
    } else {
      const int ntile = (ne + TE - 1) / TE;
      for (long long q = 0; q < (long long)nt * cpb * ntile; ++q) part.push_back({s, (int)q});
      const int RE = restrict_fin_edges(cpb);
      const int nb = (ne + RE - 1) / RE;
      for (int q = 0; q < nt * nb; ++q) fin.push_back({s, q});
    }
  }
  RestrictTables rt{};
  int rc = upload_table(c, single, rt.single);
  if (!rc) rc = upload_table(c, part, rt.part);
  if (!rc) rc = upload_table(c, fin, rt.fin);
  if (rc) return rc;
  if (mode == 0)
    c->t_red[key] = rt;
  else
    c->t_red_op[to] = rt;
  return TR_OK;
}

LaunchEnv env_of(const tr_ctx *c, hipStream_t st) { return LaunchEnv{c->d_sd, c->pd, st}; }

// LO solves of a level, one launch per block size in use.
void launch_lo_all(const tr_ctx *c, const LaunchEnv &env, const Ctl *ctl, int pmode, int lcyc, int level,
                   const LoIn &in, const LoSol &sol) {
  for (int kb = 0; kb < 4; ++kb) launch_lo(env, c->t_lo[kb][level], 64 << kb, ctl, pmode, lcyc, level, in, sol);
}

int sweep_bucket(int nx) {
  int b = 0, lim = 64;
  while (b < TR_NBUCKET - 1 && nx > lim) {
    ++b;
    lim *= 2;
  }
  return b;
}

// One sweep launch per non-empty slab-size bucket; with timed, each launch
// records its start and end on the bucket's event pair.
void launch_sweeps(const tr_ctx *c, const LaunchEnv &env, const Ctl *ctl, int pmode, const double *kappa,
                   const double *B, const void *Ip, void *Io, double *mom, double *bnd, bool timed = false) {
  for (int b = 0; b < TR_NBUCKET; ++b)
    launch_sweep(env, c->t_sweep_b[b], c->sweep_K[b], c->sweep_S[b], c->cfg.precision == TR_PREC_F32_STORAGE,
                 c->sweep_nt, ctl, pmode, 0, kappa, B, Ip, Io, mom, bnd, timed ? c->ev_sw[b][0] : nullptr,
                 timed ? c->ev_sw[b][1] : nullptr);
}

// Kernel time of the last timed sweep launches (after a synchronisation).
void sweep_time(const tr_ctx *c, double *t_ms, long long *n_launch) {
  for (int b = 0; b < TR_NBUCKET; ++b) {
    if (c->t_sweep_b[b].n == 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_sw[b][0], c->ev_sw[b][1]) == hipSuccess) {
      t_ms[TR_T_SWEEP] += ms;
      n_launch[TR_T_SWEEP] += 1;
    } else {
      (void)hipGetLastError();  // no timing for this launch; leave no error behind
    }
  }
}

// Events that only time work read after a stream synchronisation: without
// the system-scope fence of a default event, recording them does not add a
// cache writeback and invalidation to the timed interval.
hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Waits until the end kernel of the iteration with serial number `expect`
// has published its counts (h_count[2]), spinning on the coherent host word
// instead of a stream synchronisation; after about a second without it the
// stream is synchronised (that also reports a failed launch), and a serial
// still missing after that is an error.
int wait_iteration(tr_ctx *c, int expect, hipStream_t st) {
  volatile const int *ser = c->h_count + 2;
  for (long long k = 0; *ser != expect; ++k) {
    if ((k & 4095) == 4095) {
      static const double limit_s = 1.0;
      static thread_local std::chrono::steady_clock::time_point t0;
      if (k == 4095) t0 = std::chrono::steady_clock::now();
      if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit_s) {
        const int rc = hip_err(hipStreamSynchronize(st));
        if (rc) return rc;
        return *ser == expect ? TR_OK : TR_EHIP;
      }
    }
  }
  return TR_OK;
}

// Event marks around kernel groups (cfg.timing).  A group records its cycle
// index (-1 outside the cycles) so that launches of cycles a slab skipped can
// be left out of the sums.
int tim_mark(tr_ctx *c, hipStream_t st) {
  if (c->ev_used == (int)c->events.size()) {
    hipEvent_t e;
    if (timing_event(&e) != hipSuccess) return -1;
    c->events.push_back(e);
  }
  const int k = c->ev_used++;
  if (hipEventRecord(c->events[k], st) != hipSuccess) return -1;
  return k;
}

struct TimedScope {
  tr_ctx *c;
  hipStream_t st;
  int cat, cycle, e0;
  TimedScope(tr_ctx *c_, hipStream_t st_, int cat_, int cycle_) : c(c_), st(st_), cat(cat_), cycle(cycle_), e0(-1) {
    if (c->cfg.timing) e0 = tim_mark(c, st);
  }
  ~TimedScope() {
    if (!c->cfg.timing || e0 < 0) return;
    const int e1 = tim_mark(c, st);
    if (e1 >= 0) c->groups.push_back({cat, cycle, e0, e1});
  }
};

// After a synchronisation: adds the recorded durations of groups whose cycle
// ran (cycle < ncyc_ran, or outside the cycles) to the stats of every slab.
void tim_collect(tr_ctx *c, int ncyc_ran, double *t_ms, long long *n_launch) {
  for (const auto &g : c->groups) {
    if (g.cycle >= ncyc_ran) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->events[g.e0], c->events[g.e1]) == hipSuccess) {
      t_ms[g.cat] += ms;
      n_launch[g.cat] += 1;
    }
  }
  c->groups.clear();
  c->ev_used = 0;
}

LoIn fine_in(const tr_ctx *c, const double *kappa, const double *B, const double *f, const double *fbnd,
             const double *C, const double *Phi, const double *Eold, const double *Fold) {
  LoIn in{};
  in.kappa = kappa;
  in.B = B;
  in.sgr = c->sigR;
  in.f = f;
  in.fbnd = fbnd;
  in.C = C;
  in.Phi = Phi;
  in.Eold = Eold;
  in.Fold = Fold;
  return in;
}

LoIn level_in(const tr_ctx *c, int l) {
  LoIn in{};
  const auto &L = c->lev[l];
  in.sigE = L.sigE;
  in.emis = L.emis;
  in.a = L.a;
  in.b = L.b;
  in.sigR = L.sigR;
  in.C = L.C;
  in.Phi = L.Phi;
  in.Eold = L.Eold;
  in.Fold = L.Fold;
  return in;
}

LoSol level_sol(const tr_ctx *c, int l) {
  const auto &L = c->lev[l];
  return LoSol{L.E, L.F, L.Ebnd};
}

LoOut level_out(const tr_ctx *c, int l) {
  const auto &L = c->lev[l];
  return LoOut{L.sigE, L.emis, L.a, L.b, L.sigR, L.C, L.Phi, L.Eold, L.Fold, L.Esum, nullptr, nullptr};
}

// Grey-level output of a restriction inside a step: it also reduces the dS
// chunk partials of the current opacity tables for the grey solve.
LoOut grey_out(const tr_ctx *c) {
  LoOut o = level_out(c, c->nlev - 1);
  o.dSpart = c->dSpart;
  o.dS = c->dS;
  return o;
}

LoIn coeffs_in(const tr_lo_coeffs *in) {
  LoIn r{};
  r.kappa = in->kappa;
  r.B = in->B;
  r.sgr = in->sigRc;
  r.f = in->f;
  r.fbnd = in->fbnd;
  r.sigE = in->sigE;
  r.emis = in->emis;
  r.a = in->a;
  r.b = in->b;
  r.sigR = in->sigR;
  r.C = in->C;
  r.Phi = in->Phi;
  r.Eold = in->Eold;
  r.Fold = in->Fold;
  return r;
}

}  // namespace

extern "C" {

const char *tr_error_string(int code) {
  switch (code) {
    case TR_OK: return "ok";
    case TR_EINVAL: return "invalid argument or shape";
    case TR_ENOMEM: return "device allocation failed";
    case TR_EHIP: return "HIP runtime call failed";
    case TR_ENOCONV: return "transport iterations did not converge within max_outer";
    case TR_ENAN: return "non-finite temperature or energy density";
  }
  return "unknown error";
}

int tr_destroy(tr_ctx *c) {
  if (!c) return TR_OK;
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  for (auto &g : c->graphs) {
    if (g.first) (void)hipGraphExecDestroy(g.first);
    if (g.next) (void)hipGraphExecDestroy(g.next);
    if (g.rest) (void)hipGraphExecDestroy(g.rest);
    if (g.next1) (void)hipGraphExecDestroy(g.next1);
    if (g.tail) (void)hipGraphExecDestroy(g.tail);
  }
  for (int b = 0; b < TR_NBUCKET; ++b)
    for (int q = 0; q < 2; ++q)
      if (c->ev_sw[b][q]) (void)hipEventDestroy(c->ev_sw[b][q]);
  if (c->gs) (void)hipStreamDestroy(c->gs);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->h_count) (void)hipHostFree(c->h_count);
  if (c->h_ctl_out) (void)hipHostFree(c->h_ctl_out);
  if (c->h_ctl_in) (void)hipHostFree(c->h_ctl_in);
  if (c->a1.h_err) (void)hipHostFree(c->a1.h_err);
  if (c->a1.h_outer) (void)hipHostFree(c->a1.h_outer);
  delete c;
  return TR_OK;
}

int tr_create(tr_ctx **out, const tr_problem *probs, int n_slab, const tr_solver_cfg *cfg) {
  if (!out || !probs || n_slab <= 0 || !cfg) return TR_EINVAL;
  *out = nullptr;
  if (cfg->lmax < 1 || cfg->lmax > TR_MAXOUT || cfg->max_outer < 1 || cfg->max_outer >= TR_MAXOUT ||
      cfg->cycle < 0 || cfg->cycle > 2 || cfg->precision < 0 || cfg->precision > 1)
    return TR_EINVAL;
  const int nlev = probs[0].n_levels;
  if (nlev < 2 || nlev > TR_MAXLEV) return TR_EINVAL;
  int nx_max = 0;
  for (int s = 0; s < n_slab; ++s) {
    const tr_problem &P = probs[s];
    if (P.nx < 2 || P.ng < 1 || P.nmu < 2 || (P.nmu & 1) || P.nmu > 64 || P.n_levels != nlev || !P.level_ng ||
        !P.x_edges || !P.nu_edges || !P.nu_center || !P.mu || !P.w || !P.C_cell)
      return TR_EINVAL;
    if (!(P.dt > 0) || !(P.cv > 0) || !(P.c > 0) || !(P.aR > 0)) return TR_EINVAL;
    if (P.opacity != TR_OPAC_POINT && P.opacity != TR_OPAC_SPECTRAL) return TR_EINVAL;
    if (P.level_ng[0] != P.ng || P.level_ng[nlev - 1] != 1) return TR_EINVAL;
    for (int l = 1; l < nlev; ++l) {
      const int a = P.level_ng[l - 1], b = P.level_ng[l];
      if (b < 1 || a % b) return TR_EINVAL;
    }
    for (int i = 0; i < P.nx; ++i)
      if (!(P.x_edges[i + 1] > P.x_edges[i])) return TR_EINVAL;
    for (int m = 0; m < P.nmu; ++m) {
      if (m > 0 && !(P.mu[m] > P.mu[m - 1])) return TR_EINVAL;
      if (std::fabs(P.mu[m] + P.mu[P.nmu - 1 - m]) > 1e-14) return TR_EINVAL;
    }
    nx_max = std::max(nx_max, P.nx);
  }
  const int rows = nx_max + 2;
  int T = ((rows + TR_LO_K - 1) / TR_LO_K + 63) / 64 * 64;
  if (T > 512) return TR_EINVAL;  // nx <= 2046

  tr_ctx *c = new (std::nothrow) tr_ctx();
  if (!c) return TR_ENOMEM;
  c->nslab = n_slab;
  c->cfg = *cfg;
  c->nlev = nlev;
  c->sched = schedule_for(cfg->cycle, nlev);
  c->grey_threads = ((rows + TR_GREY_K - 1) / TR_GREY_K + 63) / 64 * 64;
  c->hs.resize(n_slab);

  std::vector<double> h_dx, h_C, h_mu, h_w, h_nue, h_nuc;
  for (int s = 0; s < n_slab; ++s) {
    const tr_problem &P = probs[s];
    SlabDev &S = c->hs[s];
    std::memset(&S, 0, sizeof(S));
    S.nx = P.nx;
    S.ng = P.ng;
    S.nmu = P.nmu;
    S.nlev = nlev;
    for (int l = 0; l < nlev; ++l) S.lev_ng[l] = P.level_ng[l];
    S.nchunk = (P.ng + 63) / 64;
    S.opac = P.opacity;
    if (P.opacity == TR_OPAC_SPECTRAL) c->spectral = true;
    S.rtarget = std::max(16, 4096 / n_slab);
    S.cv = P.cv;
    S.dt = P.dt;
    S.c = P.c;
    S.aR = P.aR;
    S.inv_cdt = 1.0 / (P.c * P.dt);
    double wall = 0.0, wmu2all = 0.0;
    for (int m = 0; m < P.nmu; ++m) {
      const double mu = P.mu[m], w = P.w[m];
      wall += w;
      wmu2all += w * mu * mu;
      if (mu > 0) {
        S.wpos += w;
        S.wmupos += w * mu;
        S.wmu2pos += w * mu * mu;
      } else {
        S.wneg += w;
        S.wmuneg += w * mu;
        S.wmu2neg += w * mu * mu;
      }
    }
    S.f_iso = wmu2all / wall;
    S.T_left = P.T_left;
    S.c_iso = S.wmupos / S.wpos;
    S.o_cell = c->n_cell;
    S.o_edge = c->n_edge;
    S.o_I = c->n_I;
    S.o_gi = c->n_gi;
    S.o_ge = c->n_ge;
    S.o_g = c->n_g;
    S.o_g2 = 2 * c->n_g;
    S.o_nu = c->n_nu;
    S.o_mu = c->n_mu;
    S.o_chunk = c->n_chunk;
    S.o_red = c->n_red;
    c->n_cell += P.nx;
    c->n_edge += P.nx + 1;
    c->n_I += (long long)P.ng * P.nmu * P.nx * 2;
    c->n_gi += (long long)P.ng * P.nx;
    c->n_ge += (long long)P.ng * (P.nx + 1);
    c->n_g += P.ng;
    c->n_nu += P.ng + 1;
    c->n_mu += P.nmu;
    c->n_chunk += (long long)S.nchunk * P.nx;
    {
      // chunk records of the largest two-pass restriction between any two levels
      long long worst = 0;
      for (int a = 0; a < nlev; ++a)
        for (int b = a + 1; b < nlev; ++b) {
          const int r = P.level_ng[a] / P.level_ng[b];
          const int cpb = restrict_cpb(r, P.level_ng[b], P.nx + 1, S.rtarget);
          if (!restrict_single(r, P.level_ng[b], P.nx + 1)) worst = std::max(worst, (long long)P.level_ng[b] * cpb);
        }
      c->n_red += worst * (P.nx + 1) * 22;  // up to 22 fields per record
    }
    {
      // stage dS partials: rows per cell of the fused restriction fine -> gm
      // (every intermediate grid: the schedule can change between steps)
      long long worst = 0;
      for (int gm : schedule_for(TR_CYCLE_F, nlev)) {
        const int r = P.level_ng[0] / P.level_ng[gm];
        S.dsnp[gm] = P.level_ng[gm] * restrict_cpb(r, P.level_ng[gm], P.nx + 1, S.rtarget);
        worst = std::max(worst, (long long)S.dsnp[gm]);
      }
      S.o_dsop = c->n_dsop;
      c->n_dsop += worst * P.nx;
    }
    S.o_lpi[0] = S.o_gi;
    S.o_lpe[0] = S.o_ge;
    S.o_lp2[0] = S.o_g2;
    for (int l = 1; l < nlev; ++l) {
      S.o_lpi[l] = c->n_lpi[l];
      S.o_lpe[l] = c->n_lpe[l];
      S.o_lp2[l] = c->n_lp2[l];
      c->n_lpi[l] += (long long)S.lev_ng[l] * P.nx;
      c->n_lpe[l] += (long long)S.lev_ng[l] * (P.nx + 1);
      c->n_lp2[l] += 2LL * S.lev_ng[l];
    }
    S.o_gpi = S.o_lpi[nlev - 1];
    S.o_gpe = S.o_lpe[nlev - 1];
    S.o_gp2 = S.o_lp2[nlev - 1];
    for (int i = 0; i < P.nx; ++i) {
      h_dx.push_back(P.x_edges[i + 1] - P.x_edges[i]);
      h_C.push_back(P.C_cell[i]);
    }
    for (int m = 0; m < P.nmu; ++m) {
      h_mu.push_back(P.mu[m]);
      h_w.push_back(P.w[m]);
    }
    for (int g = 0; g <= P.ng; ++g) h_nue.push_back(P.nu_edges[g]);
    for (int g = 0; g < P.ng; ++g) h_nuc.push_back(P.nu_center[g]);
  }
  int rc = TR_OK;
  auto fail = [&](int code) {
    tr_destroy(c);
    return code;
  };
  {
    const long long ibytes = c->n_I * (cfg->precision == TR_PREC_F32_STORAGE ? 4 : 8);
    c->sweep_nt = 2 * ibytes > TR_LLC_BYTES;
  }

  double *d_dx, *d_C, *d_mu, *d_w, *d_nue, *d_nuc;
  if ((rc = dalloc(c, &d_dx, c->n_cell)) || (rc = dalloc(c, &d_C, c->n_cell)) || (rc = dalloc(c, &d_mu, c->n_mu)) ||
      (rc = dalloc(c, &d_w, c->n_mu)) || (rc = dalloc(c, &d_nue, c->n_nu)) || (rc = dalloc(c, &d_nuc, c->n_g)) ||
      (rc = dalloc(c, &c->d_inc, 2 * c->n_g)) || (rc = dalloc(c, &c->d_sd, n_slab)))
    return fail(rc);
  auto up = [&](void *d, const void *h, size_t bytes) { return hipMemcpy(d, h, bytes, hipMemcpyHostToDevice); };
  if (up(d_dx, h_dx.data(), 8 * h_dx.size()) || up(d_C, h_C.data(), 8 * h_C.size()) ||
      up(d_mu, h_mu.data(), 8 * h_mu.size()) || up(d_w, h_w.data(), 8 * h_w.size()) ||
      up(d_nue, h_nue.data(), 8 * h_nue.size()) || up(d_nuc, h_nuc.data(), 8 * h_nuc.size()) ||
      up(c->d_sd, c->hs.data(), sizeof(SlabDev) * n_slab))
    return fail(TR_EHIP);
  c->pd.dx = d_dx;
  c->pd.Ccell = d_C;
  c->pd.mu = d_mu;
  c->pd.w = d_w;
  c->pd.nu_e = d_nue;
  c->pd.nu_c = d_nuc;
  c->pd.inc = c->d_inc;

  // workspace
  if ((rc = dalloc(c, &c->kappa, c->n_gi)) || (rc = dalloc(c, &c->B, c->n_gi)) ||
      (rc = dalloc(c, &c->dSpart, c->n_chunk)) || (rc = dalloc(c, &c->mom, 4 * c->n_gi)) ||
      (rc = dalloc(c, &c->bnd, 6 * c->n_g)) || (rc = dalloc(c, &c->Phi, 2 * c->n_g)) ||
      (rc = dalloc(c, &c->Eold, c->n_gi)) || (rc = dalloc(c, &c->Fold, c->n_ge)) || (rc = dalloc(c, &c->red, c->n_red)) || (rc = dalloc(c, &c->dsop, c->n_dsop)))
    return fail(rc);
  // sigma_R of spectral slabs has a table of its own; under the point law it
  // is the kappa table (same addresses, no extra traffic)
  if (c->spectral) {
    if ((rc = dalloc(c, &c->sigR, c->n_gi))) return fail(rc);
  } else {
    c->sigR = c->kappa;
  }
  double **cells[] = {&c->dS, &c->Told, &c->Ts, &c->Tcyc, &c->Tstar, &c->Tprev, &c->sigprev, &c->Ecyc, &c->Es};
  for (double **p : cells)
    if ((rc = dalloc(c, p, c->n_cell))) return fail(rc);
  for (int l = 1; l < nlev; ++l) {
    auto &L = c->lev[l];
    double **pi[] = {&L.sigE, &L.emis, &L.Eold, &L.E, &L.Esum};
    double **pe[] = {&L.a, &L.b, &L.sigR, &L.Fold, &L.F};
    double **p2[] = {&L.C, &L.Phi, &L.Ebnd};
    for (double **p : pi)
      if ((rc = dalloc(c, p, c->n_lpi[l]))) return fail(rc);
    for (double **p : pe)
      if ((rc = dalloc(c, p, c->n_lpe[l]))) return fail(rc);
    for (double **p : p2)
      if ((rc = dalloc(c, p, c->n_lp2[l]))) return fail(rc);
  }
  if ((rc = dalloc(c, &c->d_ctl, n_slab)) || (rc = dalloc(c, &c->d_serial, 1)))
    return fail(rc);
  if (hipMemset(c->d_serial, 0, sizeof(int)) != hipSuccess) return fail(TR_EHIP);
  // the active-slab count is written by the GPU straight into coherent pinned
  // host memory (read after the synchronisation of every transport iteration)
  if (hipHostMalloc((void **)&c->h_count, 3 * sizeof(int), hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void **)&c->h_ctl_out, sizeof(Ctl) * n_slab, hipHostMallocCoherent) != hipSuccess ||
      hipHostMalloc((void **)&c->h_ctl_in, sizeof(Ctl) * n_slab, hipHostMallocCoherent) != hipSuccess)
    return fail(TR_ENOMEM);
  c->h_count[0] = c->h_count[1] = c->h_count[2] = 0;
  if (hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking) != hipSuccess) return fail(TR_EHIP);
  for (int b = 0; b < TR_NBUCKET; ++b)
    for (int q = 0; q < 2; ++q)
      if (timing_event(&c->ev_sw[b][q]) != hipSuccess) return fail(TR_EHIP);

  // work tables
  {
    // small tables: one group per opacity thread (shortest chains); large
    // ones: runs of 4 groups sharing their edge integrals
    c->opac_run = c->n_gi <= (1LL << 21) ? 1 : 4;
    std::vector<Item> opac, dsum, cell, gi, g, grey;
    std::vector<std::vector<std::pair<long long, Item>>> sweepb(TR_NBUCKET);
    std::vector<std::vector<Item>> lo[4];
    for (int kb = 0; kb < 4; ++kb) lo[kb].resize(nlev);
    for (int s = 0; s < n_slab; ++s) {
      const SlabDev &S = c->hs[s];
      const int ncb = (S.nx + 4 * c->opac_run - 1) / (4 * c->opac_run);
      for (int q = 0; q < S.nchunk * ncb; ++q) opac.push_back({s, q});
      for (int st = 0; st < S.nx; st += 64) dsum.push_back({s, st});
      for (int st = 0; st < S.nx; st += 256) cell.push_back({s, st});
      const long long cost = (long long)S.nx * S.nmu;
      for (int gg = 0; gg < S.ng; ++gg) sweepb[sweep_bucket(S.nx)].push_back({cost, Item{s, gg}});
      for (long long st = 0; st < (long long)S.ng * S.nx; st += 256) gi.push_back({s, (int)st});
      for (int st = 0; st < S.ng; st += 256) g.push_back({s, st});
      grey.push_back({s, 0});
      for (int l = 0; l < nlev; ++l)
        for (int p = 0; p < S.lev_ng[l]; ++p) lo[lo_block(S.nx)][l].push_back({s, p});
    }
    if ((rc = upload_table(c, opac, c->t_opac)) || (rc = upload_table(c, dsum, c->t_dS)) ||
        (rc = upload_table(c, cell, c->t_cell)) ||
        (rc = upload_table(c, gi, c->t_gi)) ||
        (rc = upload_table(c, g, c->t_g)) || (rc = upload_table(c, grey, c->t_grey)))
      return fail(rc);
    for (int l = 0; l < nlev; ++l)
      for (int kb = 0; kb < 4; ++kb)
        if ((rc = upload_table(c, lo[kb][l], c->t_lo[kb][l]))) return fail(rc);
    for (int b = 0; b < TR_NBUCKET; ++b) {
      // longest-processing-time order: the most expensive slabs start first
      auto &v = sweepb[b];
      std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
      std::vector<Item> items;
      for (auto &e : v) items.push_back(e.second);
      if ((rc = upload_table(c, items, c->t_sweep_b[b]))) return fail(rc);
    }
    if ((rc = build_restrict_tables(c, 0, nlev - 1))) return fail(rc);
    for (int gsched : schedule_for(TR_CYCLE_F, nlev)) {
      if ((rc = build_restrict_tables(c, 0, gsched)) || (rc = build_restrict_tables(c, 0, gsched, 1)) ||
          (rc = build_restrict_tables(c, gsched, nlev - 1)))
        return fail(rc);
    }
  }

  // incoming Planck radiation at T_left / T_right: B table of a one-cell
  // evaluation per slab through the opacity kernel would need a second
  // layout, so evaluate the same device routine on a scratch pooled table.
  c->h_inc.assign(2 * c->n_g, 0.0);
  {
    // temperature per cell: left boundary temperature in even passes
    std::vector<double> Tb(c->n_cell);
    for (int side = 0; side < 2; ++side) {
      for (int s = 0; s < n_slab; ++s) {
        const double Tv = side == 0 ? probs[s].T_left : probs[s].T_right;
        for (int i = 0; i < c->hs[s].nx; ++i) Tb[c->hs[s].o_cell + i] = Tv > 0 ? Tv : 1.0;
      }
      if (up(c->Told, Tb.data(), 8 * Tb.size())) return fail(TR_EHIP);
      LaunchEnv env = env_of(c, 0);
      launch_opacity(env, c->t_opac, c->opac_run, nullptr, PRED_ALL, 0, c->Told, c->kappa, c->B, c->dSpart);
      if (hipDeviceSynchronize() != hipSuccess) return fail(TR_EHIP);
      std::vector<double> hB(c->n_gi);
      if (hipMemcpy(hB.data(), c->B, 8 * hB.size(), hipMemcpyDeviceToHost) != hipSuccess) return fail(TR_EHIP);
      for (int s = 0; s < n_slab; ++s) {
        const SlabDev &S = c->hs[s];
        const double Tv = side == 0 ? probs[s].T_left : probs[s].T_right;
        for (int gg = 0; gg < S.ng; ++gg)
          c->h_inc[2 * S.o_g + side * S.ng + gg] = Tv > 0 ? hB[S.o_gi + (long long)gg * S.nx] : 0.0;
      }
    }
    if (up(c->d_inc, c->h_inc.data(), 8 * c->h_inc.size())) return fail(TR_EHIP);
  }
  *out = c;
  return TR_OK;
}

int tr_layout(const tr_ctx *c, int kind, int slab, long long *offset, long long *total) {
  if (!c || slab < 0 || slab >= c->nslab) return TR_EINVAL;
  const SlabDev &S = c->hs[slab];
  long long o = 0, t = 0;
  if (kind >= TR_K_LEV_P2 && kind < TR_K_LEV_P2 + c->nlev) {
    const int l = kind - TR_K_LEV_P2;
    o = S.o_lp2[l];
    t = l == 0 ? 2 * c->n_g : c->n_lp2[l];
  } else if (kind >= TR_K_LEV_PE && kind < TR_K_LEV_PE + c->nlev) {
    const int l = kind - TR_K_LEV_PE;
    o = S.o_lpe[l];
    t = l == 0 ? c->n_ge : c->n_lpe[l];
  } else if (kind >= TR_K_LEV_PI && kind < TR_K_LEV_PI + c->nlev) {
    const int l = kind - TR_K_LEV_PI;
    o = S.o_lpi[l];
    t = l == 0 ? c->n_gi : c->n_lpi[l];
  } else {
    switch (kind) {
      case TR_K_CELL: o = S.o_cell; t = c->n_cell; break;
      case TR_K_EDGE: o = S.o_edge; t = c->n_edge; break;
      case TR_K_I: o = S.o_I; t = c->n_I; break;
      case TR_K_GI: o = S.o_gi; t = c->n_gi; break;
      case TR_K_GE: o = S.o_ge; t = c->n_ge; break;
      case TR_K_G2: o = S.o_g2; t = 2 * c->n_g; break;
      case TR_K_G: o = S.o_g; t = c->n_g; break;
      default: return TR_EINVAL;
    }
  }
  if (offset) *offset = o;
  if (total) *total = t;
  return TR_OK;
}

int tr_set_incoming(tr_ctx *c, int slab, const double *inc_left, const double *inc_right) {
  if (!c || slab < 0 || slab >= c->nslab) return TR_EINVAL;
  const SlabDev &S = c->hs[slab];
  if (inc_left)
    for (int g = 0; g < S.ng; ++g) c->h_inc[2 * S.o_g + g] = inc_left[g];
  if (inc_right)
    for (int g = 0; g < S.ng; ++g) c->h_inc[2 * S.o_g + S.ng + g] = inc_right[g];
  return hip_err(hipMemcpy(c->d_inc, c->h_inc.data(), 8 * c->h_inc.size(), hipMemcpyHostToDevice));
}

int tr_opacity(tr_ctx *c, const double *T, const double *Egrey, double *kappa, double *B, double *sigR, double *dS,
               hipStream_t st) {
  if (!c || !T || !kappa || !B || (c->spectral && !sigR)) return TR_EINVAL;
  LaunchEnv env = env_of(c, st);
  launch_opacity(env, c->t_opac, c->opac_run, nullptr, PRED_ALL, 0, T, kappa, B, c->dSpart, c->spectral, Egrey,
                 sigR);
  if (dS) launch_dS_sum(env, c->t_dS, nullptr, PRED_ALL, 0, c->dSpart, dS);
  return hip_err(hipGetLastError());
}

int tr_sweep(tr_ctx *c, const double *kappa, const double *B, const double *I_prev, double *I_out, double *mom,
             double *bnd, hipStream_t st) {
  if (!c || !kappa || !B || !I_prev || !I_out || !mom || !bnd || I_prev == I_out) return TR_EINVAL;
  launch_sweeps(c, env_of(c, st), nullptr, PRED_ALL, kappa, B, I_prev, I_out, mom, bnd);
  return hip_err(hipGetLastError());
}

int tr_moments(tr_ctx *c, const double *mom, const double *bnd, double *f, double *fbnd, double *C, double *Phi,
               hipStream_t st) {
  if (!c || !mom || !bnd || !f || !fbnd || !C || !Phi) return TR_EINVAL;
  launch_moments(env_of(c, st), c->t_gi, nullptr, PRED_ALL, 0, mom, bnd, f, fbnd, C, Phi);
  return hip_err(hipGetLastError());
}

int tr_lo_solve(tr_ctx *c, int level, const tr_lo_coeffs *in, const tr_lo_fields *out, hipStream_t st) {
  if (!c || !in || !out || level < 0 || level >= c->nlev || !out->E || !out->F || !out->Ebnd) return TR_EINVAL;
  if (level == 0 && (!in->kappa || !in->B || !in->f || !in->fbnd)) return TR_EINVAL;
  if (level > 0 && (!in->sigE || !in->emis || !in->a || !in->b || !in->sigR)) return TR_EINVAL;
  if (!in->C || !in->Phi || !in->Eold || !in->Fold) return TR_EINVAL;
  LoSol sol{out->E, out->F, out->Ebnd};
  launch_lo_all(c, env_of(c, st), nullptr, PRED_ALL, 0, level, coeffs_in(in), sol);
  return hip_err(hipGetLastError());
}

int tr_restrict(tr_ctx *c, int from, int to, const tr_lo_coeffs *in, const tr_lo_fields *sol, const tr_lo_out *out,
                hipStream_t st) {
  if (!c || !in || !sol || !out || from < 0 || to <= from || to >= c->nlev) return TR_EINVAL;
  for (int s = 0; s < c->nslab; ++s) {
    const SlabDev &S = c->hs[s];
    if (S.lev_ng[from] % S.lev_ng[to]) return TR_EINVAL;
  }
  int rc = build_restrict_tables(c, from, to);
  if (rc) return rc;
  LoSol s{sol->E, sol->F, sol->Ebnd};
  LoOut o{out->sigE, out->emis, out->a, out->b, out->sigR, out->C, out->Phi, out->Eold, out->Fold, out->Esum,
          nullptr, nullptr};
  launch_restrict(env_of(c, st), c->t_red[std::make_pair(from, to)], nullptr, PRED_ALL, 0, from, to, coeffs_in(in), s,
                  o, c->red, true);
  return hip_err(hipGetLastError());
}

int tr_grey_solve(tr_ctx *c, const tr_lo_coeffs *grey, const double *Tstar, const double *Told, const double *dS,
                  const double *Estar, const double *D, double *T_out, const tr_lo_fields *out, hipStream_t st) {
  if (!c || !grey || !Tstar || !Told || !dS || !Estar || !D || !T_out || !out) return TR_EINVAL;
  GreyArgs ga{};
  ga.grey = coeffs_in(grey);
  ga.Estar = Estar;
  ga.sol = LoSol{out->E, out->F, out->Ebnd};
  ga.Tstar = Tstar;
  ga.Tout = T_out;
  ga.Told = Told;
  ga.dS = dS;
  ga.D = D;
  ga.ctl_dummy = c->d_ctl;
  launch_grey(env_of(c, st), c->t_grey, c->grey_threads, nullptr, PRED_ALL, 0, ga);
  return hip_err(hipGetLastError());
}

int tr_set_tiles(tr_ctx *c, const int *K, const int *split) {
  if (!c || !K) return TR_EINVAL;
  for (int b = 0; b < TR_NBUCKET; ++b) {
    if (K[b] != 1 && K[b] != 2 && K[b] != 4 && K[b] != 8) return TR_EINVAL;
    if (split && split[b] != 1 && split[b] != 2 && split[b] != 4) return TR_EINVAL;
  }
  for (int b = 0; b < TR_NBUCKET; ++b) {
    c->sweep_K[b] = K[b];
    c->sweep_S[b] = split ? split[b] : 1;
  }
  // captured launch sequences hold the old tiles
  for (auto &g : c->graphs) {
    if (g.first) (void)hipGraphExecDestroy(g.first);
    if (g.next) (void)hipGraphExecDestroy(g.next);
    if (g.rest) (void)hipGraphExecDestroy(g.rest);
    if (g.next1) (void)hipGraphExecDestroy(g.next1);
    if (g.tail) (void)hipGraphExecDestroy(g.tail);
  }
  c->graphs.clear();
  return TR_OK;
}

int tr_get_tiles(const tr_ctx *c, int *K, int *split, int *items) {
  if (!c || !K) return TR_EINVAL;
  for (int b = 0; b < TR_NBUCKET; ++b) {
    K[b] = c->sweep_K[b];
    if (split) split[b] = c->sweep_S[b];
    if (items) items[b] = c->t_sweep_b[b].n;
  }
  return TR_OK;
}

int tr_autotune(tr_ctx *c, const double *I_prev, double *I_out, int reps, int *K_out, int *split_out,
                double *us_out, hipStream_t st) {
  if (!c || !I_prev || !I_out || I_prev == I_out || reps < 1) return TR_EINVAL;
  static const int candK[4] = {1, 2, 4, 8}, candS[3] = {1, 2, 4};
  hipEvent_t e0, e1;
  if (timing_event(&e0) != hipSuccess || timing_event(&e1) != hipSuccess) return TR_EHIP;
  LaunchEnv env = env_of(c, st);
  const bool f32 = c->cfg.precision == TR_PREC_F32_STORAGE;
  int K[TR_NBUCKET], Sp[TR_NBUCKET];
  int rc = TR_OK;
  for (int b = 0; b < TR_NBUCKET && !rc; ++b) {
    K[b] = c->sweep_K[b];
    Sp[b] = c->sweep_S[b];
    if (c->t_sweep_b[b].n == 0) {
      if (us_out)
        for (int q = 0; q < 12; ++q) us_out[12 * b + q] = 0.0;
      continue;
    }
    double best = 1e300;
    for (int q = 0; q < 12 && !rc; ++q) {
      const int kk = candK[q / 3], ss = candS[q % 3];
      launch_sweep(env, c->t_sweep_b[b], kk, ss, f32, c->sweep_nt, nullptr, PRED_ALL, 0, c->kappa, c->B, I_prev, I_out,
                   c->mom, c->bnd);
      if (hipEventRecord(e0, st) != hipSuccess) rc = TR_EHIP;
      for (int r = 0; r < reps; ++r)
        launch_sweep(env, c->t_sweep_b[b], kk, ss, f32, c->sweep_nt, nullptr, PRED_ALL, 0, c->kappa, c->B, I_prev,
                     I_out, c->mom, c->bnd);
      float ms = 0.f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = TR_EHIP;
      // a tile whose launch was refused (resources) is not a candidate
      const bool launched = hipGetLastError() == hipSuccess;
      const double us = launched ? 1e3 * ms / reps : 0.0;
      if (us_out) us_out[12 * b + q] = us;
      if (launched && us < best) {
        best = us;
        K[b] = kk;
        Sp[b] = ss;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (K_out)
    for (int b = 0; b < TR_NBUCKET; ++b) K_out[b] = K[b];
  if (split_out)
    for (int b = 0; b < TR_NBUCKET; ++b) split_out[b] = Sp[b];
  return tr_set_tiles(c, K, Sp);
}

int tr_mlp_features(tr_ctx *c, const double *T, const double *T_prev, const double *kappa, const double *f,
                    const float *mean, const float *std, float *X, hipStream_t st) {
  if (!c || !T || !kappa || !f || !mean || !std || !X) return TR_EINVAL;
  MlpStats ms;
  for (int k = 0; k < TR_MLP_NFEAT; ++k) {
    ms.mean[k] = mean[k];
    ms.std[k] = std[k];
    if (!(std[k] > 0)) return TR_EINVAL;
  }
  launch_mlp_features(env_of(c, st), c->t_gi, T, T_prev, kappa, f, ms, X);
  return hip_err(hipGetLastError());
}

int tr_closure_targets(tr_ctx *c, const double *f, const double *f_prev, const double *E_new, const double *E_prev,
                       int block, float *Y, hipStream_t st) {
  if (!c || !f || !f_prev || !E_new || !E_prev || !Y || block < 1) return TR_EINVAL;
  launch_closure_targets(env_of(c, st), c->t_gi, f, f_prev, E_new, E_prev, block, Y);
  return hip_err(hipGetLastError());
}

int tr_prolong(tr_ctx *c, int level, const double *E_coarse, const double *E_prev, const float *r, double *E_fine,
               hipStream_t st) {
  if (!c || level < 1 || level >= c->nlev || !E_coarse || !E_prev || !E_fine || E_prev == E_fine) return TR_EINVAL;
  if (!c->t_pro.count(level)) {
    std::vector<Item> items;
    for (int s = 0; s < c->nslab; ++s) {
      const SlabDev &S = c->hs[s];
      if (S.ng % S.lev_ng[level]) return TR_EINVAL;
      for (int q = 0; q < S.lev_ng[level] * S.nx; q += 256) items.push_back({s, q});
    }
    Table t{};
    const int rc = upload_table(c, items, t);
    if (rc) return rc;
    c->t_pro[level] = t;
  }
  launch_prolong(env_of(c, st), c->t_pro[level], level, E_coarse, E_prev, r, E_fine);
  return hip_err(hipGetLastError());
}

int tr_set_closure(tr_ctx *c, const float *params, const float *mean, const float *std) {
  if (!c) return TR_EINVAL;
  if (!params) {
    c->mlp_params = nullptr;
    return TR_OK;
  }
  if (!mean || !std) return TR_EINVAL;
  for (int k = 0; k < TR_MLP_NFEAT; ++k) {
    if (!(std[k] > 0)) return TR_EINVAL;
    c->mlp_stats.mean[k] = mean[k];
    c->mlp_stats.std[k] = std[k];
  }
  if (!c->d_seed_counts) {
    int rc;
    if ((rc = dalloc(c, &c->d_seed_counts, 2)) || (rc = dalloc(c, &c->T_hist, c->n_cell))) return rc;
  }
  c->mlp_params = params;
  return TR_OK;
}

int tr_closure_seed(tr_ctx *c, const double *T, const double *T_prev, const double *kappa, double *f,
                    unsigned long long *counts, hipStream_t st) {
  if (!c || !c->mlp_params || !T || !kappa || !f || !counts) return TR_EINVAL;
  launch_closure_seed(env_of(c, st), c->t_gi, T, T_prev, kappa, f, c->mlp_stats, c->mlp_params, counts);
  return hip_err(hipGetLastError());
}

int tr_state_init(tr_ctx *c, const tr_state *s, double T0, hipStream_t st) {
  if (!c || !s || !s->T || !s->I_out || !s->E || !s->F || !s->Ebnd || !s->f || !s->fbnd || !s->C || !s->Egrey ||
      !(T0 > 0))
    return TR_EINVAL;
  c->have_hist = 0;  // a new run: no temperature history for the closure
  LaunchEnv env = env_of(c, st);
  launch_fill(env, s->T, T0, c->n_cell);
  launch_opacity(env, c->t_opac, c->opac_run, nullptr, PRED_ALL, 0, s->T, c->kappa, c->B, c->dSpart);
  launch_init_state(env, c->t_gi, c->cfg.precision == TR_PREC_F32_STORAGE, c->B, s->I_out, s->E, s->F, s->Ebnd,
                    c->mom, c->bnd);
  launch_moments(env, c->t_gi, nullptr, PRED_ALL, 0, c->mom, c->bnd, s->f, s->fbnd, s->C, c->Phi);
  launch_group_sum(env, c->t_cell, s->E, s->Egrey);
  return hip_err(hipGetLastError());
}

}  // extern "C"

namespace {

// One transport iteration: (sweep + moments when with_sweep), the predicated
// cycles l in [lbeg, lend) (default all Lmax; a slab whose inner loop has
// finished skips the rest), the start of the next iteration and the
// active-slab count.  With sweep_outside the sweep launches are left to the
// caller (timed launches).
void enqueue_iteration(tr_ctx *c, const tr_state *s, hipStream_t st, int Lmax, bool with_sweep,
                       bool sweep_outside, int lbeg = 0, int lend = -1) {
  if (lend < 0) lend = Lmax;
  const int ns = c->nslab, gl = c->nlev - 1;
  LaunchEnv env = env_of(c, st);
  const LoIn fine = fine_in(c, c->kappa, c->B, s->f, s->fbnd, s->C, c->Phi, c->Eold, c->Fold);
  const LoSol fsol{s->E, s->F, s->Ebnd};
  GreyArgs ga{};
  ga.grey = level_in(c, gl);
  ga.Estar = c->lev[gl].Esum;
  ga.sol = level_sol(c, gl);
  ga.Tstar = c->Tstar;
  ga.Tout = c->Tstar;
  ga.Told = c->Told;
  ga.dS = c->dS;
  ga.Tprev = c->Tprev;
  ga.sigprev = c->sigprev;
  ga.Egrey = s->Egrey;
  ga.Tcyc = c->Tcyc;
  ga.Ecyc = c->Ecyc;
  ga.Ts = c->Ts;
  ga.Es = c->Es;
  ga.ctl_dummy = c->d_ctl;
  ga.stage_mask = 0;
  for (int gm : c->sched) ga.stage_mask |= 1 << gm;
  ga.secant = c->cfg.secant;
  ga.lmax = c->cfg.lmax;
  ga.eps = c->cfg.eps;
  ga.eps_inner = c->cfg.eps_inner;
  const int nsch = (int)c->sched.size();
  if (with_sweep && !sweep_outside)
    launch_sweeps(c, env, c->d_ctl, PRED_SWEEP, c->kappa, c->B, s->I_prev, s->I_out, c->mom, c->bnd);
  // after a sweep the first fine solve forms the QD factors from the sweep's
  // partials (its slabs are exactly those that swept: every slab leaves the
  // s = 0 iteration at s >= 1, and an iteration with a sweep starts at cycle 0)
  LoIn fine0 = fine;
  if (with_sweep) {
    fine0.mom = c->mom;
    fine0.bnd = c->bnd;
    fine0.f_out = s->f;
    fine0.fbnd_out = s->fbnd;
    fine0.C_out = s->C;
    fine0.Phi_out = c->Phi;
  }
  for (int l = lbeg; l < lend; ++l) {
    // old-time sums are constant during the step: restricted in its first
    // cycle only (every slab runs cycle 0 of iteration s = 0)
    const bool old = !with_sweep && l == 0;
    {
      TimedScope ts(c, st, TR_T_LO_FINE, l);
      launch_lo_all(c, env, c->d_ctl, PRED_CYCLE, l, 0, l == 0 ? fine0 : fine, fsol);
    }
    {
      TimedScope ts(c, st, TR_T_RESTRICT, l);
      launch_restrict(env, c->t_red[std::make_pair(0, gl)], c->d_ctl, PRED_CYCLE, l, 0, gl, fine, fsol,
                      grey_out(c), c->red, old);
    }
    ga.end_cycle = nsch == 0;
    {
      TimedScope ts(c, st, TR_T_GREY, l);
      launch_grey(env, c->t_grey, c->grey_threads, c->d_ctl, PRED_CYCLE, l, ga);
    }
    for (int q = 0; q < nsch; ++q) {
      const int gm = c->sched[q];
      if (c->spectral) {
        // group averages at the stage temperature and the radiation
        // temperature of the grey E just solved, into the tables (the fine
        // solve of this cycle is done with them; the end of the cycle
        // evaluates them again at its final T), then the plain restriction;
        // the stage-to-grey restriction reduces dS from the tables' partials
        {
          TimedScope ts(c, st, TR_T_OPACITY, l);
          launch_opacity(env, c->t_opac, c->opac_run, c->d_ctl, PRED_CYCLE, l, c->Tstar, c->kappa, c->B, c->dSpart,
                         true, s->Egrey, c->sigR);
        }
        {
          TimedScope ts(c, st, TR_T_RESTRICT, l);
          launch_restrict(env, c->t_red[std::make_pair(0, gm)], c->d_ctl, PRED_CYCLE, l, 0, gm, fine, fsol,
                          level_out(c, gm), c->red, old);
        }
        {
          TimedScope ts(c, st, TR_T_LO_COARSE, l);
          launch_lo_all(c, env, c->d_ctl, PRED_CYCLE, l, gm, level_in(c, gm), level_sol(c, gm));
        }
        {
          TimedScope ts(c, st, TR_T_RESTRICT, l);
          launch_restrict(env, c->t_red[std::make_pair(gm, gl)], c->d_ctl, PRED_CYCLE, l, gm, gl, level_in(c, gm),
                          level_sol(c, gm), grey_out(c), c->red, old);
        }
      } else {
      {
        // the stage's kappa, B at T* are evaluated inside the restriction
        // (not written to the tables), with the stage dS partials
        TimedScope ts(c, st, TR_T_RESTRICT, l);
        launch_restrict(env, c->t_red_op[gm], c->d_ctl, PRED_CYCLE, l, 0, gm, fine, fsol, level_out(c, gm), c->red,
                        old, 1, c->Tstar, c->dsop);
      }
      {
        TimedScope ts(c, st, TR_T_LO_COARSE, l);
        launch_lo_all(c, env, c->d_ctl, PRED_CYCLE, l, gm, level_in(c, gm), level_sol(c, gm));
      }
      {
        TimedScope ts(c, st, TR_T_RESTRICT, l);
        launch_restrict(env, c->t_red[std::make_pair(gm, gl)], c->d_ctl, PRED_CYCLE, l, gm, gl, level_in(c, gm),
                        level_sol(c, gm), grey_out(c), c->red, old, 2, nullptr, c->dsop);
      }
      }
      ga.end_cycle = q == nsch - 1;
      {
        TimedScope ts(c, st, TR_T_GREY, l);
        launch_grey(env, c->t_grey, c->grey_threads, c->d_ctl, PRED_CYCLE, l, ga);
      }
    }
    {
      TimedScope ts(c, st, TR_T_OPACITY, l);
      launch_opacity(env, c->t_opac, c->opac_run, c->d_ctl, PRED_DONECYC, l + 1, c->Tstar, c->kappa, c->B, c->dSpart,
                     c->spectral, s->Egrey, c->sigR);
    }
  }
  // start of the next transport iteration (s + 1) for slabs still iterating
  launch_outer_end(env, c->d_ctl, ns, c->cfg.max_outer, c->h_count, c->h_ctl_out, c->d_serial);
}

int capture_iteration(tr_ctx *c, const tr_state *s, int Lmax, bool with_sweep, bool sweep_outside,
                      hipGraphExec_t *out, int lbeg = 0, int lend = -1) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->gs, hipStreamCaptureModeThreadLocal) != hipSuccess) return TR_EHIP;
  enqueue_iteration(c, s, c->gs, Lmax, with_sweep, sweep_outside, lbeg, lend);
  if (hipStreamEndCapture(c->gs, &g) != hipSuccess || !g) return TR_EHIP;
  const hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e == hipSuccess ? TR_OK : TR_EHIP;
}


}  // namespace

extern "C" {

int tr_set_schedule(tr_ctx *c, int cycle, int lmax) {
  if (!c || cycle < 0 || cycle > 2 || lmax < 1 || lmax > TR_MAXOUT) return TR_EINVAL;
  c->cfg.cycle = cycle;
  c->cfg.lmax = lmax;
  c->sched = schedule_for(cycle, c->nlev);
  return TR_OK;
}

int tr_set_grids(tr_ctx *c, int n, const int *grids, int lmax) {
  if (!c || n < 0 || n > c->nlev - 2 || (n > 0 && !grids) || lmax < 1 || lmax > TR_MAXOUT) return TR_EINVAL;
  std::vector<int> sched;
  for (int q = 0; q < n; ++q) {
    const int gm = grids[q];
    if (gm < 1 || gm > c->nlev - 2) return TR_EINVAL;
    for (int p : sched)
      if (p == gm) return TR_EINVAL;
    sched.push_back(gm);
  }
  c->sched = sched;
  c->cfg.cycle = n == 0 ? TR_CYCLE_V : n == 1 ? TR_CYCLE_W : TR_CYCLE_F;
  c->cfg.lmax = lmax;
  return TR_OK;
}

int tr_set_sweep_timing(tr_ctx *c, int on) {
  if (!c || (on != 0 && on != 1)) return TR_EINVAL;
  c->sweep_events = on;
  return TR_OK;
}

}  // extern "C"

namespace {

int step_impl(tr_ctx *c, const tr_state *s, const int *replay, tr_stats *stats, hipStream_t st) {
  if (!c || !s || !s->T || !s->I_prev || !s->I_out || s->I_prev == s->I_out || !s->E || !s->F || !s->Ebnd ||
      !s->f || !s->fbnd || !s->C || !s->Egrey)
    return TR_EINVAL;
  const int ns = c->nslab;
  // control records
  std::vector<Ctl> hc(ns);
  int Lmax = c->cfg.lmax;
  for (int q = 0; q < ns; ++q) {
    Ctl &k = hc[q];
    std::memset(&k, 0, sizeof(Ctl));
    k.active = 1;
    if (replay) {
      const int *row = replay + (size_t)q * TR_MAXOUT;
      if (row[0] < 0) return TR_EINVAL;
      int n = 0;
      while (n < TR_MAXOUT && row[n] > 0) {
        k.replay[n] = row[n];
        Lmax = std::max(Lmax, row[n]);
        ++n;
      }
      k.n_replay = n;  // 0: this slab runs its own convergence tests
    }
  }
  // everything runs on the caller's stream (graphs are captured on the
  // library's own stream and replayed here), so no ordering between streams
  hipStream_t gs = st;
  // (coherent pinned memory, read by the step-start kernel; the previous
  // step has finished with the buffer)
  static_assert(sizeof(Ctl) % sizeof(int) == 0, "control records are copied as ints");
  std::memcpy(c->h_ctl_in, hc.data(), sizeof(Ctl) * ns);
  LaunchEnv env = env_of(c, gs);
  // step start: control records, old-time copies, convergence references,
  // Phi with the current incoming, the opacity tables at T
  launch_step_start(env, s->T, s->Egrey, s->E, s->F, c->n_cell, c->n_gi, c->n_ge, c->Told, c->Ts, c->Tcyc, c->Tstar,
                    c->Es, c->Ecyc, c->Eold, c->Fold, c->h_ctl_in, c->d_ctl, ns, c->t_g, s->C, c->Phi, c->t_opac,
                    c->opac_run, c->kappa, c->B, c->dSpart, c->spectral, c->sigR);
  unsigned long long seed_counts[2] = {0, 0};
  if (c->mlp_params) {
    // learned closure: predicted cell factors replace the previous step's
    if (hipMemsetAsync(c->d_seed_counts, 0, 2 * sizeof(unsigned long long), gs) != hipSuccess) return TR_EHIP;
    // inputs at the step start: T^{j-1}, the previous step's T (after a
    // first closure step), the current factors; inputs, network and seeding
    // in one kernel
    launch_closure_seed(env, c->t_gi, c->Tstar, c->have_hist ? c->T_hist : nullptr, c->kappa, s->f, c->mlp_stats,
                        c->mlp_params, c->d_seed_counts);
    launch_copy(env, c->Tstar, c->T_hist, c->n_cell);
    c->have_hist = 1;
  }

  // graphs for this state (ping-pong buffers give two keys per run)
  tr_ctx::GraphEntry *ge = nullptr;
  if (!c->cfg.timing) {
    std::vector<const void *> key = {s->I_prev, s->I_out, s->E, s->F, s->Ebnd, s->f, s->fbnd, s->C, s->Egrey,
                                     reinterpret_cast<const void *>((intptr_t)Lmax),
                                     reinterpret_cast<const void *>((intptr_t)c->cfg.lmax),
                                     reinterpret_cast<const void *>((intptr_t)c->cfg.cycle)};
    // the grids visited after each grey solve, in order (tr_set_grids)
    for (int gm : c->sched) key.push_back(reinterpret_cast<const void *>((intptr_t)(1000 + gm)));
    for (auto &g : c->graphs)
      if (g.key == key) ge = &g;
    if (!ge) {
      if (c->graphs.size() >= TR_GRAPH_CACHE) {
        auto &old = c->graphs.front();
        (void)hipGraphExecDestroy(old.first);
        (void)hipGraphExecDestroy(old.next);
        if (old.rest) (void)hipGraphExecDestroy(old.rest);
        if (old.next1) (void)hipGraphExecDestroy(old.next1);
        if (old.tail) (void)hipGraphExecDestroy(old.tail);
        c->graphs.erase(c->graphs.begin());
      }
      tr_ctx::GraphEntry e;
      e.key = key;
      // capture needs the stream idle of earlier uncaptured work ordering; the
      // step-start work above is already enqueued and stays before replays
      int rc = capture_iteration(c, s, Lmax, false, false, &e.first);
      if (!rc) rc = capture_iteration(c, s, Lmax, true, false, &e.next);
      if (!rc && Lmax > 1) rc = capture_iteration(c, s, Lmax, true, false, &e.next1, 0, 1);
      if (!rc && Lmax > 1) rc = capture_iteration(c, s, Lmax, false, false, &e.tail, 1, Lmax);
      if (rc) return rc;
      c->graphs.push_back(e);
      ge = &c->graphs.back();
    }
    if (c->sweep_events && !ge->rest) {
      const int rc = capture_iteration(c, s, Lmax, true, true, &ge->rest);
      if (rc) return rc;
    }
  }
  // sweeps launched outside the graphs with their start / end events
  const bool sweep_ev = c->cfg.timing || c->sweep_events;
  double t_ms[TR_T_N] = {0};
  long long n_launch[TR_T_N] = {0};
  c->groups.clear();
  c->ev_used = 0;
  int s0 = 0;  // transport iteration of slab 0 (event timing mode)
  // graph replay without timed sweeps: the iterations the previous step needed
  // are launched back to back (one host synchronisation for all of them);
  // iterations past convergence are predicated off on the device
  const int chain = (ge && !sweep_ev) ? std::min(c->last_iters, c->cfg.max_outer + 2) : 0;
  bool done = false;  // every slab stopped (seen on the host)
  volatile const int *hc_active = c->h_count, *hc_mid = c->h_count + 1;
  if (ge && !sweep_ev) {
    // graph replay: the iterations the previous step needed are launched back
    // to back, the last of them with its first cycle only; a slab still in
    // the middle of that iteration then gets the remaining cycles (tail)
    const int L = std::max(1, chain), cap = c->cfg.max_outer + 2;
    const bool one = ge->next1 != nullptr;
    int launched = 1;
    bool part = false;
    // the new temperature goes to the state after every launched chain,
    // ahead of the synchronisation (a later chain copies it again), so a
    // converged step needs no launch after it
    // every iteration graph ends with the end kernel, which publishes its
    // serial number: the host waits for the serial of the last one launched
    int expect = *(c->h_count + 2);
    if (hipGraphLaunch(ge->first, gs) != hipSuccess) return TR_EHIP;
    for (int q = 1; q < L; ++q, ++launched) {
      part = one && q == L - 1;
      if (hipGraphLaunch(part ? ge->next1 : ge->next, gs) != hipSuccess) return TR_EHIP;
    }
    expect += L;
    launch_copy(env, c->Tstar, s->T, c->n_cell);
    for (;;) {
      const int rc = wait_iteration(c, expect, gs);
      if (rc) return rc;
      if (*hc_active == 0) {
        done = true;
        break;
      }
      if (part && *hc_mid > 0) {
        part = false;
        if (hipGraphLaunch(ge->tail, gs) != hipSuccess) return TR_EHIP;
        ++expect;
        launch_copy(env, c->Tstar, s->T, c->n_cell);
        continue;
      }
      if (launched >= cap) break;
      part = false;
      ++launched;
      if (hipGraphLaunch(ge->next, gs) != hipSuccess) return TR_EHIP;
      ++expect;
      launch_copy(env, c->Tstar, s->T, c->n_cell);
    }
  } else {
    // timed sweeps without per-group timing: the sweep of iteration s + 1 is
    // queued behind iteration s before the host waits for it (it sweeps only
    // the slabs still active then, as a launch after the wait would), so its
    // start event is not recorded on an idle stream ahead of the kernel's
    // submission; a launch that found no active slab is not counted
    const bool ahead = sweep_ev && !c->cfg.timing;
    for (int outer = 0; outer <= c->cfg.max_outer + 1; ++outer) {
      // transport sweep of iteration s >= 1 (predicated per slab)
      if (outer > 0 && sweep_ev && !ahead)
        launch_sweeps(c, env, c->d_ctl, PRED_SWEEP, c->kappa, c->B, s->I_prev, s->I_out, c->mom, c->bnd, true);
      if (ge) {
        hipGraphExec_t gx = outer == 0 ? ge->first : ge->rest;
        if (hipGraphLaunch(gx, gs) != hipSuccess) return TR_EHIP;
      } else {
        enqueue_iteration(c, s, gs, Lmax, outer > 0, true);
      }
      const bool next = ahead && outer < c->cfg.max_outer + 1;
      if (next)
        launch_sweeps(c, env, c->d_ctl, PRED_SWEEP, c->kappa, c->B, s->I_prev, s->I_out, c->mom, c->bnd, true);
      if (hipStreamSynchronize(gs) != hipSuccess) return TR_EHIP;
      if (ahead ? (next && *hc_active > 0) : (outer > 0 && sweep_ev)) sweep_time(c, t_ms, n_launch);
      if (c->cfg.timing) {
        // cycles run by slab 0 in the iteration just completed (exact for one slab)
        Ctl k0;
        if (hipMemcpy(&k0, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return TR_EHIP;
        tim_collect(c, s0 < TR_MAXOUT ? k0.cycles[s0] : 0, t_ms, n_launch);
        s0 = k0.s;
      }
      if (*hc_active == 0) {
        done = true;
        break;
      }
    }
  }
  if (!(ge && !sweep_ev)) launch_copy(env, c->Tstar, s->T, c->n_cell);
  if (done) {
    // the last iteration's end kernel wrote the final records to host memory
    // before the synchronisation above
    std::memcpy(hc.data(), c->h_ctl_out, sizeof(Ctl) * ns);
  } else if (hipMemcpyAsync(hc.data(), c->d_ctl, sizeof(Ctl) * ns, hipMemcpyDeviceToHost, gs) != hipSuccess) {
    return TR_EHIP;
  }
  if (c->mlp_params &&
      hipMemcpyAsync(seed_counts, c->d_seed_counts, sizeof(seed_counts), hipMemcpyDeviceToHost, gs) != hipSuccess)
    return TR_EHIP;
  if ((!done || c->mlp_params) && hipStreamSynchronize(gs) != hipSuccess) return TR_EHIP;
  int err = TR_OK;
  c->last_iters = 0;
  for (int q = 0; q < ns; ++q) {
    const Ctl &k = hc[q];
    c->last_iters = std::max(c->last_iters, k.s + 1);
    if (k.active) err = TR_ENOCONV;
    if (k.err) err = k.err;
    if (stats) {
      tr_stats &o = stats[q];
      o.n_ti += k.n_ti;
      o.n_c += k.n_c;
      o.n_lo += k.n_lo;
      o.n_floor += k.n_floor;
      o.n_outer = k.s + 1;
      for (int i = 0; i < 64; ++i) o.cycles[i] = i < TR_MAXOUT ? k.cycles[i] : 0;
      for (int i = 0; i < TR_T_N; ++i) {
        o.t_ms[i] += t_ms[i];
        o.n_launch[i] += n_launch[i];
      }
      if (q == 0) {  // closure counters cover the whole context
        o.n_seeded += (long long)seed_counts[0];
        o.n_fallback += (long long)seed_counts[1];
      }
    }
  }
  return err;
}

}  // namespace

extern "C" {

int tr_step(tr_ctx *c, const tr_state *s, const int *replay, tr_stats *stats, hipStream_t st) {
  return step_impl(c, s, replay, stats, st);
}

int tr_run(tr_ctx *c, const tr_state *s, int nsteps, tr_stats *stats, int *done, hipStream_t st) {
  if (done) *done = 0;
  if (!c || !s || nsteps < 0) return TR_EINVAL;
  tr_state w = *s;
  for (int k = 0; k < nsteps; ++k) {
    const int rc = step_impl(c, &w, nullptr, stats, st);
    if (rc) return rc;
    if (done) *done = k + 1;
    // the two buffers exchange roles (both are the caller's writable arrays)
    double *prev = const_cast<double *>(w.I_prev);
    w.I_prev = w.I_out;
    w.I_out = prev;
  }
  return TR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Alg. 1 on the GPU: one backward-Euler step by transport iterations whose
// low-order stage solves the multigroup LOQD equations and the multigroup MEB
// (Eq. eb-group) together on the fine grid (Newton in T, see the kernels).
// ---------------------------------------------------------------------------
#define TR_A1_NEWTON 60

namespace {

int a1_alloc(tr_ctx *c) {
  auto &a = c->a1;
  if (a.ready) return TR_OK;
  long long nM = 0, nP = 0;
  std::vector<long long> hoM(c->nslab), hoP(c->nslab);
  std::vector<Item> mm, sg;
  for (int k = 0; k < c->nslab; ++k) {
    const SlabDev &S = c->hs[k];
    hoM[k] = nM;
    hoP[k] = nP;
    nM += (long long)S.nx * S.nx;
    nP += (long long)S.ng * S.nx * S.nx;
    for (long long q = 0; q < (long long)S.nx * S.nx; q += 256) mm.push_back({k, (int)q});
    for (int g = 0; g < S.ng; ++g) sg.push_back({k, g});
    const int need = (S.nx + 2 + TR_LO_K - 1) / TR_LO_K;
    a.sg_threads = std::max(a.sg_threads, (need + 63) / 64 * 64);
  }
  const long long nrow = c->n_gi + 2 * c->n_g;
  int rc;
  double **gi[] = {&a.dem, &a.kprev, &a.w};
  for (double **p : gi)
    if ((rc = dalloc(c, p, c->n_gi))) return rc;
  double **rows[] = {&a.ra, &a.cp, &a.dn};
  for (double **p : rows)
    if ((rc = dalloc(c, p, nrow))) return rc;
  double **cells[] = {&a.rhs, &a.phi, &a.alpha, &a.beta, &a.Tprev, &a.Ts, &a.Esum, &a.Esp, &a.Er};
  for (double **p : cells)
    if ((rc = dalloc(c, p, c->n_cell))) return rc;
  if ((rc = dalloc(c, &a.P, nP)) || (rc = dalloc(c, &a.M, nM)) || (rc = dalloc(c, &a.err, c->nslab)) ||
      (rc = dalloc(c, &a.outer, 4LL * c->nslab)) || (rc = dalloc(c, &a.oM, c->nslab)) ||
      (rc = dalloc(c, &a.oP, c->nslab)))
    return rc;
  if (hipMemcpy(a.oM, hoM.data(), 8 * hoM.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(a.oP, hoP.data(), 8 * hoP.size(), hipMemcpyHostToDevice) != hipSuccess)
    return TR_EHIP;
  if ((rc = upload_table(c, mm, a.t_mm)) || (rc = upload_table(c, sg, a.t_sg))) return rc;
  if (hipHostMalloc((void **)&a.h_err, 8 * c->nslab, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&a.h_outer, 32 * c->nslab, hipHostMallocDefault) != hipSuccess)
    return TR_ENOMEM;
  a.ready = true;
  return TR_OK;
}

// Control records of the slabs still iterating (sweep predication and the
// Alg. 1 kernels): active, transport iteration so.
int a1_upload_ctl(tr_ctx *c, const std::vector<int> &act, int so, hipStream_t st) {
  for (int k = 0; k < c->nslab; ++k) {
    Ctl r{};
    r.active = act[k];
    r.s = so;
    c->h_ctl_in[k] = r;
  }
  return hip_err(hipMemcpyAsync(c->d_ctl, c->h_ctl_in, sizeof(Ctl) * c->nslab, hipMemcpyHostToDevice, st));
}

}  // namespace

extern "C" {

int tr_alg1_step(tr_ctx *c, const tr_state *s, tr_stats *stats, hipStream_t st) {
  if (!c || !s || !s->T || !s->I_prev || !s->I_out || !s->E || !s->F || !s->Ebnd || !s->f || !s->fbnd || !s->C ||
      !s->Egrey || s->I_prev == s->I_out)
    return TR_EINVAL;
  int max_nx = 0;
  for (const SlabDev &S : c->hs) {
    if (S.nx > TR_A1_MAX_CELLS) return TR_EINVAL;
    max_nx = std::max(max_nx, S.nx);
  }
  int rc = a1_alloc(c);
  if (rc) return rc;
  auto &w = c->a1;
  const int ns = c->nslab;
  LaunchEnv env = env_of(c, st);
  std::vector<int> act(ns, 1);
  // step start: old-time copies, Phi of the incoming with the state's C
  for (int k = 0; k < ns; ++k) {
    Ctl r{};
    r.active = 1;
    c->h_ctl_in[k] = r;
  }
  launch_step_start(env, s->T, s->Egrey, s->E, s->F, c->n_cell, c->n_gi, c->n_ge, c->Told, c->Ts, c->Tcyc, c->Tstar,
                    c->Es, c->Ecyc, c->Eold, c->Fold, c->h_ctl_in, c->d_ctl, ns, c->t_g, s->C, c->Phi, c->t_opac,
                    c->opac_run, c->kappa, c->B, c->dSpart, c->spectral, c->sigR);
  // radiation temperature of the spectral averages: from the total energy
  // density of the latest solution (held during each Newton solve)
  launch_copy(env, s->Egrey, w.Er, c->n_cell);
  launch_copy(env, s->T, w.Ts, c->n_cell);
  launch_copy(env, s->Egrey, w.Esp, c->n_cell);
  A1Args a{};
  a.in = fine_in(c, c->kappa, c->B, s->f, s->fbnd, s->C, c->Phi, c->Eold, c->Fold);
  a.dem = w.dem;
  a.T = s->T;
  a.Told = c->Told;
  a.Tprev = w.Tprev;
  a.kprev = w.kprev;
  a.Ek = s->E;
  a.alpha = w.alpha;
  a.beta = w.beta;
  a.w = w.w;
  a.ra = w.ra;
  a.cp = w.cp;
  a.dn = w.dn;
  a.P = w.P;
  a.M = w.M;
  a.rhs = w.rhs;
  a.phi = w.phi;
  a.oM = w.oM;
  a.oP = w.oP;
  a.ctl = c->d_ctl;
  a.E = s->E;
  a.F = s->F;
  a.Ebnd = s->Ebnd;
  a.Tout = s->T;
  a.err = w.err;
  std::vector<long long> n_ti(ns, 0), n_c(ns, 0), n_lo(ns, 0);
  std::vector<int> newton_per_it;
  for (int so = 0;; ++so) {
    if ((rc = a1_upload_ctl(c, act, so, st))) return rc;
    if (so > 0) {
      // transport sweep with the opacities at the current T, QD factors
      launch_opacity(env, c->t_opac, c->opac_run, nullptr, PRED_ALL, 0, s->T, c->kappa, c->B, c->dSpart,
                     c->spectral, w.Er, c->sigR);
      launch_sweeps(c, env, c->d_ctl, PRED_SWEEP, c->kappa, c->B, s->I_prev, s->I_out, c->mom, c->bnd);
      launch_moments(env, c->t_gi, c->d_ctl, PRED_SWEEP, 0, c->mom, c->bnd, s->f, s->fbnd, s->C, c->Phi);
      for (int k = 0; k < ns; ++k) n_ti[k] += act[k];
    }
    // Newton iterations of the multigroup LOQD + MEB at fixed factors
    double prev_worst = 0.0;
    int k = 0;
    for (;; ++k) {
      if (k >= TR_A1_NEWTON) return TR_ENOCONV;
      launch_opacity(env, c->t_opac, c->opac_run, nullptr, PRED_ALL, 0, s->T, c->kappa, c->B, c->dSpart,
                     c->spectral, w.Er, c->sigR, w.dem);
      a.first = k == 0;
      launch_a1_prep(env, c->t_cell, a);
      launch_a1_factor(env, c->t_g, a);
      launch_a1_solve_blk(env, w.t_sg, w.sg_threads, a, false);
      launch_a1_rhs(env, c->t_cell, a);
      launch_a1_cols(env, c->t_gi, a);
      launch_a1_mred(env, w.t_mm, a);
      launch_a1_dense(env, ns, max_nx, a);
      launch_a1_solve_blk(env, w.t_sg, w.sg_threads, a, true);
      launch_a1_update(env, ns, a, w.Tprev);
      launch_copy(env, c->kappa, w.kprev, c->n_gi);
      if (hipMemcpyAsync(w.h_err, w.err, 8 * ns, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return TR_EHIP;
      double worst = 0.0;
      for (int q = 0; q < ns; ++q) {
        if (!act[q]) continue;
        if (!std::isfinite(w.h_err[q])) return TR_ENAN;
        worst = std::max(worst, w.h_err[q]);
        n_c[q] += 1;
        n_lo[q] += 2LL * c->hs[q].ng;
      }
      // converged to rounding, or stalled there after a few iterations
      if (worst <= 1e-15 || (k >= 3 && worst <= 1e-13 && worst >= 0.5 * prev_worst)) break;
      prev_worst = worst;
    }
    newton_per_it.push_back(k + 1);
    // outer test (from s = 1 on): T and the total energy density
    launch_a1_outer(env, ns, c->d_ctl, s->T, w.Ts, s->E, w.Esum, w.Esp, w.outer);
    if (hipMemcpyAsync(w.h_outer, w.outer, 32 * ns, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return TR_EHIP;
    int left = 0;
    for (int q = 0; q < ns; ++q) {
      if (!act[q]) continue;
      const double *o = w.h_outer + 4 * q;
      if (so >= 1 && o[0] <= c->cfg.eps * o[1] && o[2] <= c->cfg.eps * o[3]) act[q] = 0;
      left += act[q];
    }
    launch_copy(env, s->T, w.Ts, c->n_cell);
    launch_copy(env, w.Esum, w.Esp, c->n_cell);
    launch_copy(env, w.Esum, w.Er, c->n_cell);
    if (left == 0) break;
    if (so >= c->cfg.max_outer) return TR_ENOCONV;
  }
  launch_copy(env, w.Esum, s->Egrey, c->n_cell);
  if (stats) {
    for (int q = 0; q < ns; ++q) {
      stats[q].n_ti += n_ti[q];
      stats[q].n_c += n_c[q];
      stats[q].n_lo += n_lo[q];
      stats[q].n_outer = (int)newton_per_it.size();
      for (int i = 0; i < 64; ++i) stats[q].cycles[i] = i < (int)newton_per_it.size() ? newton_per_it[i] : 0;
    }
  }
  return hip_err(hipStreamSynchronize(st));
}

}  // extern "C"
