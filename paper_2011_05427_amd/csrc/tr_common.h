// Shared host/device definitions of the MI355X MLQD library (gfx950, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TR_MAXLEV 8
#define TR_MAXOUT 64

// Per-slab descriptor (device resident).  Offsets are element offsets into
// the pooled arrays of each kind (see include/tr.h).
struct SlabDev {
  int nx, ng, nmu, nlev;
  int lev_ng[TR_MAXLEV];
  int nchunk;            // 64-group chunks of the fine grid (opacity partials)
  int rtarget;           // restriction chunk pass: blocks aimed at per slab
  int opac;              // TR_OPAC_POINT / TR_OPAC_SPECTRAL
  double cv, dt, c, aR, inv_cdt;
  double wpos, wmupos, wmu2pos;  // half-range quadrature sums over mu > 0
  double wneg, wmuneg, wmu2neg;  // over mu < 0 (wmuneg < 0)
  double f_iso, c_iso;
  double T_left;  // incoming Planck temperature at x = 0 (<= 0: vacuum)
  long long o_cell, o_edge, o_I, o_gi, o_ge, o_g, o_g2, o_nu, o_mu, o_chunk;
  long long o_lpi[TR_MAXLEV], o_lpe[TR_MAXLEV], o_lp2[TR_MAXLEV];
  long long o_red;  // restriction scratch records (per slab)
  long long o_gpi, o_gpe, o_gp2;  // grey level offsets (= o_lpi / o_lpe / o_lp2 of the last level)
  long long o_dsop;          // stage dS partials (per slab)
  int dsnp[TR_MAXLEV];       // stage dS partial rows of the restriction fine -> level
};

// Problem constants (device, pooled).
struct ProbDev {
  const double *dx;      // [cells]
  const double *Ccell;   // [cells]
  const double *mu, *w;  // [o_mu + nmu]
  const double *nu_e;    // [o_nu + ng + 1]
  const double *nu_c;    // [o_g + ng]
  const double *inc;     // [2 * (o_g + ng)]: incoming left at 2*o_g, right at 2*o_g + ng
};

// Per-slab iteration control (device resident).
struct Ctl {
  int active;      // still iterating in this step
  int s;           // transport iteration index
  int ncyc;        // cycles run in the current transport iteration
  int inner_done;  // inner loop of the current transport iteration finished
  int has_prev;    // a grey stage of this step exists (secant derivative)
  int err;         // TR_ENOCONV / TR_ENAN
  int n_replay;    // > 0: replay mode with this many transport iterations
  int pad_;
  int replay[TR_MAXOUT];
  int cycles[TR_MAXOUT];
  long long n_ti, n_c, n_lo, n_floor;
};

// Work tables map a block (or wave) to (slab, first item).
struct Item {
  int slab;
  int idx;
};
