"""Autotuning: sweep tiles of a batch, and the cycle and lmax of time steps.

The library times each sweep tile (cells per lane K = 1, 2, 4, 8 and split =
1, 2, 4 wavefronts per group and half range) on every slab-size bucket of a
context (``tr_autotune``).  This module keeps the choice
in a JSON cache keyed by device name and by the bucket's occupancy signature,
so a later context over the same kind of batch reuses it (``tr_set_tiles``)
without timing again.

``tune_schedule`` and ``StageSchedule`` choose the multigrid cycle and lmax
(``tr_set_schedule``) from measured step times: once in a set-up, or step by
step as the problem passes through its stages.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "tiles.json")
BUCKETS = ["nx<=64", "nx<=128", "nx<=256", "nx<=512", "nx<=1024", "nx>1024"]


def _key(sv) -> str:
    import torch

    _, _, items = sv.get_tiles()
    dev = torch.cuda.get_device_name(0)
    # bucket occupancy rounded to powers of two: nearby batches share a choice
    sig = [0 if n == 0 else int(n).bit_length() for n in items]
    return f"{dev}|{sig}"


def load(path: str = DEFAULT_CACHE) -> Dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def tune(sv, st, reps: int = 3, path: Optional[str] = DEFAULT_CACHE, force: bool = False) -> Dict:
    """Applies the cached tiles for this batch, or times them and caches."""
    cache = load(path) if path else {}
    key = _key(sv)
    if key in cache and not force:
        sv.set_tiles(cache[key]["K"], cache[key].get("split"))
        return dict(cache[key], cached=True)
    K, split, us = sv.autotune(st, reps)
    entry = {"K": K, "split": split, "us": us, "buckets": BUCKETS}
    if path:
        cache[key] = entry
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dict(entry, cached=False)


# ---------------------------------------------------------------------------
# Cycle and lmax per time step (tr_set_schedule)
# ---------------------------------------------------------------------------

def _sync():
    import torch

    if torch.cuda.is_available():
        torch.cuda.synchronize()


def tune_schedule(sv, st, candidates, steps: int = 2) -> Dict:
    """Milliseconds per step of every (cycle, lmax) candidate over the same
    `steps` steps from the state `st`, which is restored afterwards (untimed
    set-up, like the tile autotuner).  Two untimed steps per candidate build
    its graphs first.  Returns {candidate: ms per step}, cheapest first."""
    snap = {k: v.clone() for k, v in st.items()}

    def restore():
        for k, v in snap.items():
            st[k].copy_(v)
        _sync()

    out = {}
    for cand in candidates:
        cand = (int(cand[0]), int(cand[1]))
        sv.set_schedule(*cand)
        restore()
        for _ in range(2):
            sv.step(st)
        restore()
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.step(st)
        _sync()
        out[cand] = 1e3 * (time.perf_counter() - t0) / steps
    restore()
    return dict(sorted(out.items(), key=lambda kv: kv[1]))


class StageSchedule:
    """Chooses (cycle, lmax) for each time step from measured step times.

    Which cycle and lmax are cheapest changes with the stage of the problem
    (radiation entering the slab, the wave forming, a developed wave, near
    steady state) and with the time step (paper, Sec. 6 and the conclusions, Sec. 7).
    Per candidate the controller keeps an exponentially weighted mean of its
    measured milliseconds per step (weight `decay` on the older mean).  A
    candidate without a measurement is tried first (in the given order);
    afterwards the cheapest runs, except that every `probe`-th step re-runs
    the candidate measured longest ago, so that a change of stage can reorder
    them.  `initial` seeds the means (e.g. from ``tune_schedule``).  The
    choices depend only on the recorded times (ties: candidate order)."""

    def __init__(self, candidates, probe: int = 8, decay: float = 0.5, initial: Optional[Dict] = None):
        self.cands = [(int(c[0]), int(c[1])) for c in candidates]
        if not self.cands:
            raise ValueError("no candidate schedule")
        if probe < 0 or not (0.0 <= decay < 1.0):
            raise ValueError("probe >= 0 and 0 <= decay < 1 required")
        self.probe, self.decay = probe, decay
        self.cost: Dict = {}
        self.seen: Dict = {}
        self.k = 0
        self.history = []
        for c, ms in (initial or {}).items():
            c = (int(c[0]), int(c[1]))
            if c in self.cands:
                self.cost[c] = float(ms)
                self.seen[c] = -1

    def _rank(self, c):
        return self.cands.index(c)

    def choose(self):
        for c in self.cands:
            if c not in self.cost:
                return c
        if self.probe and self.k > 0 and self.k % self.probe == 0:
            return min(self.cands, key=lambda c: (self.seen[c], self._rank(c)))
        return min(self.cands, key=lambda c: (self.cost[c], self._rank(c)))

    def record(self, cand, ms: float):
        cand = (int(cand[0]), int(cand[1]))
        old = self.cost.get(cand)
        self.cost[cand] = float(ms) if old is None else self.decay * old + (1.0 - self.decay) * float(ms)
        self.seen[cand] = self.k
        self.history.append((cand, float(ms)))
        self.k += 1

    def step(self, sv, st, **kw):
        """One time step of `sv` with the chosen schedule; records its time."""
        cand = self.choose()
        if tuple(getattr(sv, "schedule", ())) != cand:
            sv.set_schedule(*cand)
        t0 = time.perf_counter()
        out = sv.step(st, **kw)
        _sync()
        self.record(cand, 1e3 * (time.perf_counter() - t0))
        return out


# ---------------------------------------------------------------------------
# Hierarchy per time step (tr_set_grids) chosen by a cost model
# ---------------------------------------------------------------------------

def apply_schedule(sv, cand):
    """cand = (sched, lmax): sched an int cycle (tr_set_schedule over the
    context's grids) or a tuple of context grid indices visited after each
    grey solve (tr_set_grids)."""
    sched, lmax = cand
    if isinstance(sched, tuple):
        sv.set_grids(sched, lmax)
    else:
        sv.set_schedule(int(sched), int(lmax))


def measure_sweep_ms(sv, st, steps: int = 1) -> float:
    """Kernel time of one transport sweep (start / end events of the sweep
    launches over `steps` steps from a snapshot of `st`, restored after)."""
    from . import binding

    snap = {k: v.clone() for k, v in st.items()}
    acc = (binding.TrStats * sv.n)()
    sv.set_sweep_timing(True)
    try:
        for _ in range(steps):
            sv.step(st, stats=acc)
    finally:
        sv.set_sweep_timing(False)
    for k, v in snap.items():
        st[k].copy_(v)
    _sync()
    sweeps = max(int(a.n_ti) for a in acc)
    return acc[0].t_ms[binding.T_SWEEP] / max(sweeps, 1)


class CostModelSchedule:
    """Chooses the grid hierarchy (grids visited after each grey solve) and
    lmax of every time step from a cost model of the step,

        cost(c) = s_c t_sweep + (s_c + 1) k_c t_c,   s_c = r_c d,

    with t_sweep the measured kernel time of a sweep, and per candidate c its
    cycles per transport iteration k_c and time per cycle t_c (measured:
    (step time - sweeps t_sweep) / cycles), and its sweeps per step relative
    to the others r_c.  d, the transport difficulty of the current stage of
    the problem (sweeps per step of a reference candidate), is updated by every
    step whatever candidate ran it: the paper's tables show the number of
    transport iterations changing little between hierarchies while the
    low-order work changes by up to 3x, so one candidate's sweeps predict the
    others' and the choice follows the stage (e.g. when few sweeps per step
    remain, the per-step cycle of iteration s = 0 weighs more) without
    running every candidate.  Weighted means use weight `decay` on the older
    value.  Unmeasured candidates run first (in the given order); every
    `probe`-th step re-runs the candidate measured longest ago among those
    predicted within `probe_margin` of the best.  `seed` starts the model from
    measurements of the candidates over the same steps (an untimed set-up).
    `ratio_prior`, if given, replaces the seeded sweep ratios by that value
    for every candidate: the set-up's first steps from the initial state are
    the problem's hardest transient, where the hierarchies' sweep counts
    differ most, so their ratios can rank a candidate by a difference that the
    later steps do not have; the prior (1: the transport iterations do not
    depend on the hierarchy) keeps the seeded cycle costs and lets the
    recorded steps move the ratios.  Deterministic in the recorded counts and
    times (ties: candidate order)."""

    def __init__(self, candidates, t_sweep: float, probe: int = 8, decay: float = 0.5, ratio_decay: float = 0.9,
                 seed=None, probe_margin: float = 1.25, ratio_prior=None):
        self.cands = [self._norm(c) for c in candidates]
        self.ratio_decay = float(ratio_decay)
        if not self.cands:
            raise ValueError("no candidate schedule")
        if probe < 0 or not (0.0 <= decay < 1.0) or not (t_sweep >= 0.0) or not (probe_margin >= 1.0):
            raise ValueError("probe >= 0, 0 <= decay < 1, t_sweep >= 0 and probe_margin >= 1 required")
        self.t_sweep, self.probe, self.decay, self.margin = float(t_sweep), probe, decay, float(probe_margin)
        self.r, self.k_c, self.t_c, self.seen = {}, {}, {}, {}
        self.d = None
        self.k = 0
        self.history = []
        if ratio_prior is not None and not (float(ratio_prior) > 0.0):
            raise ValueError("ratio_prior > 0 required")
        self.ratio_prior = None if ratio_prior is None else float(ratio_prior)
        if seed:
            self._seed(seed)

    @staticmethod
    def _norm(c):
        return (tuple(c[0]) if isinstance(c[0], (tuple, list)) else int(c[0]), int(c[1]))

    def _seed(self, seed):
        """seed: {candidate: (ms, sweeps, cycles, steps)} measured over the
        same steps from the same state (an untimed set-up), so that the
        sweep ratios carry no difference of stage.  The first candidate of
        the list with a measurement is the reference (r = 1)."""
        seed = {self._norm(c): v for c, v in seed.items()}
        ref = next((c for c in self.cands if c in seed), None)
        if ref is None:
            return
        s_ref = max(float(seed[ref][1]), 1.0)
        for c in self.cands:
            if c not in seed:
                continue
            ms, sw, cyc, n = (float(x) for x in seed[c])
            self.r[c] = max(sw, 1.0) / s_ref if self.ratio_prior is None else self.ratio_prior
            self.k_c[c] = cyc / (sw + n)
            self.t_c[c] = max(ms - sw * self.t_sweep, 0.0) / max(cyc, 1.0)
            self.seen[c] = -1
        self.d = s_ref / max(float(seed[ref][3]), 1.0)

    def _mix(self, old, new):
        return float(new) if old is None else self.decay * old + (1.0 - self.decay) * float(new)

    def predict(self, c) -> float:
        s = self.r[c] * self.d
        return s * self.t_sweep + (s + 1.0) * self.k_c[c] * self.t_c[c]

    def choose(self):
        for c in self.cands:
            if c not in self.r:
                return c
        best = min(self.cands, key=lambda c: (self.predict(c), self.cands.index(c)))
        if self.probe and self.k > 0 and self.k % self.probe == 0:
            # re-measure the candidate measured longest ago among those
            # predicted within the margin of the best
            near = [c for c in self.cands if self.predict(c) <= self.margin * self.predict(best)]
            return min(near, key=lambda c: (self.seen[c], self.cands.index(c)))
        return best

    def record(self, cand, ms: float, sweeps: int, cycles: int):
        sweeps, cycles = max(int(sweeps), 0), max(int(cycles), 1)
        s = float(max(sweeps, 1))
        if self.d is None:
            self.d, self.r[cand] = s, 1.0
        elif cand not in self.r:
            self.r[cand] = s / self.d
        else:
            # the stage's difficulty from the candidate's known ratio, then the
            # ratio itself drifts slowly towards the new observation
            self.d = self._mix(self.d, s / self.r[cand])
            self.r[cand] = self.ratio_decay * self.r[cand] + (1.0 - self.ratio_decay) * s / self.d
        self.k_c[cand] = self._mix(self.k_c.get(cand), cycles / (sweeps + 1.0))
        self.t_c[cand] = self._mix(self.t_c.get(cand), max(ms - sweeps * self.t_sweep, 0.0) / cycles)
        self.seen[cand] = self.k
        self.history.append((cand, float(ms), sweeps, cycles))
        self.k += 1

    def step(self, sv, st, **kw):
        """One time step of `sv` with the chosen hierarchy; records its time
        and its counts (the slowest slab's)."""
        from . import binding

        cand = self.choose()
        if tuple(getattr(sv, "schedule", ())) != cand:
            apply_schedule(sv, cand)
        one = (binding.TrStats * sv.n)()
        t0 = time.perf_counter()
        out = sv.step(st, stats=one)
        _sync()
        ms = 1e3 * (time.perf_counter() - t0)
        self.record(cand, ms, max(int(a.n_ti) for a in one), max(int(a.n_c) for a in one))
        acc = kw.get("stats")
        if acc is not None:
            for q in range(sv.n):
                for f in ("n_ti", "n_c", "n_lo", "n_floor", "n_seeded", "n_fallback"):
                    setattr(acc[q], f, getattr(acc[q], f) + getattr(one[q], f))
        return out
