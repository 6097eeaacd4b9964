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
