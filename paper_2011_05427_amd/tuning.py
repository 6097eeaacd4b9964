"""Autotuner cache for the batched sweep tiles.

The library times each sweep tile (cells per lane K = 1, 2, 4, 8 and split =
1, 2, 4 wavefronts per group and half range) on every slab-size bucket of a
context (``tr_autotune``).  This module keeps the choice
in a JSON cache keyed by device name and by the bucket's occupancy signature,
so a later context over the same kind of batch reuses it (``tr_set_tiles``)
without timing again.
"""
from __future__ import annotations

import json
import os
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
