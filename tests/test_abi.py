"""The C ABI library loads and exports every entry point declared in
include/tr.h (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2011_05427_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(tr_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    assert set(binding.EXPORTS) == set(names), names


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="libtr.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    lib.tr_error_string.restype = ctypes.c_char_p
    assert lib.tr_error_string(-4).startswith(b"transport iterations")


def test_structs_match_header_field_order():
    src = open(os.path.join(ROOT, "include", "tr.h")).read()
    body = src[src.index("typedef struct tr_state"):]
    body = body[:body.index("} tr_state;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\*\s*(\w+)", body)
    assert [f for f, _ in binding.TrState._fields_] == fields


def _create(slabs, levels, cfg):
    """tr_create through the C ABI on host-side arrays (argument checks run
    before any device work, so this needs no GPU)."""
    import ctypes as C

    import numpy as np

    lib = binding.load()
    keep = []
    probs = (binding.TrProblem * max(1, len(slabs)))()
    for k, (s, lv) in enumerate(zip(slabs, levels)):
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in
                (s.x_edges, s.nu_edges, s.nu_center, s.mu, s.w, s.C_cell)]
        lvl = np.ascontiguousarray(lv, dtype=np.int32)
        keep += arrs + [lvl]
        p = probs[k]
        p.nx, p.ng, p.nmu = s.nx, s.ng, s.nmu
        p.x_edges, p.nu_edges, p.nu_center, p.mu, p.w, p.C_cell = [a.ctypes.data_as(binding._dp) for a in arrs]
        p.T_left, p.T_right, p.cv, p.dt, p.c, p.aR = s.T_left, s.T_right, s.cv, s.dt, s.c, s.aR
        p.n_levels = len(lv)
        p.level_ng = lvl.ctypes.data_as(binding._ip)
    c = binding.TrSolverCfg(cycle=cfg.cycle, lmax=cfg.lmax, eps=cfg.eps, eps_inner=cfg.eps_inner,
                            max_outer=cfg.max_outer, secant=1, timing=0, precision=cfg.precision)
    ctx = C.c_void_p()
    rc = lib.tr_create(C.byref(ctx), probs, len(slabs), C.byref(c))
    assert not ctx, "an invalid problem must not create a context"
    return rc


def test_create_rejects_invalid_problems():
    """Shapes outside the documented limits return TR_EINVAL (before any
    allocation): more than 2046 cells, one cell, odd or too many directions,
    level sizes that do not divide, a last level that is not grey, non-
    increasing cell edges, an asymmetric quadrature, bad solver settings and
    an empty batch."""
    import dataclasses

    import numpy as np

    from paper_2011_05427_amd import inputs

    EINVAL = -1  # TR_EINVAL
    ok = inputs.make_slab(10, 8, 4)
    cfg = inputs.SolverCfg(levels=[8, 1])
    assert _create([inputs.make_slab(2047, 4, 2)], [[4, 1]], cfg) == EINVAL
    assert _create([inputs.make_slab(1, 4, 2)], [[4, 1]], cfg) == EINVAL
    odd = dataclasses.replace(ok, mu=np.array([-0.5, 0.0, 0.5]), w=np.array([0.5, 1.0, 0.5]))
    assert _create([odd], [[8, 1]], cfg) == EINVAL
    many = dataclasses.replace(ok, mu=np.linspace(-0.99, 0.99, 66), w=np.full(66, 2.0 / 66))
    assert _create([many], [[8, 1]], cfg) == EINVAL
    assert _create([ok], [[8, 3, 1]], inputs.SolverCfg(levels=[8, 3, 1])) == EINVAL
    assert _create([ok], [[8, 2]], inputs.SolverCfg(levels=[8, 2])) == EINVAL
    bad_x = dataclasses.replace(ok, x_edges=np.concatenate([[0.0, 0.5, 0.5], np.linspace(1, 4, 8)]))
    assert _create([bad_x], [[8, 1]], cfg) == EINVAL
    asym = dataclasses.replace(ok, mu=np.array([-0.6, -0.2, 0.3, 0.6]))
    assert _create([asym], [[8, 1]], cfg) == EINVAL
    assert _create([ok], [[8, 1]], dataclasses.replace(cfg, lmax=0)) == EINVAL
    assert _create([ok], [[8, 1]], dataclasses.replace(cfg, precision=2)) == EINVAL
    assert _create([], [], cfg) == EINVAL
    # a batch whose slabs disagree on the number of levels
    assert _create([ok, ok], [[8, 1], [8, 4, 1]], cfg) == EINVAL


@pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="libtr.so not built (run __graft_entry__.build())")
def test_calls_without_a_context_are_rejected():
    """Every entry point taking a context returns TR_EINVAL for a null one
    before touching the device (tile, timing and closure calls here)."""
    lib = binding.load()
    EINVAL = -1
    K = (ctypes.c_int * 6)(4, 4, 4, 4, 4, 4)
    S = (ctypes.c_int * 6)(1, 2, 4, 1, 2, 4)
    assert lib.tr_set_tiles(None, K, S) == EINVAL
    assert lib.tr_get_tiles(None, K, S, None) == EINVAL
    assert lib.tr_autotune(None, None, None, 1, K, S, None, None) == EINVAL
    assert lib.tr_set_sweep_timing(None, 1) == EINVAL
    assert lib.tr_set_schedule(None, 0, 1) == EINVAL
    assert lib.tr_run(None, None, 1, None, None, None) == EINVAL
    assert lib.tr_step(None, None, None, None, None) == EINVAL
