"""Helpers shared by the GPU parity tests (host-side marshalling only)."""
import sys

import numpy as np

from paper_2011_05427_amd import inputs


def note(msg):
    """Names the case before a GPU step (flushed, so a failure is traceable)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).to("cuda")


def to_np(t, shape=None):
    a = t.detach().cpu().numpy()
    return a if shape is None else a.reshape(shape)


def assert_close(name, got, ref, rtol, atol_scale=None):
    """Elementwise |got - ref| <= rtol |ref| + rtol * max|ref| (the second term
    admits the roundoff of entries far below the array's scale)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    scale = np.max(np.abs(ref)) if atol_scale is None else atol_scale
    tol = rtol * np.abs(ref) + rtol * scale
    bad = ~(np.abs(got - ref) <= tol)
    if np.any(bad):
        idx = np.argwhere(bad)[0]
        raise AssertionError(f"{name}: {np.count_nonzero(bad)} mismatches, first at {tuple(idx)}: "
                             f"got {got[tuple(idx)]!r} ref {ref[tuple(idx)]!r} (rtol {rtol})")


def rel_err(got, ref):
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def slab_case(nx, ng, nmu, *, levels=None, cycle=inputs.CYCLE_V, lmax=4, eps=1e-10, eps_inner=1e-11, **kw):
    slab = inputs.make_slab(nx, ng, nmu, **kw)
    lv = levels if levels is not None else [ng, 1]
    cfg = inputs.SolverCfg(levels=lv, cycle=cycle, lmax=lmax, eps=eps, eps_inner=eps_inner)
    return slab, cfg
