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


FLOOR = 1e-290  # values at or below this carry no relative precision (subnormal range nearby)


def assert_close(name, got, ref, rtol, atol_scale=None):
    """Elementwise |got - ref| <= rtol |ref| + rtol * scale + FLOOR, where the
    scale is the largest |ref| of the element's own row: a group's values
    ([G, n] arrays: per group), a group-direction's corner values ([G, M, n, 2]
    intensities: per (g, m); [M, n, 2]: per m), the whole array for 1-D
    arrays.  So a cold group many decades below the hot ones is held to its
    own scale, and only entries near zero inside a row (sign changes,
    attenuation across the slab) get the row's absolute slack.  atol_scale
    overrides the row scale (0: purely relative)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    if atol_scale is not None:
        scale = atol_scale
    elif ref.ndim <= 1:
        scale = np.max(np.abs(ref)) if ref.size else 0.0
    else:
        lead = ref.ndim - 1 if ref.ndim == 2 else ref.ndim - 2
        axes = tuple(range(lead, ref.ndim))
        scale = np.max(np.abs(ref), axis=axes, keepdims=True)
    tol = rtol * np.abs(ref) + rtol * scale + FLOOR
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
