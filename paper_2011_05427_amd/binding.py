"""Thin ctypes binding of libtr.so (argument marshalling only).

PyTorch is used for device memory and the current stream; every computation
runs in the library's HIP kernels.  There is no fallback: if the library is not
built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtr.so")

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EHIP, TR_ENOCONV, TR_ENAN = 0, -1, -2, -3, -4, -5
TR_K_CELL, TR_K_EDGE, TR_K_I, TR_K_GI, TR_K_GE, TR_K_G2, TR_K_G = 0, 1, 2, 3, 4, 5, 6
TR_K_LEV_PI, TR_K_LEV_PE, TR_K_LEV_P2 = 8, 16, 24
TR_MLP_NOALLOC_MAX_N = 4096  # samples per tr_mlp_grad_noalloc call (size of its device scratch)
MAXOUT = 64

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class TrProblem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ng", C.c_int), ("nmu", C.c_int),
                ("x_edges", _dp), ("nu_edges", _dp), ("nu_center", _dp), ("mu", _dp), ("w", _dp),
                ("C_cell", _dp), ("T_left", C.c_double), ("T_right", C.c_double), ("cv", C.c_double),
                ("dt", C.c_double), ("c", C.c_double), ("aR", C.c_double), ("n_levels", C.c_int),
                ("level_ng", _ip), ("opacity", C.c_int)]


class TrSolverCfg(C.Structure):
    _fields_ = [("cycle", C.c_int), ("lmax", C.c_int), ("eps", C.c_double), ("eps_inner", C.c_double),
                ("max_outer", C.c_int), ("secant", C.c_int), ("timing", C.c_int), ("precision", C.c_int)]


class TrLoCoeffs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("kappa", "B", "f", "fbnd", "sigRc", "sigE", "emis", "a", "b", "sigR", "C", "Phi", "Eold",
                 "Fold")]


class TrLoFields(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("E", "F", "Ebnd")]


class TrLoOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("sigE", "emis", "a", "b", "sigR", "C", "Phi", "Eold", "Fold", "Esum")]


class TrState(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("T", "I_prev", "I_out", "E", "F", "Ebnd", "f", "fbnd", "C", "Egrey")]


class TrStats(C.Structure):
    _fields_ = [("n_ti", C.c_longlong), ("n_c", C.c_longlong), ("n_lo", C.c_longlong),
                ("n_floor", C.c_longlong), ("n_outer", C.c_int), ("cycles", C.c_int * 64),
                ("t_ms", C.c_double * 8), ("n_launch", C.c_longlong * 8),
                ("n_seeded", C.c_longlong), ("n_fallback", C.c_longlong)]


T_OPACITY, T_SWEEP, T_MOMENTS, T_LO_FINE, T_RESTRICT, T_LO_COARSE, T_GREY = range(7)


EXPORTS = ["tr_create", "tr_destroy", "tr_error_string", "tr_layout", "tr_set_incoming", "tr_opacity",
           "tr_sweep", "tr_moments", "tr_lo_solve", "tr_restrict", "tr_grey_solve", "tr_state_init", "tr_step",
           "tr_mlp_nparam", "tr_mlp_work_bytes", "tr_mlp_train_work_bytes", "tr_mlp_forward", "tr_mlp_grad",
           "tr_mlp_grad_noalloc", "tr_mlp_adam", "tr_mlp_train_epoch", "tr_mlp_features", "tr_closure_targets", "tr_set_closure",
           "tr_closure_seed",
           "tr_autotune", "tr_set_tiles", "tr_get_tiles", "tr_set_sweep_timing",
           "tr_prolong", "tr_set_schedule", "tr_run", "tr_alg1_step", "tr_set_grids"]

_lib = None


class TrError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {load().tr_error_string(code).decode()} ({code})")


def load():
    """Loads libtr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2011_05427_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.tr_create.argtypes = [C.POINTER(vp), C.POINTER(TrProblem), C.c_int, C.POINTER(TrSolverCfg)]
    lib.tr_destroy.argtypes = [vp]
    lib.tr_error_string.argtypes = [C.c_int]
    lib.tr_error_string.restype = C.c_char_p
    lib.tr_layout.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
    lib.tr_set_incoming.argtypes = [vp, C.c_int, _dp, _dp]
    lib.tr_opacity.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tr_sweep.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tr_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.tr_lo_solve.argtypes = [vp, C.c_int, C.POINTER(TrLoCoeffs), C.POINTER(TrLoFields), vp]
    lib.tr_restrict.argtypes = [vp, C.c_int, C.c_int, C.POINTER(TrLoCoeffs), C.POINTER(TrLoFields),
                                C.POINTER(TrLoOut), vp]
    lib.tr_grey_solve.argtypes = [vp, C.POINTER(TrLoCoeffs), vp, vp, vp, vp, vp, vp, C.POINTER(TrLoFields), vp]
    lib.tr_state_init.argtypes = [vp, C.POINTER(TrState), C.c_double, vp]
    lib.tr_step.argtypes = [vp, C.POINTER(TrState), _ip, C.POINTER(TrStats), vp]
    lib.tr_set_sweep_timing.argtypes = [vp, C.c_int]
    lib.tr_set_schedule.argtypes = [vp, C.c_int, C.c_int]
    lib.tr_set_grids.argtypes = [vp, C.c_int, _ip, C.c_int]
    lib.tr_run.argtypes = [vp, C.POINTER(TrState), C.c_int, C.POINTER(TrStats), _ip, vp]
    lib.tr_alg1_step.argtypes = [vp, C.POINTER(TrState), C.POINTER(TrStats), vp]
    lib.tr_prolong.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    lib.tr_mlp_nparam.argtypes = []
    lib.tr_mlp_work_bytes.argtypes = [C.c_longlong]
    lib.tr_mlp_work_bytes.restype = C.c_size_t
    lib.tr_mlp_train_work_bytes.argtypes = [C.c_int]
    lib.tr_mlp_train_work_bytes.restype = C.c_size_t
    lib.tr_mlp_forward.argtypes = [vp, vp, C.c_longlong, vp, vp, vp]
    lib.tr_mlp_grad.argtypes = [vp, vp, vp, C.c_longlong, vp, vp, vp, vp]
    lib.tr_mlp_grad_noalloc.argtypes = [vp, vp, vp, C.c_longlong, vp, vp, vp]
    lib.tr_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, vp]
    lib.tr_mlp_train_epoch.argtypes = [vp, vp, vp, _ip, C.c_float, vp, vp, C.c_longlong, vp, C.c_int, vp, vp, vp]
    lib.tr_mlp_features.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_float), C.POINTER(C.c_float), vp, vp]
    lib.tr_closure_targets.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp]
    lib.tr_set_closure.argtypes = [vp, vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    lib.tr_closure_seed.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.tr_autotune.argtypes = [vp, vp, vp, C.c_int, _ip, _ip, _dp, vp]
    lib.tr_set_tiles.argtypes = [vp, _ip, _ip]
    lib.tr_get_tiles.argtypes = [vp, _ip, _ip, _ip]
    for name in EXPORTS:
        if name not in ("tr_error_string", "tr_mlp_work_bytes", "tr_mlp_train_work_bytes"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(code, what):
    if code != TR_OK:
        raise TrError(code, what)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _as_dp(a: np.ndarray):
    return a.ctypes.data_as(_dp)


class Solver:
    """One context over a batch of slab problems.

    slabs: sequence of ``inputs.Slab``; levels: per-slab list of groups per
    frequency grid (fine first, grey last); cfg: ``inputs.SolverCfg``."""

    def __init__(self, slabs: Sequence, levels: Sequence[Sequence[int]], cfg, timing: bool = False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the MLQD library needs a ROCm GPU; none is visible")
        self.torch = torch
        self.lib = load()
        self.slabs = list(slabs)
        self._keep = []
        probs = (TrProblem * len(self.slabs))()
        for k, (s, lv) in enumerate(zip(self.slabs, levels)):
            arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in
                    (s.x_edges, s.nu_edges, s.nu_center, s.mu, s.w, s.C_cell)]
            lvl = np.ascontiguousarray(lv, dtype=np.int32)
            self._keep += arrs + [lvl]
            p = probs[k]
            p.nx, p.ng, p.nmu = s.nx, s.ng, s.nmu
            p.x_edges, p.nu_edges, p.nu_center, p.mu, p.w, p.C_cell = [_as_dp(a) for a in arrs]
            p.T_left, p.T_right, p.cv, p.dt, p.c, p.aR = s.T_left, s.T_right, s.cv, s.dt, s.c, s.aR
            p.n_levels = len(lv)
            p.level_ng = lvl.ctypes.data_as(_ip)
            p.opacity = int(getattr(s, "opacity", 0))
        self.levels = [list(lv) for lv in levels]
        self.nlev = len(self.levels[0])
        self.precision = int(getattr(cfg, "precision", 0))
        c = TrSolverCfg(cycle=cfg.cycle, lmax=cfg.lmax, eps=cfg.eps, eps_inner=cfg.eps_inner,
                        max_outer=cfg.max_outer, secant=1 if cfg.secant else 0, timing=1 if timing else 0,
                        precision=self.precision)
        self._ctx = C.c_void_p()
        _check(self.lib.tr_create(C.byref(self._ctx), probs, len(self.slabs), C.byref(c)), "tr_create")
        self.n = len(self.slabs)
        self.schedule = (int(cfg.cycle), int(cfg.lmax))

    def close(self):
        if self._ctx:
            self.lib.tr_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout -----------------------------------------------------------
    def layout(self, kind: int, slab: int = 0):
        off, tot = C.c_longlong(), C.c_longlong()
        _check(self.lib.tr_layout(self._ctx, kind, slab, C.byref(off), C.byref(tot)), "tr_layout")
        return off.value, tot.value

    def total(self, kind: int) -> int:
        return self.layout(kind, 0)[1]

    def offsets(self, kind: int) -> List[int]:
        return [self.layout(kind, s)[0] for s in range(self.n)]

    def empty(self, kind: int, mult: int = 1):
        return self.torch.zeros(self.total(kind) * mult, dtype=self.torch.float64, device="cuda")

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    # -- stages -----------------------------------------------------------
    def set_incoming(self, slab: int, left=None, right=None):
        l = None if left is None else np.ascontiguousarray(left, dtype=np.float64)
        r = None if right is None else np.ascontiguousarray(right, dtype=np.float64)
        _check(self.lib.tr_set_incoming(self._ctx, slab, None if l is None else _as_dp(l),
                                        None if r is None else _as_dp(r)), "tr_set_incoming")

    def opacity(self, T, kappa, B, dS=None, Egrey=None, sigR=None):
        _check(self.lib.tr_opacity(self._ctx, _ptr(T), _ptr(Egrey), _ptr(kappa), _ptr(B), _ptr(sigR), _ptr(dS),
                                   self._stream()), "tr_opacity")

    def sweep(self, kappa, B, I_prev, I_out, mom, bnd):
        _check(self.lib.tr_sweep(self._ctx, _ptr(kappa), _ptr(B), _ptr(I_prev), _ptr(I_out), _ptr(mom),
                                 _ptr(bnd), self._stream()), "tr_sweep")

    def moments(self, mom, bnd, f, fbnd, Cb, Phi):
        _check(self.lib.tr_moments(self._ctx, _ptr(mom), _ptr(bnd), _ptr(f), _ptr(fbnd), _ptr(Cb), _ptr(Phi),
                                   self._stream()), "tr_moments")

    @staticmethod
    def _coeffs(d: Dict) -> TrLoCoeffs:
        c = TrLoCoeffs()
        for name, _ in TrLoCoeffs._fields_:
            setattr(c, name, _ptr(d.get(name)))
        return c

    def lo_solve(self, level: int, coeffs: Dict, E, F, Ebnd):
        f = TrLoFields(E=_ptr(E), F=_ptr(F), Ebnd=_ptr(Ebnd))
        _check(self.lib.tr_lo_solve(self._ctx, level, C.byref(self._coeffs(coeffs)), C.byref(f), self._stream()),
               "tr_lo_solve")

    def restrict(self, frm: int, to: int, coeffs: Dict, sol: Dict, out: Dict):
        s = TrLoFields(E=_ptr(sol["E"]), F=_ptr(sol["F"]), Ebnd=_ptr(sol["Ebnd"]))
        o = TrLoOut()
        for name, _ in TrLoOut._fields_:
            setattr(o, name, _ptr(out[name]))
        _check(self.lib.tr_restrict(self._ctx, frm, to, C.byref(self._coeffs(coeffs)), C.byref(s), C.byref(o),
                                    self._stream()), "tr_restrict")

    def grey_solve(self, grey: Dict, Tstar, Told, dS, Estar, D, T_out, E, F, Ebnd):
        f = TrLoFields(E=_ptr(E), F=_ptr(F), Ebnd=_ptr(Ebnd))
        _check(self.lib.tr_grey_solve(self._ctx, C.byref(self._coeffs(grey)), _ptr(Tstar), _ptr(Told), _ptr(dS),
                                      _ptr(Estar), _ptr(D), _ptr(T_out), C.byref(f), self._stream()),
               "tr_grey_solve")

    # -- state and steps ----------------------------------------------------
    def new_state(self) -> Dict:
        """Device state; the corner intensities are float32 when the context
        stores them in binary32."""
        e = self.empty
        tI = self.torch.float32 if self.precision == 1 else self.torch.float64
        nI = self.total(TR_K_I)
        return dict(T=e(TR_K_CELL), I_prev=self.torch.zeros(nI, dtype=tI, device="cuda"),
                    I_out=self.torch.zeros(nI, dtype=tI, device="cuda"), E=e(TR_K_GI), F=e(TR_K_GE),
                    Ebnd=e(TR_K_G2), f=e(TR_K_GI), fbnd=e(TR_K_G2), C=e(TR_K_G2), Egrey=e(TR_K_CELL))

    @staticmethod
    def _state(st: Dict) -> TrState:
        s = TrState()
        for name, _ in TrState._fields_:
            setattr(s, name, _ptr(st[name]))
        return s

    def state_init(self, st: Dict, T0: float):
        """Initial condition into st; afterwards I_prev holds I^0."""
        _check(self.lib.tr_state_init(self._ctx, C.byref(self._state(st)), float(T0), self._stream()),
               "tr_state_init")
        st["I_prev"], st["I_out"] = st["I_out"], st["I_prev"]

    def step(self, st: Dict, replay: Optional[Sequence[Sequence[int]]] = None, stats=None, swap: bool = True):
        """One time step of every slab; returns the per-slab TrStats array.
        replay: per slab, cycles per transport iteration."""
        if stats is None:
            stats = (TrStats * self.n)()
        rp = None
        if replay is not None:
            arr = np.zeros((self.n, MAXOUT), dtype=np.int32)
            for k, row in enumerate(replay):
                arr[k, :len(row)] = row
            self._replay = arr
            rp = arr.ctypes.data_as(_ip)
        code = self.lib.tr_step(self._ctx, C.byref(self._state(st)), rp, stats, self._stream())
        _check(code, "tr_step")
        if swap:
            st["I_prev"], st["I_out"] = st["I_out"], st["I_prev"]
        return stats

    def alg1_step(self, st: Dict, stats=None, swap: bool = True):
        """One time step of every slab by the single-grid method (Alg. 1);
        returns the per-slab TrStats array."""
        if stats is None:
            stats = (TrStats * self.n)()
        _check(self.lib.tr_alg1_step(self._ctx, C.byref(self._state(st)), stats, self._stream()), "tr_alg1_step")
        if swap:
            st["I_prev"], st["I_out"] = st["I_out"], st["I_prev"]
        return stats

    def run(self, st: Dict, nsteps: int, stats=None):
        """tr_run: nsteps free-running steps in one call; the dict's
        intensity buffers end exchanged as after nsteps calls of step()."""
        if stats is None:
            stats = (TrStats * self.n)()
        done = C.c_int(0)
        code = self.lib.tr_run(self._ctx, C.byref(self._state(st)), int(nsteps), stats,
                               C.cast(C.byref(done), _ip), self._stream())
        if done.value % 2 == 1:
            st["I_prev"], st["I_out"] = st["I_out"], st["I_prev"]
        _check(code, "tr_run")
        return stats

    def prolong(self, level, E_coarse, E_prev, r, E_fine):
        """tr_prolong: E_fine from level `level` energy densities (r: closure
        output [gi][2] float32 or None)."""
        _check(self.lib.tr_prolong(self._ctx, int(level), _ptr(E_coarse), _ptr(E_prev),
                                   _ptr(r) if r is not None else None, _ptr(E_fine), self._stream()), "tr_prolong")

    def set_schedule(self, cycle: int, lmax: int):
        """Cycle (CYCLE_V / W / F over this context's grids) and lmax of the
        following steps (paper Alg. 3; chosen per step by a caller such as
        ``tuning.StageSchedule``)."""
        _check(self.lib.tr_set_schedule(self._ctx, int(cycle), int(lmax)), "tr_set_schedule")
        self.schedule = (int(cycle), int(lmax))

    def set_grids(self, grids, lmax: int):
        """Grids visited after each grey solve (context grid indices, in order)
        and lmax of the following steps (tr_set_grids)."""
        g = np.ascontiguousarray(list(grids), dtype=np.int32)
        _check(self.lib.tr_set_grids(self._ctx, len(g), g.ctypes.data_as(_ip) if len(g) else None, int(lmax)),
               "tr_set_grids")
        self.schedule = (tuple(int(x) for x in g), int(lmax))

    def set_sweep_timing(self, on: bool):
        """Sweeps of tr_step launched with start / end events (kernel time in
        TrStats.t_ms[T_SWEEP]) instead of inside the replayed graphs."""
        _check(self.lib.tr_set_sweep_timing(self._ctx, 1 if on else 0), "tr_set_sweep_timing")


# ---------------------------------------------------------------------------
# Learned closure network (MFMA kernels in the library)
# ---------------------------------------------------------------------------
def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f32(a):
    return (C.c_float * len(a))(*[float(x) for x in a])


class Mlp:
    """Device-side network parameters and Adam state (float32, torch tensors)."""

    def __init__(self, params):
        import torch

        self.torch = torch
        self.lib = load()
        self.nparam = self.lib.tr_mlp_nparam()
        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to("cuda")
        assert p.numel() == self.nparam
        self.params = p.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = C.c_int(0)
        self._work = {}

    def _work_for(self, n, train=False):
        key = (n, train)
        if key not in self._work:
            nb = self.lib.tr_mlp_train_work_bytes(n) if train else self.lib.tr_mlp_work_bytes(n)
            self._work[key] = self.torch.empty(int(nb), dtype=self.torch.uint8, device="cuda")
        return self._work[key]

    def forward(self, X):
        n = X.shape[0]
        out = self.torch.empty((n, 2), dtype=self.torch.float32, device="cuda")
        _check(self.lib.tr_mlp_forward(_ptr(self.params), _ptr(X), n, _ptr(out), _ptr(self._work_for(n)), _stream()),
               "tr_mlp_forward")
        return out

    def grad(self, X, Y):
        n = X.shape[0]
        g = self.torch.empty(self.nparam, dtype=self.torch.float32, device="cuda")
        loss = self.torch.empty(1, dtype=self.torch.float32, device="cuda")
        _check(self.lib.tr_mlp_grad(_ptr(self.params), _ptr(X), _ptr(Y), n, _ptr(g), _ptr(loss),
                                    _ptr(self._work_for(n)), _stream()), "tr_mlp_grad")
        return g, loss

    def grad_noalloc(self, X, Y, g, loss):
        """tr_mlp_grad_noalloc into caller tensors g [nparam], loss [1]."""
        _check(self.lib.tr_mlp_grad_noalloc(_ptr(self.params), _ptr(X), _ptr(Y), X.shape[0], _ptr(g), _ptr(loss),
                                            _stream()), "tr_mlp_grad_noalloc")

    def adam(self, grad, lr):
        self.t.value += 1
        _check(self.lib.tr_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(grad), self.t.value,
                                    C.c_float(lr), _stream()), "tr_mlp_adam")

    def train_epoch(self, X, Y, perm, batch, lr):
        """perm: device int32 tensor; returns the mean batch loss."""
        n = X.shape[0]
        loss = self.torch.zeros(1, dtype=self.torch.float32, device="cuda")
        _check(self.lib.tr_mlp_train_epoch(_ptr(self.params), _ptr(self.m), _ptr(self.v), C.byref(self.t),
                                           C.c_float(lr), _ptr(X), _ptr(Y), n, _ptr(perm), batch,
                                           _ptr(self._work_for(batch, True)), _ptr(loss), _stream()),
               "tr_mlp_train_epoch")
        return float(loss.item()) / max(1, n // batch)


def _solver_methods():
    def mlp_features(self, T, T_prev, kappa, f, mean, std, X):
        """Closure inputs (T_prev may be None: no temperature change)."""
        _check(self.lib.tr_mlp_features(self._ctx, _ptr(T), _ptr(T_prev), _ptr(kappa), _ptr(f), _f32(mean),
                                        _f32(std), _ptr(X), self._stream()), "tr_mlp_features")

    def closure_targets(self, f, f_prev, E_new, E_prev, block, Y):
        _check(self.lib.tr_closure_targets(self._ctx, _ptr(f), _ptr(f_prev), _ptr(E_new), _ptr(E_prev), int(block),
                                           _ptr(Y), self._stream()), "tr_closure_targets")

    def closure_seed(self, T, T_prev, kappa, f, counts):
        """The attached closure's s = 0 seeding of f in place (T_prev may be
        None); counts: int64 device tensor [2] (seeded, kept), accumulated."""
        _check(self.lib.tr_closure_seed(self._ctx, _ptr(T), _ptr(T_prev), _ptr(kappa), _ptr(f), _ptr(counts),
                                        self._stream()), "tr_closure_seed")

    def set_closure(self, mlp, mean=None, std=None):
        if mlp is None:
            _check(self.lib.tr_set_closure(self._ctx, None, None, None), "tr_set_closure")
            self._closure = None
            return
        _check(self.lib.tr_set_closure(self._ctx, _ptr(mlp.params), _f32(mean), _f32(std)), "tr_set_closure")
        self._closure = mlp

    def autotune(self, st, reps=3):
        """Times the sweep tiles (K, split) per slab-size bucket; returns
        (K[6], split[6], us[6][12]) with tile q = (K index q // 3, split index q % 3)."""
        K, S = (C.c_int * 6)(), (C.c_int * 6)()
        us = (C.c_double * 72)()
        _check(self.lib.tr_autotune(self._ctx, _ptr(st["I_prev"]), _ptr(st["I_out"]), reps, K, S, us,
                                    self._stream()), "tr_autotune")
        return list(K), list(S), [list(us[12 * b:12 * b + 12]) for b in range(6)]

    def set_tiles(self, K, split=None):
        arr = (C.c_int * 6)(*[int(k) for k in K])
        sp = None if split is None else (C.c_int * 6)(*[int(k) for k in split])
        _check(self.lib.tr_set_tiles(self._ctx, arr, sp), "tr_set_tiles")

    def get_tiles(self):
        """(K[6], split[6], items[6]) of the current sweep tiles."""
        K, S, n = (C.c_int * 6)(), (C.c_int * 6)(), (C.c_int * 6)()
        _check(self.lib.tr_get_tiles(self._ctx, K, S, n), "tr_get_tiles")
        return list(K), list(S), list(n)

    Solver.autotune = autotune
    Solver.set_tiles = set_tiles
    Solver.get_tiles = get_tiles
    Solver.mlp_features = mlp_features
    Solver.closure_targets = closure_targets
    Solver.set_closure = set_closure
    Solver.closure_seed = closure_seed


_solver_methods()
