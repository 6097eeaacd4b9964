"""Benchmark: converged backward-Euler time steps of the MLQD method with
multigrid in frequency on one MI355X.

A "step" is one converged time step of the whole hot path (opacity/Planck
tables, SCB transport sweeps with their moments, fine and coarse LO solves,
restriction, grey LO + MEB Newton, cycle control) over the workload's slabs.
The default (headline) workload is the large single problem: 2000 cells, S32,
4096 log groups, F cycle on the hierarchy 4096,1024,256,64,16,1, dt = 0.002
ns; the timed region is --steps steps from the initial condition (inputs
resident in HBM).  The paper-scale slab (200 cells, S16, 512 groups, V cycle)
and the batch of 256 uneven slabs are measured in the same run and reported
under their own keys.

Printed: one JSON line with the throughput in phase-space cell-updates per
second (sweep cell-updates of the timed steps / wall time), ms per step, the
live-measured roofline of the sweep kernel (HIP events around its launches,
algorithmic bytes per launch / average launch time), the fraction of the HBM
peak of the restriction and fine LO kernel groups, the learned closure vs the
plain method, and the CPU oracle timed on a bounded sample (one thread and all
cores).
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "paper": ("config_paper_scale",
              "paper-scale slab: 200 cells, S16 Gauss-Legendre, 512 log groups on [0.01,100] keV, "
              "V cycle on 512,128,32,8,1, dt=0.002 ns, eps=1e-10"),
    "small": ("config_small",
              "small slab: 50 cells, S8, 16 groups, two-grid V 16,1, dt=0.002 ns, eps=1e-10"),
    "large": ("config_large",
              "large slab: 2000 cells, S32, 4096 groups, F cycle on 4096,1024,256,64,16,1, dt=0.002 ns, "
              "eps=1e-10"),
    "batch": ("config_batch",
              "batch of 256 uneven slabs (seed 201105427): nx in [50,400], groups in {64..1024}, S8/S16, "
              "zone opacity constants log-uniform in [1,100], T_left in [0.5,1.5], W cycle G,G/8,1, "
              "autotuned sweep tiles"),
}
KERNELS = ["opacity", "sweep", "moments", "lo_fine", "restrict", "lo_coarse", "grey"]
LMAX_CANDIDATES = (1, 2, 4)  # cycles per transport iteration tried in the set-up


def lo_fine_bytes(slab, n_cycles, n_sweeps):
    """Algorithmic HBM bytes of the fine LO solves: per (group, cell) and
    solve read the QD factor, kappa, B, E_old and F_old and write E and F (56
    B); the first solve after each sweep reads the two half-range moment
    partial pairs instead of the factor (32 B instead of 8) and writes the
    factor (8 B)."""
    gi = slab.ng * slab.nx
    return 56.0 * gi * n_cycles + 32.0 * gi * n_sweeps


def restrict_bytes(slab, n_stage_levels, n_cycles, n_steps):
    """Algorithmic HBM bytes of the fine-grid restrictions: per (group, edge)
    and cycle the fine-to-grey pass reads the QD factor, kappa, B, E and F (40
    B) and every stage of the schedule reads the factor, E and F (24 B; kappa
    and B at the stage temperature are recomputed); the first cycle of a step
    also reads E_old and F_old (16 B) once per target grid.  The coarse-to-grey
    passes read the coarse levels (under 1/4 of the fine bytes) and are not
    counted."""
    ge = slab.ng * (slab.nx + 1)
    return (40.0 + 24.0 * n_stage_levels) * ge * n_cycles + 16.0 * (1 + n_stage_levels) * ge * n_steps


from paper_2011_05427_amd.profsum import measured_traffic, sweep_bytes  # noqa: E402


def cpu_baseline(workload, budget_s=20.0, lmax=None):
    """The CPU oracle (numpy, FP64) on a bounded sample of the workload, in a
    child process that never touches the GPU (BLAS / OpenMP pools limited to
    one thread per process)."""
    import subprocess

    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", workload, "--cpu-budget", str(budget_s)]
    if lmax is not None:
        cmd += ["--cpu-lmax", str(lmax)]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _host_cpus():
    """(usable cores, cores reported by the OS, model name) of this host."""
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return usable, os.cpu_count() or usable, model


_SWEEP_JOB = {}


def _sweep_chunk(bounds):
    """Oracle sweep of groups [g0, g1) of the prepared initial state (worker
    of the all-cores baseline; the inputs are inherited from the parent)."""
    from oracle.sweep import sweep

    g0, g1 = bounds
    j = _SWEEP_JOB
    t0 = time.perf_counter()
    out = sweep(j["mu"], j["x"], j["kappa"][g0:g1], j["B"][g0:g1], j["I"][g0:g1], j["il"][g0:g1], j["ir"][g0:g1],
                j["c"], j["dt"])
    return time.perf_counter() - t0, float(out[:, :, -1, 1].sum())


def _cpu_baseline_child(workload, budget_s, lmax=None):
    from oracle import mlqd
    from paper_2011_05427_amd import inputs

    slabs, cfg, _ = getattr(inputs, WORKLOADS[workload][0])()
    if lmax is not None:
        cfg = dataclasses.replace(cfg, lmax=lmax)  # the GPU run's choice
    usable, nproc, model = _host_cpus()
    host = {"nproc": nproc, "usable_cores": usable, "cpu_model": model}
    if workload == "batch":
        # the oracle on the first slabs of the batch, one step each, within the budget
        t0 = time.perf_counter()
        cu, k = 0, 0
        for slab in slabs:
            pb = mlqd.problem_from_slab(slab)
            st = mlqd.initial_state(pb, slab.T0)
            stats = mlqd.Stats()
            lv = inputs.levels_for(slab, cfg)
            sched = mlqd.schedule(len(lv), cfg.cycle)
            mlqd.step(pb, lv, sched, cfg.lmax, cfg.eps, cfg.eps_inner, st, stats=stats)
            cu += slab.cell_updates_per_sweep() * stats.n_ti
            k += 1
            if time.perf_counter() - t0 > budget_s * 0.5:
                break
        dt = time.perf_counter() - t0
        return dict(host, value=cu / dt, unit="cell-updates/s", cores=1, kind="oracle",
                    sample=f"first time step of the first {k} slabs of the batch, numpy FP64, one thread, {dt:.1f} s")
    slab = slabs[0]
    pb = mlqd.problem_from_slab(slab)
    if slab.cell_updates_per_sweep() > 5e7:
        # a whole step of this size takes minutes in the oracle: one transport
        # sweep of the initial state (every group and direction), on one thread
        # and split over processes by group (the sweep of a group is
        # independent of the others given the tables)
        import multiprocessing as mp

        st = mlqd.initial_state(pb, slab.T0)
        kappa, B = pb.tables(st.T)
        _SWEEP_JOB.update(mu=pb.mu, x=pb.x_edges, kappa=kappa, B=B, I=st.I, il=pb.inc_left, ir=pb.inc_right,
                          c=pb.c, dt=pb.dt)
        t1, _ = _sweep_chunk((0, slab.ng))
        workers = max(1, min(usable, 16))
        cuts = [round(k * slab.ng / workers) for k in range(workers + 1)]
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(workers) as pool:
            pool.map(_sweep_chunk, list(zip(cuts[:-1], cuts[1:])))
        tn = time.perf_counter() - t0
        cu = slab.cell_updates_per_sweep()
        return dict(host, value=cu / tn, unit="cell-updates/s", cores=workers, kind="oracle",
                    sample=f"one transport sweep of the workload's initial state (all {slab.ng} groups x "
                           f"{slab.nmu} directions x {slab.nx} cells), numpy FP64: {tn:.1f} s on {workers} "
                           f"processes over group ranges (incl. pool start-up), {t1:.1f} s on one thread; "
                           f"a whole oracle step of this size is not timed (minutes)",
                    one_thread={"value": cu / t1, "unit": "cell-updates/s", "cores": 1, "seconds": t1})
    st = mlqd.initial_state(pb, slab.T0)
    stats = mlqd.Stats()
    t0 = time.perf_counter()
    nsteps = 0
    while True:
        st = mlqd.step(pb, cfg.levels, mlqd.schedule(len(cfg.levels), cfg.cycle), cfg.lmax, cfg.eps,
                       cfg.eps_inner, st, stats=stats)
        nsteps += 1
        if time.perf_counter() - t0 > budget_s * 0.5:
            break
    dt = time.perf_counter() - t0
    return dict(host, value=slab.cell_updates_per_sweep() * stats.n_ti / dt, unit="cell-updates/s", cores=1,
                kind="oracle", ms_per_step=1e3 * dt / nsteps,
                sample=f"first {nsteps} time step(s) of the same workload ({stats.n_ti} sweeps), numpy FP64, "
                       f"one thread, {dt:.1f} s")


def run_steps(slabs, levels, cfg, steps, warmup, timing=False, tiles=None, closure=None, final=None, sweep_ev=0):
    """Runs warmup steps, then `steps` steps from the initial condition; returns
    (wall seconds, per-slab TrStats); with a dict `final`, the final T and E
    are copied into it.  The first `sweep_ev` timed steps launch their sweeps
    with start / end events (the sweep kernel's duration, in TrStats.t_ms)."""
    import torch

    from paper_2011_05427_amd import binding

    sv = binding.Solver(slabs, levels, cfg, timing=timing)
    if tiles is not None:
        sv.set_tiles(*tiles)
    if closure is not None:
        sv.set_closure(*closure)
    st = sv.new_state()
    sv.state_init(st, slabs[0].T0)
    if sweep_ev:
        sv.set_sweep_timing(True)  # warmup also builds the graphs of timed steps
    for _ in range(warmup):
        sv.step(st)
    if sweep_ev:
        sv.set_sweep_timing(False)
    sv.state_init(st, slabs[0].T0)
    torch.cuda.synchronize()
    acc = (binding.TrStats * len(slabs))()
    acc_ev = (binding.TrStats * len(slabs))()
    t0 = time.perf_counter()
    for _ in range(min(steps, sweep_ev)):
        # this step's sweeps are timed: its counters also go to acc_ev
        sv.set_sweep_timing(True)
        one = sv.step(st)
        for q in range(len(slabs)):
            for dst in (acc[q], acc_ev[q]):
                for f in ("n_ti", "n_c", "n_lo", "n_floor", "n_seeded", "n_fallback"):
                    setattr(dst, f, getattr(dst, f) + getattr(one[q], f))
                for i in range(len(dst.t_ms)):
                    dst.t_ms[i] += one[q].t_ms[i]
                    dst.n_launch[i] += one[q].n_launch[i]
        sv.set_sweep_timing(False)
    if steps > sweep_ev:
        sv.run(st, steps - sweep_ev, stats=acc)  # the remaining steps in one library call
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if final is not None:
        final["T"] = st["T"].cpu().numpy()
        final["E"] = st["E"].cpu().numpy()
    sv.close()
    if sweep_ev:
        return wall, acc, acc_ev
    return wall, acc


def train_closure(args):
    """Trains the closure on the plain solver's own steps of the paper-scale
    workload (its 20 steps, a bounded sample of (group, cell) pairs)."""
    from paper_2011_05427_amd import closure, inputs

    t0 = time.perf_counter()
    train_slabs, train_cfg, train_steps = inputs.config_paper_scale()
    ds = closure.generate(train_slabs[0], train_cfg, train_cfg.levels, nsteps=train_steps,
                          n_samples=args.train_samples, seed=0)
    net, losses = closure.train(ds, epochs=args.train_epochs, batch=4096, lr=1e-3, seed=0)
    return {"net": net, "ds": ds, "losses": losses, "train_s": time.perf_counter() - t0,
            "epochs": args.train_epochs}


def learned_vs_plain(slabs, levels, cfg, tiles, steps, warmup, plain_ms, plain_sweeps, trained):
    """Times a workload's steps with the trained closure seeding each step's
    factors (the plain sweeps still decide convergence)."""
    ds = trained["ds"]
    wall, acc = run_steps(slabs, levels, cfg, steps, warmup, tiles=tiles, closure=(trained["net"], ds.mean, ds.std))
    ms = 1e3 * wall / steps
    return {"ms_per_step": ms, "plain_ms_per_step": plain_ms, "speedup": plain_ms / ms,
            "sweeps": int(sum(a.n_ti for a in acc)), "plain_sweeps": plain_sweeps,
            "seeded": int(sum(a.n_seeded for a in acc)), "fallback": int(sum(a.n_fallback for a in acc)),
            "train_s": trained["train_s"], "samples": int(ds.X.shape[0]), "epochs": trained["epochs"],
            "loss_first": trained["losses"][0], "loss_last": trained["losses"][-1],
            "note": "network trained on the paper-scale workload's plain steps; at the start of every step it "
                    "seeds the cell factors with its predicted change; the plain sweeps decide convergence"}


def hierarchy_candidates(nlev):
    """(grids, lmax) candidates: the two-grid cycle, W through each
    intermediate grid, the coarsest intermediate grid with each finer one,
    the full F, and lmax 2 through the coarsest and the finest intermediate
    grid (grid indices of the workload's hierarchy)."""
    mid = list(range(1, nlev - 1))
    cands = [((), 1)] + [((g,), 1) for g in mid]
    if len(mid) > 1:
        cands += [((mid[-1], g), 1) for g in mid[:-1]] + [(tuple(reversed(mid)), 1)]
        cands += [((mid[-1],), 2), ((mid[0],), 2)]
    elif mid:
        cands += [((mid[0],), 2)]
    return list(dict.fromkeys(cands))


def run_stage_adaptive(slabs, levels, cfg, steps, warmup, tiles):
    """The same steps with the grid hierarchy and lmax chosen per step by
    ``tuning.CostModelSchedule``.  Untimed set-up: the sweep kernel time, and
    every candidate's first 2 steps from the initial state (after 2 steps
    that capture its graphs), which seed the model's cycle costs with
    measurements over the same steps; the sweep ratios start at 1 (the
    set-up's transient steps overstate their differences) and are learned
    from the timed steps."""
    import torch

    from paper_2011_05427_amd import binding, tuning

    cands = hierarchy_candidates(len(levels[0]))
    sv = binding.Solver(slabs, levels, cfg)
    sv.set_tiles(*tiles)
    st = sv.new_state()
    sv.state_init(st, slabs[0].T0)
    t_sweep = tuning.measure_sweep_ms(sv, st)
    seed = {}
    for cand in cands:
        tuning.apply_schedule(sv, cand)
        sv.state_init(st, slabs[0].T0)
        for _ in range(max(warmup, 2)):
            sv.step(st)
        sv.state_init(st, slabs[0].T0)
        acc = (binding.TrStats * len(slabs))()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            sv.step(st, stats=acc)
        torch.cuda.synchronize()
        seed[cand] = (1e3 * (time.perf_counter() - t0), max(int(a.n_ti) for a in acc),
                      max(int(a.n_c) for a in acc), 2)
    sv.state_init(st, slabs[0].T0)
    ctl = tuning.CostModelSchedule(cands, t_sweep=t_sweep, seed=seed, ratio_prior=1.0)
    torch.cuda.synchronize()
    acc = (binding.TrStats * len(slabs))()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctl.step(sv, st, stats=acc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sv.close()
    name = lambda c: ("grids" + ",".join(str(levels[0][g]) for g in c[0]) if c[0] else "two-grid") + f"/l{c[1]}"
    return {"ms_per_step": 1e3 * wall / steps,
            "value": sum(s.cell_updates_per_sweep() * int(a.n_ti) for s, a in zip(slabs, acc)) / wall,
            "sweeps": int(sum(a.n_ti for a in acc)), "cycles": int(sum(a.n_c for a in acc)),
            "t_sweep_ms": t_sweep, "choices": [name(c) for c, *_ in ctl.history],
            "candidates": [name(c) for c in cands],
            "set_up_ms_per_step": {name(c): v[0] / v[3] for c, v in seed.items()},
            "note": "hierarchy (grids visited after each grey solve) and lmax per step from the cost model "
                    "s t_sweep + (s + 1) k_c t_c, cycle costs seeded by every candidate's first 2 steps from "
                    "the initial state (untimed), sweep ratios starting at 1 and learned from the timed steps; "
                    "every 8th step re-measures a candidate predicted within 25% of the best"}


def measure(workload, steps, warmup, tiles_opt=None, lmax_opt=None, fp32=False):
    """Set-up (sweep tiles, lmax), the timed steps and an event-timed rerun of
    the same steps for one workload; returns (result dict, internals)."""
    import torch

    from paper_2011_05427_amd import binding, inputs, tuning

    fn, desc = WORKLOADS[workload]
    slabs, cfg, _ = getattr(inputs, fn)()
    levels = [inputs.levels_for(s, cfg) for s in slabs]

    # sweep tiles (cells per lane, wavefronts per group and half range) chosen
    # by the autotuner on this workload's first state (untimed set-up)
    sv = binding.Solver(slabs, levels, cfg)
    st = sv.new_state()
    sv.state_init(st, slabs[0].T0)
    t0 = time.perf_counter()
    if tiles_opt:
        ks, ss = tiles_opt.split(":")
        tiles = ([int(v) for v in ks.split(",")], [int(v) for v in ss.split(",")])
        sv.set_tiles(*tiles)
        tune_info = {"K": tiles[0], "split": tiles[1], "us": None, "fixed": True}
    else:
        tune_info = tuning.tune(sv, st, reps=3, path=None)
        tiles = (tune_info["K"], tune_info["split"])
    tune_info["tune_s"] = time.perf_counter() - t0
    # lmax of the workload's cycle chosen from the measured cost of its first
    # steps (untimed set-up, tr_set_schedule); the workload fixes the cycle
    # and the tolerances, not lmax
    cfg_lmax = cfg.lmax
    cands = [(cfg.cycle, l) for l in LMAX_CANDIDATES]
    if lmax_opt is not None:
        sched_ms = None
        cfg = dataclasses.replace(cfg, lmax=lmax_opt)
    else:
        sched_ms = tuning.tune_schedule(sv, st, cands, steps=2)
        cfg = dataclasses.replace(cfg, lmax=next(iter(sched_ms))[1])
    sv.close()
    del st
    torch.cuda.empty_cache()

    # timed: graph replay, no events, except that the first steps also time
    # their sweep launches
    fin64 = {}
    n_ev = max(1, steps // 10)
    wall, acc, acc_ev = run_steps(slabs, levels, cfg, steps, warmup, tiles=tiles, final=fin64, sweep_ev=n_ev)
    # per-kernel durations: the same steps with HIP events around each kernel
    # group (eager launches, not part of the timed value)
    _, prof = run_steps(slabs, levels, cfg, steps, 0, timing=True, tiles=tiles)

    sweeps = [int(acc[k].n_ti) for k in range(len(slabs))]
    cu = sum(s.cell_updates_per_sweep() * n for s, n in zip(slabs, sweeps))
    p = prof[0]  # kernel-group times cover the whole context
    t_sweep_s = acc_ev[0].t_ms[binding.T_SWEEP] / 1e3
    n_sweep = acc_ev[0].n_launch[binding.T_SWEEP]
    bytes_total = sum(sweep_bytes(s) * int(acc_ev[k].n_ti) for k, s in enumerate(slabs))
    achieved = bytes_total / t_sweep_s / 1e9 if t_sweep_s > 0 else 0.0
    kernel_ms = {name: p.t_ms[k] / max(steps, 1) for k, name in enumerate(KERNELS)}
    # HBM fractions of the restriction and fine LO kernel groups over the
    # event-timed steps (algorithmic bytes from the per-slab counts)
    nstage = [len(mlqd_schedule(len(lv), cfg.cycle)) for lv in levels]
    rb = sum(restrict_bytes(s, ns, int(a.n_c), steps) for s, ns, a in zip(slabs, nstage, prof))
    lb = sum(lo_fine_bytes(s, int(a.n_c), int(a.n_ti)) for s, a in zip(slabs, prof))
    groups = {}
    for name, idx, nbytes in (("restrict", binding.T_RESTRICT, rb), ("lo_fine", binding.T_LO_FINE, lb)):
        t = p.t_ms[idx] / 1e3
        gbs = nbytes / t / 1e9 if t > 0 else None
        groups[name] = {"bytes_per_step": nbytes / steps, "ms_per_step": 1e3 * t / steps, "achieved_GBs": gbs,
                        "frac": gbs / HBM_PEAK_GBS if gbs else None, "launches": int(p.n_launch[idx])}
    ms_step = 1e3 * wall / steps
    res = {
        "value": cu / wall,
        "ms_per_step": ms_step,
        "config": {
            "workload": desc,
            "slabs": len(slabs),
            "cell_updates_per_sweep": sum(s.cell_updates_per_sweep() for s in slabs),
            "levels": levels[0] if len(slabs) == 1 else "per slab G,G/8,1",
            "cycle": "VWF"[cfg.cycle], "lmax": cfg.lmax, "eps": cfg.eps, "eps_inner": cfg.eps_inner,
            "steps_timed": steps, "sweeps": sum(sweeps), "cycles": int(sum(a.n_c for a in acc)),
            "lo_solves": int(sum(a.n_lo for a in acc)), "closure": "plain",
        },
        "kernel_ms_per_step": kernel_ms,
        "kernel_groups_hbm": groups,
        "sweep_kernel_cell_updates_per_s": (sum(s.cell_updates_per_sweep() * int(acc_ev[k].n_ti)
                                                for k, s in enumerate(slabs)) / t_sweep_s) if t_sweep_s else None,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": bytes_total / max(n_sweep, 1),
            "avg_launch_us": 1e6 * t_sweep_s / max(n_sweep, 1),
            "launches": int(n_sweep),
            "timed_steps": n_ev,
            "note": "kernel start/end events of the sweep launches in the first timed steps; "
                    "achieved = algorithmic bytes (32 B per cell-update + 32 B per group-cell of moment "
                    "partials) / kernel time",
        },
        "tiles": {"K_per_bucket": tune_info["K"], "split_per_bucket": tune_info["split"],
                  "us_per_tile": tune_info["us"], "fixed_by_option": bool(tune_info.get("fixed")),
                  "tile_order": "q = (K in 1,2,4,8)[q // 3], (split in 1,2,4)[q % 3]",
                  "buckets": tuning.BUCKETS, "tune_s": tune_info["tune_s"]},
        "schedule": {
            "lmax_chosen": cfg.lmax, "lmax_configured": cfg_lmax,
            "set_up_ms_per_step": ({f"{'VWF'[c]}{l}": ms for (c, l), ms in sched_ms.items()} if sched_ms else None),
            "set_up": ("2 steps from the initial state per candidate, after 2 untimed steps that capture its graphs"
                       if sched_ms else "fixed by --lmax"),
        },
    }
    tr = measured_traffic(workload, res["roofline"]["bytes_per_launch"])
    if tr is not None:
        res["roofline"]["traffic"] = tr["bytes_per_launch"]
        res["roofline"]["traffic_detail"] = tr
    if fp32:
        import numpy as np

        cfg32 = dataclasses.replace(cfg, precision=1)
        fin32 = {}
        wall32, acc32, ev32 = run_steps(slabs, levels, cfg32, steps, warmup, tiles=tiles, final=fin32,
                                        sweep_ev=n_ev)
        t32 = ev32[0].t_ms[binding.T_SWEEP] / 1e3
        b32 = sum(sweep_bytes(s, 4) * int(ev32[k].n_ti) for k, s in enumerate(slabs))
        rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        res["fp32_storage"] = {
            "ms_per_step": 1e3 * wall32 / steps,
            "value": sum(s.cell_updates_per_sweep() * int(acc32[k].n_ti) for k, s in enumerate(slabs)) / wall32,
            "sweeps": int(sum(a.n_ti for a in acc32)),
            "sweep_achieved_GBs": b32 / t32 / 1e9 if t32 > 0 else None,
            "sweep_frac_of_hbm": b32 / t32 / 1e9 / HBM_PEAK_GBS if t32 > 0 else None,
            "max_rel_err_T_vs_f64": rel(fin32["T"], fin64["T"]),
            "max_rel_err_E_vs_f64": rel(fin32["E"], fin64["E"]),
            "note": "corner intensities stored in binary32; sweep arithmetic, moments, LO, grey and MEB in binary64",
        }
    internals = dict(slabs=slabs, levels=levels, cfg=cfg, tiles=tiles, cands=cands, sched_ms=sched_ms,
                     sweeps=sum(sweeps))
    return res, internals


def fixed_hierarchies(slabs, levels, cfg, steps, tiles):
    """ms per step, sweeps and cycles of fixed grid hierarchies (the grids
    visited after each grey solve, tr_set_grids) and lmax over the same steps
    from the initial condition, after 2 untimed steps that capture each one's
    graphs: the two-grid cycle, W through each intermediate grid, pairs, the
    full F, and lmax 2 for the best single grids."""
    import torch

    from paper_2011_05427_amd import binding, tuning

    cands = hierarchy_candidates(len(levels[0]))
    sv = binding.Solver(slabs, levels, cfg)
    sv.set_tiles(*tiles)
    st = sv.new_state()
    out = {}
    for cand in cands:
        tuning.apply_schedule(sv, cand)
        sv.state_init(st, slabs[0].T0)
        for _ in range(2):
            sv.step(st)
        sv.state_init(st, slabs[0].T0)
        torch.cuda.synchronize()
        acc = (binding.TrStats * len(slabs))()
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.step(st, stats=acc)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        name = (",".join(str(levels[0][g]) for g in cand[0]) or "two-grid") + f"/l{cand[1]}"
        out[name] = {"ms_per_step": ms, "sweeps": int(sum(a.n_ti for a in acc)),
                     "cycles": int(sum(a.n_c for a in acc)), "lo_group_solves": int(sum(a.n_lo for a in acc))}
    sv.close()
    return out


def alg1_vs_cycles(slabs, cfg, candidates, steps, warmup=1):
    """Time-to-solution of the single-grid method (Alg. 1, tr_alg1_step) and
    of multigrid cycles on the same steps from the initial condition:
    candidates = [(name, levels, cycle, lmax)].  Reports ms per step, sweeps,
    low-order work and the largest relative difference of the final T from
    Alg. 1's."""
    import numpy as np
    import torch

    from paper_2011_05427_amd import binding

    def run(levels, cyc, lmax, alg1):
        c = dataclasses.replace(cfg, levels=levels, cycle=cyc, lmax=lmax)
        sv = binding.Solver(slabs, [levels] * len(slabs), c)
        st = sv.new_state()
        sv.state_init(st, slabs[0].T0)
        for _ in range(warmup):  # workspace, graphs
            sv.alg1_step(st) if alg1 else sv.step(st)
        sv.state_init(st, slabs[0].T0)
        acc = (binding.TrStats * len(slabs))()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.alg1_step(st, stats=acc) if alg1 else sv.step(st, stats=acc)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        T = st["T"].cpu().numpy().copy()
        sv.close()
        return {"ms_per_step": 1e3 * wall / steps, "sweeps": int(sum(a.n_ti for a in acc)),
                ("newton_iterations" if alg1 else "cycles"): int(sum(a.n_c for a in acc)),
                "lo_group_solves": int(sum(a.n_lo for a in acc))}, T

    fine = candidates[0][1][0]
    out = {}
    a1, Ta = run([fine, 1], 0, 1, True)
    out["alg1"] = a1
    for name, levels, cyc, lmax in candidates:
        r, Tm = run(levels, cyc, lmax, False)
        r["max_rel_dT_vs_alg1"] = float(np.max(np.abs(Tm - Ta) / np.abs(Ta)))
        r["speedup_vs_alg1"] = a1["ms_per_step"] / r["ms_per_step"]
        out[name] = r
    return out


def mlqd_schedule(n_levels, cycle):
    """Grids visited after each grey solve in one cycle (the library's own
    rule: V none, W the second grid, F every intermediate grid); used only to
    count the restriction passes of the byte model."""
    if cycle == 0 or n_levels <= 2:
        return []
    if cycle == 1:
        return [1]
    return list(range(n_levels - 2, 0, -1))


EXTRA_STEPS = {"paper": 20, "batch": 4}


def progress(msg):
    """One line per finished phase on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--extras", default="paper,batch",
                    help="other workloads measured in the same run (comma list, '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-baseline-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-lmax", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--lmax", type=int, default=None,
                    help="use this lmax instead of the set-up choice (e.g. to profile a plain run's choice)")
    ap.add_argument("--tiles", default=None,
                    help="sweep tiles 'K1,..,K6:S1,..,S6' per slab-size bucket instead of the autotuner's")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-closure comparison")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the stage-adaptive schedule run")
    ap.add_argument("--no-alg1", action="store_true", help="skip the single-grid (Alg. 1) comparison")
    ap.add_argument("--hierarchies", action="store_true",
                    help="also time fixed grid hierarchies of the workload over the same steps")
    ap.add_argument("--train-samples", type=int, default=1000000)
    ap.add_argument("--train-epochs", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device copy (reference kernel for the HBM byte counters)")
    ap.add_argument("--fp32", action="store_true",
                    help="also time the binary32-storage sweep variant and state its error vs binary64")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        print(json.dumps(_cpu_baseline_child(args.cpu_baseline_child, args.cpu_budget, args.cpu_lmax)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 "
                                   "(sharding over GPUs is described in the design notes, not built)"}))
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.steps is None:
        args.steps = {"paper": 20, "small": 1, "large": 50, "batch": 4}[args.workload]
    res, ins = measure(args.workload, args.steps, args.warmup, args.tiles, args.lmax, args.fp32)
    progress(f"{args.workload}: {res['ms_per_step']:.3f} ms per step")
    out = {
        "metric": "phase-space cell-updates/s per sweep; ms per converged time step, learned vs plain",
        "value": res.pop("value"),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
    }
    out.update(res)
    if not args.no_adaptive:
        out["stage_adaptive"] = run_stage_adaptive(ins["slabs"], ins["levels"], ins["cfg"], args.steps, args.warmup,
                                                   ins["tiles"])
        progress("stage-adaptive run done")
    if args.hierarchies:
        out["fixed_hierarchies"] = fixed_hierarchies(ins["slabs"], ins["levels"], ins["cfg"], args.steps,
                                                     ins["tiles"])
        progress("fixed hierarchies done")
    trained = None
    if not args.no_learned:
        trained = train_closure(args)
        out["learned"] = learned_vs_plain(ins["slabs"], ins["levels"], ins["cfg"], ins["tiles"], args.steps,
                                          args.warmup, out["ms_per_step"], ins["sweeps"], trained)
        progress("learned closure run done")
    torch.cuda.empty_cache()
    for extra in [e for e in args.extras.split(",") if e and e != args.workload]:
        r, xi = measure(extra, EXTRA_STEPS.get(extra, 4), args.warmup)
        r["steps"] = EXTRA_STEPS.get(extra, 4)
        if trained is not None and extra == "batch":
            # the learned closure on the batched shapes as well
            r["learned"] = learned_vs_plain(xi["slabs"], xi["levels"], xi["cfg"], xi["tiles"], r["steps"],
                                            args.warmup, r["ms_per_step"], xi["sweeps"], trained)
        if not args.no_cpu_baseline:
            r["cpu_baseline"] = cpu_baseline(extra, args.cpu_budget, xi["cfg"].lmax)
        out[{"paper": "paper_scale"}.get(extra, extra)] = r
        progress(f"{extra}: {r['ms_per_step']:.3f} ms per step")
        torch.cuda.empty_cache()
    if not args.no_alg1:
        from paper_2011_05427_amd import inputs

        ps, pcfg, _ = inputs.config_paper_scale()
        lv = pcfg.levels
        out["single_grid_vs_multigrid"] = {
            "note": "Alg. 1 (single-grid multigroup LOQD + MEB by Newton on the device) against the multigrid "
                    "cycles on the same steps from the initial condition; eps of each workload",
            "paper_scale": dict(alg1_vs_cycles(ps, pcfg, [("V1", lv, 0, 1), ("W1", lv, 1, 1), ("F1", lv, 2, 1)],
                                               steps=5), steps=5, levels=lv),
        }
        fs, fcfg, _ = inputs.config_fc(0.02)
        out["single_grid_vs_multigrid"]["fleck_cummings"] = dict(
            alg1_vs_cycles(fs, fcfg, [("V4", [256, 1], 0, 4), ("W2", [256, 32, 1], 1, 2),
                                      ("F2", [256, 32, 16, 1], 2, 2), ("F1_6grids", [256, 128, 64, 32, 16, 1], 2, 1)],
                           steps=20),
            steps=20, dt=0.02, opacity="spectral group averages")
        progress("single grid vs multigrid done")
        torch.cuda.empty_cache()
    if args.copy_calibration:
        # a plain device copy of known size for the byte-counter calibration
        # (outside every timed region)
        n = 1 << 27
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": 8 * n, "bytes_written": 8 * n, "launches": 3}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget, ins["cfg"].lmax)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
