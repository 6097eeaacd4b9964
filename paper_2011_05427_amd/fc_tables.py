"""The paper's algorithm comparison (Sec. 6, Tables 1 and 2) on the GPU.

Runs the Fleck-Cummings set-up (``inputs.fc_slab``) to t = 3 ns with every
hierarchy, cycle and lmax of the two tables and prints the totals of transport
iterations N_ti, cycles N_c and low-order solves N_lo beside the printed ones,
with the GPU time per step.  The group opacities are the paper's spectral
averages (sigma_B,g, sigma_E,g at the radiation temperature, Rosseland
sigma_R,g; --opacity point: the point law at the group centre).  The
radiation temperature and the Newton details are readings, so the counts are
compared as context, not as a parity check.

    python -m paper_2011_05427_amd.fc_tables [--tables 1 2] [--opacity spectral|point] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import os
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLES = os.path.join(ROOT, "tests", "golden", "paper_tables.json")


def run_row(row, tiles=None, opacity=1):
    """One table row on the GPU; returns its totals and timing."""
    import torch

    from paper_2011_05427_amd import binding, inputs

    dt = 0.02 if row["table"] == 1 else 0.04
    cyc = {"V": inputs.CYCLE_V, "W": inputs.CYCLE_W, "F": inputs.CYCLE_F}[row["cycle"]]
    slabs, cfg, nsteps = inputs.config_fc(dt, row["levels"], cyc, row["lmax"], opacity=opacity)
    assert nsteps == row["steps"]
    sv = binding.Solver(slabs, [cfg.levels], cfg)
    if tiles is not None:
        sv.set_tiles(*tiles)
    st = sv.new_state()
    sv.state_init(st, slabs[0].T0)
    acc = (binding.TrStats * 1)()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        sv.step(st, stats=acc)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T = st["T"].cpu().numpy().copy()
    sv.close()
    return {"N_ti": int(acc[0].n_ti), "N_c": int(acc[0].n_c), "N_lo": int(acc[0].n_lo),
            "ms_per_step": 1e3 * wall / nsteps, "T_max": float(T.max()), "T_min": float(T.min())}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--tables", type=int, nargs="*", default=[1, 2])
    ap.add_argument("--json", default=None)
    ap.add_argument("--opacity", choices=["spectral", "point"], default="spectral")
    args = ap.parse_args(argv)
    opac = 1 if args.opacity == "spectral" else 0
    rows = [r for r in json.load(open(TABLES))["rows"] if r["table"] in args.tables]
    out = []
    print("| table | grids | cycle | lmax | paper N_ti / N_c / N_lo | GPU N_ti / N_c / N_lo | ms per step |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        g = run_row(r, opacity=opac)
        out.append({"paper": r, "gpu": g})
        print(f"| {r['table']} | {','.join(map(str, r['levels']))} | {r['cycle']} | {r['lmax']} | "
              f"{r['N_ti']} / {r['N_c']} / {r['N_lo']} | {g['N_ti']} / {g['N_c']} / {g['N_lo']} | "
              f"{g['ms_per_step']:.3f} |", flush=True)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
