"""Summaries of rocprofv3 output for the profile notes (host only, no GPU).

    python -m paper_2011_05427_amd.profsum trace RESULTS.db [--match NAME ...] [--top N] [--by-grid]
        per kernel (demangled name, template arguments kept): dispatches,
        total, mean, median, min and max duration from a --kernel-trace run,
        and the mean over launches of at least a tenth of the longest (launches
        whose slabs had all converged are predicated off and last a few us).

    python -m paper_2011_05427_amd.profsum traffic --workload large \\
            --fetch FETCH.csv --write WRITE.csv [--kernel k_sweep] [--command ...]
        HBM bytes per dispatch of one kernel from two --pmc runs (FETCH_SIZE,
        then WRITE_SIZE; KiB per dispatch), each scaled by what the same
        counter reads for the 1 GiB device copy that ``bench.py
        --copy-calibration`` ends with, against the kernel's algorithmic bytes;
        ends with the ``traffic-json`` line that ``bench.py`` reads for
        ``roofline.traffic`` while the sweep source still hashes the same.

    python -m paper_2011_05427_amd.profsum sq PASS1.csv [PASS2.csv ...] [--match NAME ...]
        per kernel and grid size, the medians over dispatches of SQ counters
        from one or more --pmc passes of the same command, per wavefront:
        instructions by type, wave cycles, the fractions of wave time with a
        vector ALU instruction active and waiting on a counter, and the mean
        active lanes per vector instruction.

The sweep kernel's algorithmic bytes and source hash live here so that the
benchmark and the summaries agree on them.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sqlite3
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

WORKLOAD_CONFIGS = {"paper": "config_paper_scale", "small": "config_small", "large": "config_large",
                    "batch": "config_batch"}

# the sweep kernel's section of the kernel file and the device headers it includes
SWEEP_SOURCES = ["paper_2011_05427_amd/csrc/tr_kernels.hip", "paper_2011_05427_amd/csrc/tr_device.h",
                 "paper_2011_05427_amd/csrc/tr_common.h"]
SWEEP_BEGIN, SWEEP_END = "// A2 (+ partial A3): SCB sweep", "// A3: QD factors"

COPY_BYTES = 8 << 27  # the calibration copy: 2^27 binary64 values read and written
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def sweep_bytes(slab, ibytes=8):
    """Algorithmic HBM bytes of one sweep of a slab: per cell-update read the
    previous-time-level corner pair and write the new one (2 x 2 values of
    ibytes each: 32 B in binary64, 16 B with binary32 storage); per (group,
    cell, half range) write the two binary64 moment partials (16 B)."""
    return 4.0 * ibytes * slab.cell_updates_per_sweep() + 32.0 * slab.ng * slab.nx


def sweep_source_hash(root=ROOT):
    """sha256 over the sweep kernel's source text (its section of the kernel
    file plus the device headers it includes)."""
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        text = open(os.path.join(root, rel)).read()
        if rel.endswith("tr_kernels.hip"):
            text = text[text.index(SWEEP_BEGIN):text.index(SWEEP_END)]
        h.update(text.encode())
    return h.hexdigest()


def measured_traffic(workload, bytes_per_launch, root=ROOT):
    """HBM traffic of one sweep launch from the committed counter summary of
    this workload, or None when there is none or the sweep source changed
    since the counters were taken."""
    path = os.path.join(root, "profiles", f"k_sweep_{workload}_traffic.md")
    try:
        for line in open(path):
            if line.startswith("traffic-json: "):
                d = json.loads(line[len("traffic-json: "):])
                if d.get("sweep_source_sha256") != sweep_source_hash(root):
                    return None
                t = d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
                return {"bytes_per_launch": t, "fetch_bytes_per_launch": d["fetch_bytes_per_launch"],
                        "write_bytes_per_launch": d["write_bytes_per_launch"],
                        "ratio_to_algorithmic": t / bytes_per_launch, "source": os.path.relpath(path, root)}
    except (OSError, ValueError, KeyError):
        return None
    return None


def short_name(name):
    """Kernel name without the return type and the argument list."""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


# ---------------------------------------------------------------------------
# kernel trace
# ---------------------------------------------------------------------------

def trace_durations(db_path, by_grid=False):
    """{short kernel name: [duration ns, ...]} from a rocprofv3 results.db;
    by_grid: keyed by name and grid size (threads), which tells the launches
    of one workload from those of another in a run that holds several."""
    con = sqlite3.connect(db_path)
    try:
        rows = con.execute(
            "SELECT ks.display_name, k.grid_size_x * k.grid_size_y * k.grid_size_z, k.end - k.start "
            "FROM rocpd_kernel_dispatch k JOIN rocpd_info_kernel_symbol ks ON k.kernel_id = ks.id").fetchall()
    finally:
        con.close()
    out = defaultdict(list)
    for name, grid, dur in rows:
        key = short_name(str(name)) + (f" [grid {grid}]" if by_grid else "")
        out[key].append(float(dur))
    return out


def trace_table(durs, match=None, top=0):
    lines = ["| kernel | dispatches | total ms | mean us | median us | min us | max us | mean us of launches >= 10% of max |",
             "|---|---|---|---|---|---|---|---|"]
    items = sorted(durs.items(), key=lambda kv: -sum(kv[1]))
    if top:
        items = items[:top]
    for name, d in items:
        if match and not any(m in name for m in match):
            continue
        lines.append(f"| `{name}` | {len(d)} | {sum(d) / 1e6:.3f} | {statistics.fmean(d) / 1e3:.2f} | "
                     f"{statistics.median(d) / 1e3:.2f} | {min(d) / 1e3:.2f} | {max(d) / 1e3:.2f} | "
                     f"{statistics.fmean([v for v in d if v >= 0.1 * max(d)]) / 1e3:.2f} |")
    return "\n".join(lines)


# ---------------------------------------------------------------------------
# byte counters
# ---------------------------------------------------------------------------

def counter_values(csv_path, counter):
    """{short kernel name: [value per dispatch, ...]} of one counter."""
    out = defaultdict(list)
    with open(csv_path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def copy_factor(vals):
    """Scale factor of a counter (bytes per KiB read) from the 1 GiB copies:
    the copy dispatches whose count is at least half the largest one's."""
    cp = vals.get(COPY_KERNEL, [])
    if not cp:
        raise SystemExit(f"no {COPY_KERNEL} dispatch: run the counters with --copy-calibration")
    big = [v for v in cp if v >= 0.5 * max(cp)]
    kib = statistics.median(big)
    return COPY_BYTES / (kib * 1024.0), kib, len(big)


def kernel_dispatches(vals, kernel):
    """Every dispatch of every instantiation of `kernel` (the sweep tiles of
    the autotuner all read and write the same rows): (names, values)."""
    names = sorted(n for n in vals if n == kernel or n.startswith(kernel + "<"))
    if not names:
        raise SystemExit(f"no dispatch of {kernel} in the counter file")
    return names, [v for n in names for v in vals[n]]


def traffic_summary(workload, fetch_csv, write_csv, kernel="k_sweep", command=None):
    sys.path.insert(0, ROOT)
    from paper_2011_05427_amd import inputs

    slabs, _, _ = getattr(inputs, WORKLOAD_CONFIGS[workload])()
    if len(slabs) != 1:
        raise SystemExit("per-launch traffic is summarised for single-slab workloads")
    alg = sweep_bytes(slabs[0])
    fv, wv = counter_values(fetch_csv, "FETCH_SIZE"), counter_values(write_csv, "WRITE_SIZE")
    ff, fkib, fn = copy_factor(fv)
    wf, wkib, wn = copy_factor(wv)
    fnames, fd = kernel_dispatches(fv, kernel)
    wnames, wd = kernel_dispatches(wv, kernel)
    kname = ", ".join(sorted(set(fnames) | set(wnames)))
    fmed, wmed = statistics.median(fd), statistics.median(wd)
    fb, wb = fmed * 1024.0 * ff, wmed * 1024.0 * wf
    rec = {"workload": workload, "kernel": kname, "sweep_source_sha256": sweep_source_hash(),
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "fetch_calibration_factor": ff,
           "write_calibration_factor": wf, "algorithmic_bytes_per_launch": alg}
    out = [f"# {kernel} HBM traffic: {workload} workload (byte counters)", ""]
    if command:
        out += ["Commands (on the MI355X host), then this summary:", ""]
        out += ["    " + c for c in command] + [""]
    out += [
        "Counter values are KiB per dispatch.  The median over the kernel's dispatches",
        "is taken (dispatches of already converged slabs are predicated off and read",
        "near zero).  Each counter is scaled by what it reads for the 1 GiB device copy",
        "at the end of the same run.",
        "",
        "| quantity | value |", "|---|---|",
        f"| kernel instantiations (all tiles pooled) | `{kname}` |",
        f"| dispatches (FETCH / WRITE run) | {len(fd)} / {len(wd)} |",
        f"| FETCH_SIZE per dispatch, median (min..max) KiB | {fmed:.1f} ({min(fd):.1f}..{max(fd):.1f}) |",
        f"| WRITE_SIZE per dispatch, median (min..max) KiB | {wmed:.1f} ({min(wd):.1f}..{max(wd):.1f}) |",
        f"| calibration: 1 GiB copy, FETCH_SIZE KiB ({fn} dispatches) | {fkib:.1f} (factor {ff:.4f}) |",
        f"| calibration: 1 GiB copy, WRITE_SIZE KiB ({wn} dispatches) | {wkib:.1f} (factor {wf:.4f}) |",
        f"| HBM bytes read per launch (scaled) | {fb / 1e6:.2f} MB |",
        f"| HBM bytes written per launch (scaled) | {wb / 1e6:.2f} MB |",
        f"| traffic per launch | {(fb + wb) / 1e6:.2f} MB |",
        f"| algorithmic bytes per launch (32 B per cell-update + 32 B per group-cell) | {alg / 1e6:.2f} MB |",
        f"| traffic / algorithmic | {(fb + wb) / alg:.4f} |",
        "",
        "The read side also carries the opacity and Planck tables and the cell widths",
        "(not counted as algorithmic bytes: they are recomputable from T).",
        "",
        "traffic-json: " + json.dumps(rec),
    ]
    return "\n".join(out)


# ---------------------------------------------------------------------------
# SQ (wavefront) counters
# ---------------------------------------------------------------------------

def sq_table(csv_paths, match=None):
    """Per (kernel, grid) medians of every counter found in the passes."""
    med = defaultdict(dict)
    for path in csv_paths:
        vals = defaultdict(lambda: defaultdict(list))
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                key = f"{short_name(r['Kernel_Name'])} [grid {r['Grid_Size']}]"
                vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
        for key, cs in vals.items():
            for c, v in cs.items():
                med[key][c] = statistics.median(v)
    cols = [("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_SALU", "SALU"), ("SQ_INSTS_SMEM", "SMEM"),
            ("SQ_INSTS_VMEM_RD", "VMEM rd"), ("SQ_INSTS_VALU_TRANS_F64", "FP64 trans")]
    lines = ["| kernel | waves | " + " | ".join(f"{n} / wave" for _, n in cols) +
             " | wave cycles / wave | VALU active | waiting on counters | lanes per VALU instr |",
             "|---|---|" + "---|" * len(cols) + "---|---|---|---|"]
    for key in sorted(med):
        if match and not any(m in key for m in match):
            continue
        m = med[key]
        w = m.get("SQ_WAVES")
        wc = m.get("SQ_WAVE_CYCLES")
        if not w or not wc:
            continue
        per = " | ".join(f"{m[c] / w:.0f}" if c in m else "-" for c, _ in cols)
        act = m.get("SQ_ACTIVE_INST_VALU")
        lanes = (f"{m['SQ_THREAD_CYCLES_VALU'] / act:.1f}" if act and "SQ_THREAD_CYCLES_VALU" in m else "-")
        lines.append(f"| `{key}` | {w:.0f} | {per} | {wc / w:.0f} | "
                     f"{(act / wc if act else 0):.2f} | {m.get('SQ_WAIT_INST_ANY', 0) / wc:.2f} | {lanes} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--match", nargs="*", default=None)
    t.add_argument("--top", type=int, default=0, help="only the N kernels of largest total time")
    t.add_argument("--by-grid", action="store_true", help="one row per kernel and grid size")
    p = sub.add_parser("traffic")
    p.add_argument("--workload", required=True, choices=sorted(WORKLOAD_CONFIGS))
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--kernel", default="k_sweep")
    p.add_argument("--command", action="append", default=None, help="command line that made the counters")
    q = sub.add_parser("sq")
    q.add_argument("csv", nargs="+")
    q.add_argument("--match", nargs="*", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "sq":
        print(sq_table(a.csv, a.match))
    elif a.cmd == "trace":
        print(trace_table(trace_durations(a.db, a.by_grid), a.match, a.top))
    else:
        print(traffic_summary(a.workload, a.fetch, a.write, a.kernel, a.command))


if __name__ == "__main__":
    main()
