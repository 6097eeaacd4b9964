"""bench.py's command line on the CPU: a request for more than one GPU is
refused before anything touches a device (one JSON line with the reason, exit
status 2), and the algorithmic-byte counts behind the roofline figures follow
their stated per-unit sizes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    line = json.loads(out.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in line["error"]


def test_algorithmic_bytes_per_unit():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2011_05427_amd import inputs
    from paper_2011_05427_amd.profsum import sweep_bytes

    slabs, _, _ = inputs.config_large()
    s = slabs[0]
    # sweep: 32 B per cell-update (corner pair in and out) + 32 B per group-cell of moment partials
    assert sweep_bytes(s) == pytest.approx(32.0 * s.ng * s.nmu * s.nx + 32.0 * s.ng * s.nx)
    # fine LO: 56 B per (group, cell) and solve, plus 32 B for each first solve after a sweep
    assert bench.lo_fine_bytes(s, 4, 3) == pytest.approx(56.0 * s.ng * s.nx * 4 + 32.0 * s.ng * s.nx * 3)
