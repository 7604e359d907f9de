"""bench.py keeps its output contract: one JSON line with the benchmark
metric, the workload, the roofline of the dominant kernel and the oracle's
CPU baseline.  A short run of the main line only (the other forms off), in a
child process."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_bench_json_line():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "200", "--warmup", "20", "--no-forms",
           "--no-batch", "--no-collisions", "--no-curvilinear", "--no-cache-resident", "--cpu-seconds", "1"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, out.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 200 and d["warmup"] == 20
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"].startswith("hartmann_4096x1024") and d["config"]["storage"] == "f32"
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0.0 < r["frac"] < 1.0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    # the same-pattern ceiling of the tiled step: the pattern alone is faster than the step
    c = r["ceiling"]
    if r["launch_plan"]["form"].startswith("tiled"):
        assert 0 < c["pattern_us"] < r["launch_us"] * 1.02 and c["copy_1GiB_GB_s"] > 1000
    c = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in c, k
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["one_core_value"] > 0
    assert isinstance(c["cpu_model"], str) and c["cpu_model"] and c["host_cpus"] >= 1


@pytest.mark.gpu
def test_ceiling_instrument_on_small_and_ragged_grids():
    """The instrument runs (in bounds) on grids smaller than a tile and with
    ragged edges, for both storage widths, and its copy and read / write
    mixes move small buffers."""
    from paper_2607_15362_amd import ceiling as CL
    for nx, ny, mhd, sb, rows, cols in [(3, 3, 1, 4, 16, 64), (70, 37, 1, 4, 8, 64), (130, 9, 0, 2, 4, 64),
                                        (200, 66, 1, 2, 16, 64), (3, 3, 1, 4, 4, 128), (200, 66, 1, 2, 4, 128)]:
        us = CL.pattern_us(nx, ny, bool(mhd), sb, rows, True, reps=5, cols=cols)
        assert 0 < us < 1e5
    assert 0 < CL.copy_us(1 << 20, reps=5) < 1e5
    # the read / write mixes, on sizes that are not a multiple of the grid
    # stride (the tail loop) and smaller than one work-group's share
    for nbytes in (16, 48, (1 << 20) + 16 * 37):
        for reads, writes in ((1, 0), (2, 0), (0, 1), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)):
            for nt in (False, True):
                for chunked in (False, True):
                    assert 0 < CL.mix_us(nbytes, reads, writes, nt, wg_per_cu=8, reps=2, chunked=chunked) < 1e5


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode != 0
    assert "one GPU" in out.stdout + out.stderr
