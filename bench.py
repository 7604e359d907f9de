#!/usr/bin/env python3
"""Benchmark of the GOC-LBM hot path on one MI355X.

One step = one pass of the whole hot path (one fused collide-and-stream
kernel launch of the central-moment GOC-LBM, plus the D2Q5 induction sweep
for MHD workloads) over the synthetic workload, inputs resident in HBM.

Prints ONE JSON line:
  metric / value / unit      MLUPS of the workload (whole job, one GPU)
  roofline                   HBM roofline of the step kernel: algorithmic
                             bytes per launch / mean launch time (HIP events
                             on the launch stream) against 8 TB/s, plus the
                             measured HBM traffic when a counter profile of
                             the current kernel source is committed
  cpu_baseline               the FP64 oracle on the host cores, on a bounded
                             sample of the same workload
  forms                      the same GPU on the 4096x1024 MHD workload in
                             FP32 and the FP16 / BF16 deviation-storage forms,
                             with their field errors against the FP32 run
  batched                    the seeded 256-run batch in one launch per step
                             against the same runs one after another
  collisions                 the main workload with the raw-moment MRT and the
                             SRT collision bodies instead of the central-moment
                             one (same data path, same launch)
  curvilinear                the curvilinear step (general 2-D metric, one
                             launch per step) on a 2048x512 conformal annular
                             sector, FP32, with its algorithmic bytes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "MLUPS + % HBM peak; FP16-store & batched vs plain FP32 on same GPU"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("goc_device.hpp", "goc_step.hpp", "goc_tile.hpp"):
        with open(os.path.join(ROOT, "paper_2607_15362_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(launch) -> str:
    """The step kernel a launch plan runs: the tiled step (waves_per_cu 0) or
    the march."""
    return "goc::tile_step_kernel" if launch["waves_per_cu"] == 0 else "goc::step_kernel"


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel on a workload from a committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('::')[-1]}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_run(run, steps: int, warmup: int):
    from paper_2607_15362_amd import binding as B
    run.step(warmup)
    run.synchronize()
    e0, e1 = B.Event(), B.Event()
    t0 = time.perf_counter()
    e0.record(run.stream_obj)
    run.step(steps)
    e1.record(run.stream_obj)
    run.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, e0.elapsed_ms(e1) / 1e3


def cpu_baseline(case, seconds: float):
    """The FP64 oracle, untuned, on the host cores: full grid of the same
    workload, as many steps as fit in about `seconds`."""
    import oracle
    m = oracle.Model(case).init()
    t0 = time.perf_counter()
    m.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(seconds / max(t1, 1e-6)))
    t0 = time.perf_counter()
    m.step(n)
    dt = time.perf_counter() - t0
    return {"value": case.nx * case.ny * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} steps of the full {case.nx}x{case.ny} {case.name} grid in FP64 "
                      f"({dt:.1f} s), after one untimed step"}


def copy_calibration(mib: int, reps: int):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters of a profiler run: prints the bytes moved per copy and the rate."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "GB_s": round(8 * n / dt / 1e9, 1)}), flush=True)


def storage_forms(steps: int):
    """The 4096x1024 Ha=100 channel in plain FP32 and in the FP16 / BF16
    deviation-storage forms on the same GPU, each started from the
    closed-form developed Hartmann flow: throughput, bytes moved, and the
    relative L2 difference of every field from the plain FP32 run after the
    same number of steps."""
    import numpy as np
    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W
    n = max(200, steps // 10)
    forms, ref = {}, None
    for st in ("f32", "f16dev", "bf16dev"):
        c = W.hartmann_4096_precision(st) if st != "f32" else W.hartmann_4096()
        r = B.Run(c)
        dd = r.derived()
        r.init(*W.hartmann_start(c, dd["nu"], dd["F1"], dd["eta"], dd["B0"]))
        tuned = r.tune(50)
        w, e = time_run(r, n, 100)
        fl = r.fields()
        forms[st] = {"workload": c.name, "steps": n + 100, "MLUPS": round(c.nx * c.ny * n / w / 1e6, 1),
                     "GB_s": round(dd["bytes_per_node"] * c.nx * c.ny / (e / n) / 1e9, 1),
                     "bytes_per_node": dd["bytes_per_node"], "waves_per_cu": tuned["waves_per_cu"]}
        if ref is None:
            ref = fl
        else:
            vel = np.linalg.norm(np.hypot(ref["U1"], ref["U2"]))
            norms = {"rho": np.linalg.norm(ref["rho"]), "U1": np.linalg.norm(ref["U1"]), "U2": vel,
                     "B1": np.linalg.norm(ref["B1"]), "B2": np.linalg.norm(ref["B2"])}
            forms[st]["rel_l2_vs_f32"] = {k: float(f"{np.linalg.norm(fl[k] - ref[k]) / norms[k]:.3e}")
                                          for k in norms}
        r.close()
    return forms


def batched_form(steps: int):
    """The seeded batch of 256 stretched Hartmann channels (uneven grids,
    beta, Re, Ha; FP32) from their developed flows: one launch per step for
    the whole batch (100-step graphs, tuned plan) against the same runs
    stepped one after another with their own launches (each tuned)."""
    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W
    runs = W.batch_256()
    nodes = sum(c.nx * c.ny for c in runs)
    n = max(100, (steps // 30) // 100 * 100)

    def start(r, c, run=None):
        d = r.derived(run=run or 0)
        init = W.hartmann_start(c, d["nu"], d["F1"], d["eta"], d["B0"])
        if run is None:
            r.init(*init)
        else:
            r.init_run(run, *init)

    b = B.Run(batch=runs)
    for k, c in enumerate(runs):
        start(b, c, k)
    tuned = b.tune(20)
    w, _ = time_run(b, n, 100)
    out = {"runs": len(runs), "nodes": nodes, "steps": n, "MLUPS": round(nodes * n / w / 1e6, 1),
           "waves_per_cu": tuned["waves_per_cu"]}
    b.close()
    singles = []
    for c in runs:
        r = B.Run(c)
        start(r, c)
        r.tune(10)
        r.step(100)
        singles.append(r)
    for r in singles:
        r.synchronize()
    t0 = time.perf_counter()
    for r in singles:
        r.step(n)
        r.synchronize()
    dt = time.perf_counter() - t0
    for r in singles:
        r.close()
    out["one_after_another_MLUPS"] = round(nodes * n / dt / 1e6, 1)
    out["speedup"] = round(out["MLUPS"] / out["one_after_another_MLUPS"], 2)
    return out


def collision_variants(case, steps: int, central_mlups: float):
    """The main workload with the raw-moment MRT and the SRT collisions:
    throughput, achieved bandwidth and the ratio to the central-moment run."""
    from paper_2607_15362_amd import binding as B
    n = max(500, steps // 5)
    out = {}
    for coll in ("raw", "srt"):
        c = case.replace(name=f"{case.name}_{coll}", collision=coll)
        r = B.Run(c)
        tuned = r.tune(50)
        w, e = time_run(r, n, 100)
        d = r.derived()
        nodes = c.nx * c.ny
        out[coll] = {"steps": n, "MLUPS": round(nodes * n / w / 1e6, 1),
                     "GB_s": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1),
                     "launch_us": round(e / n * 1e6, 2), "waves_per_cu": tuned["waves_per_cu"],
                     "vs_central": round(nodes * n / w / 1e6 / central_mlups, 3)}
        r.close()
    return out


def curvilinear_form(steps: int):
    """The curvilinear step on a large conformal annular sector (Taylor-Couette
    geometry: 2048 radial x 512 azimuthal nodes, R1 = 256, R2 = R1 + 2048, the
    sector angle chosen for cells of aspect ratio about one), FP32: MLUPS and
    the achieved bandwidth in algorithmic bytes (populations and force read
    and written, the 12 metric planes read), with the launch time of the
    kernel from HIP events."""
    import math
    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W
    n1, n2, R1 = 2048, 512, 256.0
    n_theta = 2.0 * math.pi * n1 / (n2 * math.log((R1 + n1) / R1))
    c = W.taylor_couette(n1=n1, n2=n2, R1=R1, n_theta=n_theta, U_in=0.01, U_out=0.015, storage="f32")
    r = B.Run(c)
    n = max(200, steps // 10)
    w, e = time_run(r, n, 50)
    d = r.derived()
    nodes = n1 * n2
    out = {"workload": f"annular sector {n1}x{n2}, R1 = {R1:g}, FP32", "steps": n,
           "MLUPS": round(nodes * n / w / 1e6, 1), "step_us": round(e / n * 1e6, 2),
           "bytes_per_node": d["bytes_per_node"],
           "GB_s_algorithmic": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1)}
    out["frac_of_8TBs"] = round(out["GB_s_algorithmic"] / PEAK_HBM_GBS, 4)
    r.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="cavity_1024", choices=["cavity_1024", "hartmann_4096"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-collisions", action="store_true")
    ap.add_argument("--no-curvilinear", action="store_true")
    ap.add_argument("--waves", type=float, default=-1.0, metavar="W",
                    help="fixed step form instead of the autotuner (for profiler runs): W = 0 the "
                         "tiled step, W > 0 the march with W waves per CU")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB mebibytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the hot path is a single-GPU build; see the design notes on sharding)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(1, args.steps))
        return

    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W

    case = W.cavity_1024() if args.workload == "cavity_1024" else W.hartmann_4096()
    run = B.Run(case)
    if args.waves >= 0:
        run.set_launch(args.waves)
        tuned = {"us_before": float("nan")}
    else:
        tuned = run.tune(100)     # step form and launch-plan autotuner (state unchanged)
    launch = run.launch_info()
    wall, ev = time_run(run, args.steps, args.warmup)
    d = run.derived()
    nodes = case.nx * case.ny
    mlups = nodes * args.steps / wall / 1e6
    launch_s = ev / args.steps
    bytes_per_launch = d["bytes_per_node"] * nodes
    achieved = bytes_per_launch / launch_s / 1e9
    traffic = measured_traffic(kernel_name(launch), case.name)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32"}.get(case.storage, "f32"),
        "data": "synthetic",
        "config": {"workload": f"{case.name}: lid-driven cavity {case.nx}x{case.ny}, tanh beta=2 "
                               f"on both axes, Re=1000, lid at Mach 0.1 of the finest cell, FP32 storage and arithmetic"
                   if case.flow == "cavity" else
                   f"{case.name}: Hartmann channel {case.nx}x{case.ny}, tanh beta=3, Ha=100, "
                   f"Re=100, Pm=1, D2Q9+D2Q5, FP32",
                   "nx": case.nx, "ny": case.ny, "storage": case.storage,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_node": d["bytes_per_node"], "launch_us": round(launch_s * 1e6, 2),
                     "kernel": kernel_name(launch),
                     "launch_plan": {"form": "tiled" if launch["waves_per_cu"] == 0 else "march",
                                     "waves_per_cu": launch["waves_per_cu"], "work_groups": launch["blocks"],
                                     "rows_per_segment": round(launch["rows_per_segment"], 2),
                                     "untuned_us": (round(tuned["us_before"], 2)
                                                    if tuned["us_before"] == tuned["us_before"] else None)}},
    }
    run.close()

    if not args.no_collisions:
        out["collisions"] = collision_variants(case, args.steps, mlups)
    if not args.no_curvilinear:
        out["curvilinear"] = curvilinear_form(args.steps)
    if not args.no_forms:
        out["forms"] = storage_forms(args.steps)
    if not args.no_batch:
        out["batched"] = batched_form(args.steps)
        if "forms" in out:
            out["batched"]["vs_plain_fp32_4096x1024"] = round(out["batched"]["MLUPS"] / out["forms"]["f32"]["MLUPS"], 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
