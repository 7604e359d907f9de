#!/usr/bin/env python3
"""Benchmark of the GOC-LBM hot path on one MI355X.

One step = one pass of the whole hot path (one fused collide-and-stream
kernel launch of the central-moment GOC-LBM with the coupled D2Q5 induction
sweep) over the synthetic workload, inputs resident in HBM.  The headline
workload is the 4096 x 1024 Ha = 100 Hartmann channel in plain FP32
(D2Q9 + D2Q5, 168 algorithmic bytes per node, a 0.7 GB state that does not
fit in the 256 MB Infinity Cache).

Prints ONE JSON line:
  metric / value / unit      MLUPS of the workload (whole job, one GPU)
  roofline                   HBM roofline of the step kernel: algorithmic
                             bytes per launch / mean launch time (HIP events
                             on the launch stream) against 8 TB/s, and the
                             measured HBM traffic per launch when a counter
                             profile of the current kernel source is
                             committed under profiles/; and the
                             same-pattern ceiling: a kernel with the step's
                             loads and stores and none of its arithmetic
                             (libgocceiling.so), beside a one-stream copy
  cpu_baseline               the FP64 oracle on the host cores (all of them,
                             and one), on a bounded sample of the workload
  forms                      the same GPU on the same workload in FP32 and the
                             FP16 / BF16 deviation-storage forms, from the
                             developed Hartmann flow, with their field
                             differences from the FP32 run
  batched                    the seeded 256-run batch in one launch per step
                             against the same runs one after another
  collisions                 the workload with the raw-moment MRT and the SRT
                             collision bodies instead of the central-moment one
  curvilinear                the curvilinear step (general 2-D metric) on a
                             2048x512 conformal annular sector, FP32
  cache_resident             the 1024x1024 Re = 1000 cavity in FP32, whose
                             98 MB state stays in the Infinity Cache: its
                             bytes per second are not an HBM figure
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
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


def form_tag(launch) -> str:
    """Short name of a step form, as the profile summaries are named."""
    if launch["waves_per_cu"] == 0:
        cols = int(launch.get("tile_cols", 64))
        shape = f"{int(launch['rows_per_segment'])}" if cols == 64 else f"{cols}x{int(launch['rows_per_segment'])}"
        return f"tiled{shape}{'nt' if launch['nontemporal'] else ''}"
    return f"march{launch['waves_per_cu']:g}"


def measured_traffic(kernel: str, workload: str, tag: str):
    """HBM bytes per launch of a kernel in a step form on a workload, from a
    committed rocprofv3 counter summary taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('::')[-1]}_{workload}_{tag}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_run(run, steps: int, warmup: int):
    """Wall time and HIP-event time (on the run's stream) of `steps` steps."""
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
    """The FP64 oracle, untuned, on the host cores (all of them, then one):
    full grid of the same workload, as many steps as fit in about `seconds`
    each, after one untimed step."""
    import oracle
    all_cores = oracle.threads()
    out = {}
    for label, n_threads in (("all", all_cores), ("one", 1)):
        oracle.set_threads(n_threads)
        m = oracle.Model(case).init()
        t0 = time.perf_counter()
        m.step(1)
        t1 = time.perf_counter() - t0
        n = max(1, int(seconds / max(t1, 1e-6)))
        t0 = time.perf_counter()
        m.step(n)
        dt = time.perf_counter() - t0
        out[label] = (case.nx * case.ny * n / dt / 1e6, n, dt)
    oracle.set_threads(all_cores)
    v, n, dt = out["all"]
    v1, n1, dt1 = out["one"]
    return {"value": v, "unit": "MLUPS", "cores": all_cores, "kind": "oracle",
            "sample": f"{n} steps of the full {case.nx}x{case.ny} {case.name} grid in FP64 on {all_cores} "
                      f"threads ({dt:.1f} s), and {n1} on one ({dt1:.1f} s), each after one untimed step",
            "one_core_value": v1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model() -> str:
    """The host processor's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_calibration(mib: int, reps: int):
    """A plain device-to-device copy of known size (the instrument library's
    copy kernel), for scaling the HBM byte counters of a profiler run: prints
    the bytes moved per copy and the rate."""
    from paper_2607_15362_amd import ceiling as CL
    nb = mib * (1 << 20)
    us = CL.copy_us(nb, reps)
    print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb,
                      "GB_s": round(2 * nb / us / 1e3, 1)}), flush=True)


def pattern_ceiling(case, launch, bytes_per_launch: float, launch_us: float):
    """The same-pattern ceiling of the tiled step on this workload: the
    instrument kernel with the step's loads and stores (same layout, tile
    shape and store policy) and no arithmetic, and a 1 GiB one-stream copy.
    None for the march and for FP64 storage, which it does not mirror."""
    from paper_2607_15362_amd import ceiling as CL
    if launch["waves_per_cu"] != 0 or case.storage == "f64" or case.bc_x != "periodic":
        return None
    sb = 4 if case.storage == "f32" else 2
    us = CL.pattern_us(case.nx, case.ny, case.mhd, sb, int(launch["rows_per_segment"]), bool(launch["nontemporal"]),
                       cols=int(launch.get("tile_cols", 64)))
    cu = CL.copy_us(1 << 30)
    return {"instrument": "goc_ceiling_pattern: the step's loads and stores without its arithmetic",
            "pattern_us": round(us, 2), "pattern_GB_s_algorithmic": round(bytes_per_launch / us / 1e3, 1),
            "step_over_pattern": round(launch_us / us, 4),
            "copy_1GiB_GB_s": round(2 * (1 << 30) / cu / 1e3, 1)}


def developed(run, case):
    """Start a Hartmann run from its closed-form developed flow."""
    from paper_2607_15362_amd import workloads as W
    d = run.derived()
    run.init(*W.hartmann_start(case, d["nu"], d["F1"], d["eta"], d["B0"]))


def storage_forms(case, steps: int):
    """The workload in plain FP32 and in the FP16 / BF16 deviation-storage
    forms on the same GPU, each started from the closed-form developed
    Hartmann flow: throughput, bytes moved, and the relative L2 difference of
    every field from the plain FP32 run after the same number of steps."""
    import numpy as np
    from paper_2607_15362_amd import binding as B
    n = max(600, steps // 4)
    forms, ref = {}, None
    for st in ("f32", "f16dev", "bf16dev"):
        c = case.replace(name=case.name if st == "f32" else f"{case.name}_{st}", storage=st)
        r = B.Run(c)
        developed(r, c)
        tuned = r.tune(50)
        li = r.launch_info()
        w, e = time_run(r, n, 100)
        dd = r.derived()
        fl = r.fields()
        forms[st] = {"workload": c.name, "steps": n + 100, "MLUPS": round(c.nx * c.ny * n / w / 1e6, 1),
                     "GB_s": round(dd["bytes_per_node"] * c.nx * c.ny / (e / n) / 1e9, 1),
                     "bytes_per_node": dd["bytes_per_node"], "form": form_tag(li),
                     "waves_per_cu": tuned["waves_per_cu"]}
        if ref is None:
            ref = fl
        else:
            vel = np.linalg.norm(np.hypot(ref["U1"], ref["U2"]))
            norms = {"rho": np.linalg.norm(ref["rho"]), "U1": np.linalg.norm(ref["U1"]), "U2": vel,
                     "B1": np.linalg.norm(ref["B1"]), "B2": np.linalg.norm(ref["B2"])}
            forms[st]["rel_l2_vs_f32"] = {k: float(f"{np.linalg.norm(fl[k] - ref[k]) / norms[k]:.3e}")
                                          for k in norms}
            forms[st]["vs_f32_MLUPS"] = round(forms[st]["MLUPS"] / forms["f32"]["MLUPS"], 3)
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
    li = b.launch_info()
    w, e = time_run(b, n, 100)
    d = b.derived()
    out = {"runs": len(runs), "nodes": nodes, "steps": n, "MLUPS": round(nodes * n / w / 1e6, 1),
           "GB_s": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1), "form": form_tag(li),
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
    """The workload with the raw-moment MRT and the SRT collisions:
    throughput, achieved bandwidth and the ratio to the central-moment run."""
    from paper_2607_15362_amd import binding as B
    n = max(500, steps // 5)
    out = {}
    for coll in ("raw", "srt"):
        c = case.replace(name=f"{case.name}_{coll}", collision=coll)
        r = B.Run(c)
        tuned = r.tune(50)
        li = r.launch_info()
        w, e = time_run(r, n, 100)
        d = r.derived()
        nodes = c.nx * c.ny
        out[coll] = {"steps": n, "MLUPS": round(nodes * n / w / 1e6, 1),
                     "GB_s": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1),
                     "launch_us": round(e / n * 1e6, 2), "form": form_tag(li), "waves_per_cu": tuned["waves_per_cu"],
                     "vs_central": round(nodes * n / w / 1e6 / central_mlups, 3)}
        r.close()
    return out


def curvilinear_form(steps: int):
    """The curvilinear step on a large conformal annular sector (Taylor-Couette
    geometry: 2048 radial x 512 azimuthal nodes, R1 = 256, R2 = R1 + 2048, the
    sector angle chosen for cells of aspect ratio about one), FP32: MLUPS and
    the achieved bandwidth in algorithmic bytes (populations and force read
    and written, the 12 metric planes read)."""
    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W
    n1, n2, R1 = 2048, 512, 256.0
    n_theta = 2.0 * math.pi * n1 / (n2 * math.log((R1 + n1) / R1))
    c = W.taylor_couette(n1=n1, n2=n2, R1=R1, n_theta=n_theta, U_in=0.01, U_out=0.015, storage="f32")
    r = B.Run(c)
    r.tune(50)
    li = r.launch_info()
    n = max(200, steps // 10)
    w, e = time_run(r, n, 50)
    d = r.derived()
    nodes = n1 * n2
    out = {"workload": f"annular sector {n1}x{n2}, R1 = {R1:g}, FP32", "steps": n,
           "MLUPS": round(nodes * n / w / 1e6, 1), "step_us": round(e / n * 1e6, 2),
           "bytes_per_node": d["bytes_per_node"], "form": form_tag(li),
           "GB_s_algorithmic": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1)}
    out["frac_of_8TBs"] = round(out["GB_s_algorithmic"] / PEAK_HBM_GBS, 4)
    r.close()
    return out


def cache_resident(steps: int):
    """The 1024x1024 Re = 1000 cavity in FP32 (98 MB of state, inside the
    256 MB Infinity Cache): MLUPS and algorithmic bytes per second, which
    here measure the cache, not HBM."""
    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W
    c = W.cavity_1024()
    r = B.Run(c)
    r.tune(100)
    li = r.launch_info()
    n = max(2000, steps)
    w, e = time_run(r, n, 300)
    d = r.derived()
    nodes = c.nx * c.ny
    ulid, cs = B.derive(c)[0].u_wall_hi, math.sqrt(d["cs2"])
    out = {"workload": f"{c.name}: lid-driven cavity {c.nx}x{c.ny}, tanh beta=2 on both axes, Re=1000, "
                       f"lid speed {ulid:.3e} (Mach {ulid / cs:.3f} of the GOC sound speed), FP32; "
                       "cache-resident (98 MB of state)",
           "steps": n, "MLUPS": round(nodes * n / w / 1e6, 1), "step_us": round(e / n * 1e6, 2),
           "form": form_tag(li), "GB_s_algorithmic": round(d["bytes_per_node"] * nodes / (e / n) / 1e9, 1)}
    out["frac_of_8TBs_not_hbm"] = round(out["GB_s_algorithmic"] / PEAK_HBM_GBS, 4)
    r.close()
    return out


def workload_case(name: str, storage: str):
    from paper_2607_15362_amd import workloads as W
    if name == "cavity_1024":
        c = W.cavity_1024()
    else:
        c = W.hartmann_4096()
    if storage != "f32":
        c = c.replace(name=f"{c.name}_{storage}", storage=storage)
    return c


def describe(case, run) -> str:
    d = run.derived()
    cs = math.sqrt(d["cs2"])
    if case.flow == "cavity":
        from paper_2607_15362_amd import binding as B
        ulid = B.derive(case)[0].u_wall_hi
        return (f"{case.name}: lid-driven cavity {case.nx}x{case.ny}, tanh beta=2 on both axes, Re=1000, "
                f"lid speed {ulid:.3e} (Mach {ulid / cs:.3f}), {case.storage} storage; cache-resident")
    H = case.ny / 2.0
    Uc = case.Re * d["nu"] / H
    return (f"{case.name}: Hartmann channel {case.nx}x{case.ny}, tanh beta=3, Ha=100, Re=100, Pm=1, "
            f"centre-line speed {Uc:.3e} (Mach {Uc / cs:.4f}, tau = 1), D2Q9+D2Q5, {case.storage} storage, "
            "FP32 arithmetic")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="hartmann_4096", choices=["hartmann_4096", "cavity_1024"])
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "f16dev", "bf16dev"])
    ap.add_argument("--developed", action="store_true",
                    help="start the Hartmann workload from its developed flow (default: from rest)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-collisions", action="store_true")
    ap.add_argument("--no-curvilinear", action="store_true")
    ap.add_argument("--no-cache-resident", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the same-pattern ceiling of the roofline")
    ap.add_argument("--only-main", action="store_true", help="the main line only (all of the --no-* options)")
    ap.add_argument("--waves", type=float, default=-1.0, metavar="W",
                    help="fixed step form instead of the autotuner (for profiler runs): W > 0 the march with "
                         "W waves per CU; W = 0 the tiled step with --tile rows")
    ap.add_argument("--tile", default="", metavar="ROWS[nt]",
                    help="fixed tiled step (for profiler runs): 4, 8 or 16 rows (64 columns) or 128x4, "
                         "'nt' for non-temporal stores, e.g. 4nt, 128x4nt")
    ap.add_argument("--batch", action="store_true",
                    help="the main line is the seeded 256-run batch (FP32, developed flows)")
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
    if args.only_main:
        args.no_cpu_baseline = args.no_forms = args.no_batch = args.no_collisions = True
        args.no_curvilinear = args.no_cache_resident = args.no_ceiling = True

    from paper_2607_15362_amd import binding as B
    from paper_2607_15362_amd import workloads as W

    if args.batch:
        runs = [c.replace(storage=args.storage) for c in W.batch_256()]
        run = B.Run(batch=runs)
        for k, c in enumerate(runs):
            d = run.derived(run=k)
            run.init_run(k, *W.hartmann_start(c, d["nu"], d["F1"], d["eta"], d["B0"]))
        case = runs[0].replace(name=f"batch_256_{args.storage}")
        nodes = sum(c.nx * c.ny for c in runs)
    else:
        case = workload_case(args.workload, args.storage)
        run = B.Run(case)
        if args.developed and case.flow == "hartmann":
            developed(run, case)
        nodes = case.nx * case.ny
    if args.tile:
        shape = args.tile[:-2] if args.tile.endswith("nt") else args.tile
        cols, rows = (int(v) for v in shape.split("x")) if "x" in shape else (64, int(shape))
        run.set_tile(rows, args.tile.endswith("nt"), cols=cols)
        tuned = {"us_before": float("nan")}
    elif args.waves > 0:
        run.set_launch(args.waves)
        tuned = {"us_before": float("nan")}
    else:
        tuned = run.tune(100)     # step form and launch-plan autotuner (state unchanged)
    launch = run.launch_info()
    wall, ev = time_run(run, args.steps, args.warmup)
    d = run.derived()
    mlups = nodes * args.steps / wall / 1e6
    launch_s = ev / args.steps
    bytes_per_launch = d["bytes_per_node"] * nodes
    achieved = bytes_per_launch / launch_s / 1e9
    workload = "batch_256" if args.batch else case.name
    traffic = measured_traffic(kernel_name(launch), workload, form_tag(launch))
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
        "dtype": {"f64": "f64", "f32": "f32", "f16dev": "f16 storage, f32 arithmetic",
                  "bf16dev": "bf16 storage, f32 arithmetic"}[case.storage],
        "data": "synthetic",
        "config": {"workload": (f"batch_256: the seeded 256 Hartmann channels (128x64 .. 1024x512), "
                                f"{args.storage} storage" if args.batch else describe(case, run)),
                   "nx": case.nx, "ny": case.ny, "nodes": nodes, "storage": case.storage,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_node": d["bytes_per_node"], "launch_us": round(launch_s * 1e6, 2),
                     "kernel": kernel_name(launch),
                     "launch_plan": {"form": form_tag(launch),
                                     "waves_per_cu": launch["waves_per_cu"], "work_groups": launch["blocks"],
                                     "rows_per_segment": round(launch["rows_per_segment"], 2),
                                     "tile_cols": launch["tile_cols"],
                                     "nontemporal_stores": bool(launch["nontemporal"]),
                                     "untuned_us": (round(tuned["us_before"], 2)
                                                    if tuned["us_before"] == tuned["us_before"] else None)}},
    }
    run.close()
    if not args.batch and not args.no_ceiling:
        out["roofline"]["ceiling"] = pattern_ceiling(case, launch, bytes_per_launch, launch_s * 1e6)

    if not args.no_forms and not args.batch and case.flow == "hartmann" and case.storage == "f32":
        out["forms"] = storage_forms(case, args.steps)
    if not args.no_batch and not args.batch:
        out["batched"] = batched_form(args.steps)
        if "forms" in out:
            out["batched"]["vs_plain_fp32_4096x1024"] = round(out["batched"]["MLUPS"] / out["forms"]["f32"]["MLUPS"], 3)
    if not args.no_collisions and not args.batch:
        out["collisions"] = collision_variants(case, args.steps, mlups)
    if not args.no_curvilinear:
        out["curvilinear"] = curvilinear_form(args.steps)
    if not args.no_cache_resident and case.flow != "cavity":
        out["cache_resident"] = cache_resident(args.steps)
    if not args.no_cpu_baseline and not args.batch:
        out["cpu_baseline"] = cpu_baseline(case.replace(storage="f64"), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
