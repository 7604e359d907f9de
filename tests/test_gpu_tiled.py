"""The tiled step on straight grids against the march.  A single straight
run (with or without the D2Q5 scheme) can be stepped by either kernel (one
thread per node over LDS tiles, or one wave marching up a 64-column strip);
both take the same arithmetic in the same order, up to where the compiler
fuses a multiply and an add differently.  So one step from the same
developed state stores the same values to rounding, measured at the largest
stored value (a stored value may be a small difference of larger terms): a
few eps in FP64 and FP32; and in FP64 the fields still agree to 1e-12 after
201 steps.  (In FP32 an ulp of difference changes the outcome of a
stochastic rounding now and then, after which the two are independent
random walks of the same size: the oracle parity of each is in the other GPU
tests, through the tiled step, the default for single runs, and the march,
the default for batches.)  Batches of uneven runs (plain and MHD in one
launch) likewise.  The 16-bit forms step with the tiled kernel only (it
applies their reference table); their oracle parity is in
test_gpu_parity.py.  Also the selection through goc_lbm_set_launch /
goc_lbm_tune."""
import struct

import numpy as np
import pytest

from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu


def cav(nx, ny, storage, **kw):
    return W.Case("cav", nx, ny, "wall", "wall", ("tanh", 2.0), ("tanh", 1.5), flow="cavity", Re=100.0,
                  Ma=0.1, storage=storage, **kw)


def periodic(nx, ny, storage, **kw):
    return W.Case("p", nx, ny, "periodic", "periodic", ("tanh", 0.8), ("tanh", 1.2), flow="free", tau=0.7,
                  body_force=(1e-6, -2e-6), storage=storage, **kw)


def mhd(nx, ny, storage, **kw):
    return W.Case("h", nx, ny, "periodic", "wall", ("uniform", 0.0), ("tanh", 3.0), flow="hartmann", Re=100.0,
                  Ha=20.0, mhd=True, storage=storage, **kw)


def edge(nx, ny, bcx, bcy, storage):
    """The smallest grids (a cavity at Re = 100 is unstable on three rows):
    mild clustering, a body force and moving xi1 walls."""
    return W.Case(f"edge_{nx}x{ny}", nx, ny, bcx, bcy, ("tanh", 1.0) if bcx == "wall" else ("uniform", 0.0),
                  ("tanh", 1.2) if bcy == "wall" else ("uniform", 0.0), flow="free", tau=0.8,
                  body_force=(1e-6, 5e-7), v_wall=(0.003, -0.002), storage=storage)


CASES = {
    "cavity_f64_ragged": (cav(127, 65, "f64"), None, 0.0),
    "cavity_f32_multi_tile": (cav(200, 131, "f32"), None, 0.0),
    "cavity_raw_f64": (cav(70, 45, "f64", collision="raw"), None, 0.0),
    "cavity_srt_f32": (cav(70, 45, "f32", collision="srt"), None, 0.0),
    "cavity_reading_flags": (cav(70, 45, "f64", gi_terms=0, lid_corners=0), None, 0.0),
    "edge_3x3_walls": (edge(3, 3, "wall", "wall", "f64"), None, 0.01),
    "edge_3x3_periodic": (edge(3, 3, "periodic", "periodic", "f64"), None, 0.0),
    "edge_40x5_walls": (edge(40, 5, "wall", "wall", "f64"), None, 0.01),
    "edge_5x40_f32": (edge(5, 40, "wall", "periodic", "f32"), None, 0.0),
    "edge_66x3_periodic_x": (edge(66, 3, "periodic", "wall", "f64"), None, 0.01),
    "channel_periodic_x": (W.channel_64(), None, 0.0),
    "periodic_random_f64": (periodic(96, 70, "f64"), W.smooth_fields(96, 70, seed=11, amp=0.02), 0.0),
    "moving_xi1_walls": (W.Case("cxw", 127, 65, "wall", "wall", ("tanh", 1.5), ("tanh", 1.2), flow="free",
                                tau=0.8, body_force=(0.0, 0.0), v_wall=(0.01, -0.005), storage="f64"),
                         None, 0.01),
    "mhd_f64_ragged": (mhd(65, 33, "f64"), None, 0.0),
    "mhd_f32_multi_tile": (mhd(200, 131, "f32"), None, 0.0),
    "mhd_raw_f64": (mhd(65, 33, "f64", collision="raw"), None, 0.0),
    "mhd_3x5": (W.Case("em", 3, 5, "periodic", "wall", ("uniform", 0.0), ("tanh", 0.5), flow="hartmann", Re=2.0,
                       Ha=2.0, Ma=0.1, mhd=True, storage="f64"), None, 0.0),
    "mhd_walls_all_round": (W.Case("mw", 40, 33, "wall", "wall", ("tanh", 1.0), ("tanh", 2.0), flow="hartmann",
                                   Re=20.0, Ha=5.0, mhd=True, storage="f64"), None, 0.0),
}


def _run(case, init_fields, lid, waves):
    gs, ms, ps = B.derive(case)
    if lid:
        gs.u_wall_hi = lid
    r = B.Run(case, structs=(gs, ms, ps))
    r.set_launch(waves)
    if init_fields is not None:
        r.init(*init_fields)
    return r


# checkpoint header: magic, version, storage, nruns, mhd, step, the sizes of
# the slot pool (D2Q5 slots in its rows), force and reference table, the
# reference base step; then (nx, ny, mhd) per run and the three regions
HEADER = struct.Struct("<8s4i5q")
STORED = {"f64": (np.float64, np.float64), "f32": (np.float32, np.float32)}


def _stored(blob, storage):
    """Raw slot pool (storage format: populations and, with MHD, the D2Q5
    slots) and lagged force of a checkpoint."""
    _, version, _, nruns, _, step, fb, Fb, rb, _ = HEADER.unpack_from(blob)
    assert version == 3
    o = HEADER.size + 12 * nruns + rb
    tf, tF = STORED[storage]
    f = np.frombuffer(blob, dtype=tf, count=fb // np.dtype(tf).itemsize, offset=o)
    F = np.frombuffer(blob, dtype=tF, count=Fb // np.dtype(tF).itemsize, offset=o + fb)
    assert len(blob) == o + fb + Fb
    return step, f, F


# a few units of rounding: eps of FP64 / FP32
LIMIT = {"f64": 8 * 2.0 ** -52, "f32": 8 * 2.0 ** -23}


def _values(a, storage):
    """Stored values as FP64."""
    return a.astype(np.float64)


def _ordered(a):
    """IEEE bit patterns (any width) as integers in the order of their values:
    the difference of two is their distance in ulps."""
    w = a.dtype.itemsize * 8
    bits = a.view({64: np.int64, 32: np.int32}[w]).astype(np.int64)
    mag = bits & ((1 << (w - 1)) - 1)
    return np.where(bits < 0, -mag, mag)


@pytest.mark.parametrize("name", list(CASES))
def test_one_step_within_ulps_of_march(name):
    case, init_fields, lid = CASES[name]
    print("tiled vs march, one step:", name, case.nx, case.ny, case.storage, flush=True)
    m = _run(case, init_fields, lid, 8)
    m.step(120)   # a developed state
    t = _run(case, init_fields, lid, 0)
    assert t.launch_info()["waves_per_cu"] == 0 and m.launch_info()["waves_per_cu"] == 8
    t.set_state(m.get_state())
    t.step(1)
    m.step(1)
    st, ft, Ft = _stored(t.get_state(), case.storage)
    sm, fm, Fm = _stored(m.get_state(), case.storage)
    assert st == sm == 121
    d = np.abs(_ordered(ft) - _ordered(fm))
    print(name, "max ulps", int(d.max()), "differing", f"{np.count_nonzero(d) / d.size:.3%}", flush=True)
    assert np.count_nonzero(d) <= 0.25 * d.size
    # (a stored value may be a small difference of larger terms: bounded by
    # the format's rounding at the largest stored value)
    vt, vm = _values(ft, case.storage), _values(fm, case.storage)
    assert np.max(np.abs(vt - vm)) <= LIMIT[case.storage] * np.max(np.abs(vm))
    # the force is a sum of pressure and stress terms of order c_s^2 rho0
    # that cancel to a much smaller value: compared at their rounding
    scale = m.derived()["cs2"] * case.rho0
    eps = np.finfo(Fm.dtype).eps
    assert np.max(np.abs(Ft.astype(np.float64) - Fm.astype(np.float64))) <= 64 * eps * scale
    t.close()
    m.close()


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c[0].storage == "f64"])
def test_fp64_agrees_with_march_after_201_steps(name):
    case, init_fields, lid = CASES[name]
    print("tiled vs march, FP64:", name, case.nx, case.ny, flush=True)
    t = _run(case, init_fields, lid, 0)
    m = _run(case, init_fields, lid, 8)
    assert t.get_state() == m.get_state()
    for steps in (1, 40, 160):   # single launches and captured graph blocks
        t.step(steps)
        m.step(steps)
    a, b = t.fields(), m.fields()
    un = np.linalg.norm(np.hypot(b["U1"], b["U2"]))
    e = {"rho": float(np.linalg.norm(a["rho"] - b["rho"]) / np.linalg.norm(b["rho"])),
         "U1": float(np.linalg.norm(a["U1"] - b["U1"]) / un),
         "U2": float(np.linalg.norm(a["U2"] - b["U2"]) / un)}
    print(name, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-12, (k, e)
    ft, Ft, gt = t.populations()
    fm, Fm, gm = m.populations()
    assert np.max(np.abs(ft - fm)) < 1e-13 * np.max(np.abs(fm))
    assert np.max(np.abs(Ft - Fm)) < 1e-12 * max(np.max(np.abs(Fm)), 1e-300)
    if case.mhd:
        assert np.max(np.abs(gt - gm)) < 1e-13 * np.max(np.abs(gm))
        for k in ("B1", "B2"):
            assert np.linalg.norm(a[k] - b[k]) <= 1e-12 * np.linalg.norm(np.hypot(b["B1"], b["B2"])), k
    t.close()
    m.close()


def test_default_and_tuner_selection():
    """A single straight run starts on the tiled step; the tuner times it at
    its four tile shapes, each with non-temporal and with plain stores,
    beside the 17 plans of the march and keeps whichever is fastest."""
    r = B.Run(cav(256, 256, "f32"))
    assert r.launch_info()["waves_per_cu"] == 0
    info = r.tune(5)
    assert info["candidates"] == 25   # four shapes x two store policies, 17 march plans
    assert info["us_before"] > 0.0   # the tiled step was in use and was timed
    li = r.launch_info()
    assert li["waves_per_cu"] == info["waves_per_cu"]
    r.close()


BATCHES = {
    "batch_mixed_f64": [cav(70, 45, "f64"), mhd(65, 33, "f64"), cav(130, 70, "f64"), mhd(200, 67, "f64"),
                        edge(3, 3, "wall", "wall", "f64")],
    "batch_hartmann_f32": W.batch_256(n=6),
}


@pytest.mark.parametrize("name", list(BATCHES))
def test_batch_one_step_within_rounding_of_march(name):
    """A batch of uneven runs (plain and MHD in one launch) in one tiled
    launch against the march, one step from the same developed state."""
    runs = BATCHES[name]
    storage = runs[0].storage
    print("tiled vs march, batch:", name, len(runs), storage, flush=True)
    m = B.Run(batch=runs)
    assert m.launch_info()["waves_per_cu"] > 0   # batches start on the march
    m.step(120)
    t = B.Run(batch=runs)
    t.set_launch(0)
    t.set_state(m.get_state())
    t.step(1)
    m.step(1)
    st, ft, Ft = _stored(t.get_state(), storage)
    sm, fm, Fm = _stored(m.get_state(), storage)
    assert st == sm == 121
    d = np.abs(_ordered(ft) - _ordered(fm))
    print(name, "max ulps", int(d.max()), "differing", f"{np.count_nonzero(d) / d.size:.3%}", flush=True)
    assert np.count_nonzero(d) <= 0.25 * d.size
    vt, vm = _values(ft, storage), _values(fm, storage)
    assert np.max(np.abs(vt - vm)) <= LIMIT[storage] * np.max(np.abs(vm))
    t.close()
    m.close()


def test_batch_fp64_agrees_with_march_after_201_steps():
    runs = BATCHES["batch_mixed_f64"]
    t, m = B.Run(batch=runs), B.Run(batch=runs)
    t.set_launch(0)
    for steps in (1, 40, 160):
        t.step(steps)
        m.step(steps)
    for r, case in enumerate(runs):
        a, b = t.fields(run=r), m.fields(run=r)
        un = np.linalg.norm(np.hypot(b["U1"], b["U2"]))
        e = {"rho": float(np.linalg.norm(a["rho"] - b["rho"]) / np.linalg.norm(b["rho"])),
             "U1": float(np.linalg.norm(a["U1"] - b["U1"]) / un),
             "U2": float(np.linalg.norm(a["U2"] - b["U2"]) / un)}
        if case.mhd:
            bn = np.linalg.norm(np.hypot(b["B1"], b["B2"]))
            e["B"] = float(np.linalg.norm(np.hypot(a["B1"] - b["B1"], a["B2"] - b["B2"])) / bn)
        print(r, case.name, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        for k, v in e.items():
            assert v < 1e-12, (r, k, e)
    t.close()
    m.close()


def test_selection_of_the_form():
    """Single straight runs start on the tiled step, batches on the march;
    either takes the other through goc_lbm_set_launch; a run on a 2-D
    metric has only the tiled step."""
    h = B.Run(mhd(65, 33, "f64"))
    assert h.launch_info()["waves_per_cu"] == 0
    h.set_launch(8)
    assert h.launch_info()["waves_per_cu"] == 8
    h.set_launch(0)
    assert h.launch_info()["waves_per_cu"] == 0
    h.close()
    b = B.Run(batch=[cav(70, 45, "f64"), cav(40, 33, "f64")])
    assert b.launch_info()["waves_per_cu"] > 0
    b.set_launch(0)
    li = b.launch_info()
    assert li["waves_per_cu"] == 0 and li["blocks"] == 2 * 12 + 1 * 9   # tiles of 64 x 4 in FP64
    b.close()
    c = B.Run(W.taylor_couette(n1=32, n2=6, R1=8.0, n_theta=20.0))
    assert c.launch_info()["waves_per_cu"] == 0
    c.set_launch(0)
    with pytest.raises(B.GocError) as ei:
        c.set_launch(8)
    assert ei.value.code == B.GOC_EINVAL
    c.close()


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_16bit_storage_has_only_the_tiled_step(storage):
    """The 16-bit forms step with the tiled kernel, single runs and batches
    alike; the march is refused and the tuner times the tiled step only."""
    h = B.Run(mhd(130, 70, storage))
    assert h.launch_info()["waves_per_cu"] == 0
    with pytest.raises(B.GocError) as ei:
        h.set_launch(8)
    assert ei.value.code == B.GOC_EINVAL
    info = h.tune(3)
    assert info["candidates"] == 8 and info["waves_per_cu"] == 0   # four tile shapes x two store policies
    assert h.launch_info()["rows_per_segment"] in (4, 8, 16)
    h.close()
    b = B.Run(batch=[c.replace(storage=storage) for c in W.batch_256(n=3)])
    assert b.launch_info()["waves_per_cu"] == 0
    b.close()


@pytest.mark.parametrize("name", ["cavity_f64_ragged", "mhd_f64_ragged", "moving_xi1_walls"])
def test_tile_heights_agree_fp64(name):
    """The tiled step at 4 and 8 rows per 64-column tile (FP64's heights) and
    in 128 x 4 tiles computes the same step: fields within 1e-13 after 201
    steps."""
    case, init_fields, lid = CASES[name]
    runs = {}
    for rows in (4, 8, "128x4"):
        r = _run(case, init_fields, lid, 0)
        if rows == "128x4":
            r.set_tile(4, cols=128)
        else:
            r.set_tile(rows)
            assert r.launch_info()["rows_per_segment"] == rows
        for steps in (1, 40, 160):
            r.step(steps)
        runs[rows] = r
    b = runs[4].fields()
    un = np.linalg.norm(np.hypot(b["U1"], b["U2"]))
    for other in (8, "128x4"):
        a = runs[other].fields()
        for k in a:
            ref = un if k.startswith("U") else np.linalg.norm(b[k])
            assert np.linalg.norm(a[k] - b[k]) <= 1e-13 * ref, (name, other, k)
    for r in runs.values():
        r.close()


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
def test_tile_heights_agree(storage):
    """The tiled step at 4, 8 and 16 rows per 64-column tile and in 128 x 4
    tiles from the same developed state (a batch of plain and MHD runs): FP32
    stores the same values within a few eps of the largest; the 16-bit forms'
    fields agree far inside their rounding (an ulp of FP32 difference can flip
    a stochastic rounding)."""
    runs = [c.replace(storage=storage) for c in W.batch_256(n=3)] + [cav(130, 70, storage)]
    base = B.Run(batch=runs)
    base.set_launch(0)
    base.step(120)
    blob = base.get_state()
    out = {}
    for rows in (4, 8, 16, "128x4"):
        r = B.Run(batch=runs)
        if rows == "128x4":
            r.set_tile(4, True, cols=128)
            assert r.launch_info()["tile_cols"] == 128
        else:
            r.set_tile(rows, rows == 8)   # (both store policies)
        r.set_state(blob)
        r.step(1)
        out[rows] = r
    for rows in (8, 16, "128x4"):
        for k, case in enumerate(runs):
            if storage == "f32":
                fa, Fa, ga = out[rows].populations(run=k)
                fb, Fb, gb = out[4].populations(run=k)
                assert np.max(np.abs(fa - fb)) <= LIMIT["f32"] * np.max(np.abs(fb)), (rows, k)
                if case.mhd:
                    assert np.max(np.abs(ga - gb)) <= LIMIT["f32"] * np.max(np.abs(gb)), (rows, k)
            else:
                a, b = out[rows].fields(run=k), out[4].fields(run=k)
                un = np.linalg.norm(np.hypot(b["U1"], b["U2"]))
                for q in a:
                    ref = un if q.startswith("U") else np.linalg.norm(b[q])
                    assert np.linalg.norm(a[q] - b[q]) <= 1e-5 * ref, (rows, k, q)
    for r in out.values():
        r.close()
    base.close()
