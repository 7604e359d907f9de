"""GPU parity of the curvilinear step (general 2-D metric: theta12, theta21
!= 0, h2 varying along xi1) and of walls moving along xi2, through the
C-ABI, against the FP64 oracle.  Tolerances as for the straight grids:
1e-12 in FP64, 1e-5 after 1000 FP32 steps, a few units of the format's
rounding for the 16-bit storage after one step."""
import math

import numpy as np
import pytest

import test_gpu_parity as G
from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(oracle_lib, case, init_fields=None, lid=0.0):
    """GPU run and oracle model of a case; lid: speed of the xi2 = ny wall."""
    gs, ms, ps = B.derive(case)
    gs.u_wall_hi = lid
    g = B.Run(case, structs=(gs, ms, ps))
    mt = W.wavy_metric(case.nx, case.ny, case.grid2d[1]) if case.grid2d and case.grid2d[0] == "wavy" else None
    o = oracle_lib.Model(case, metric2d=mt)
    if lid:
        o.lat.u_wall_hi = lid
        o.cfg = o._make_cfg()
    if init_fields is not None:
        g.init(*init_fields)
        o.init(*init_fields)
    else:
        o.init()
    return g, o


def _tc_errors(gf, of):
    """Relative L2 errors of a circular Couette flow, whose radial velocity U1
    vanishes: both components by the norm of the velocity, rho by its own."""
    un = np.linalg.norm(np.hypot(of["U1"], of["U2"]))
    return {"rho": float(np.linalg.norm(gf["rho"] - of["rho"]) / np.linalg.norm(of["rho"])),
            "U1": float(np.linalg.norm(gf["U1"] - of["U1"]) / un),
            "U2": float(np.linalg.norm(gf["U2"] - of["U2"]) / un)}


def _check(oracle_lib, case, steps, tol, init_fields=None, lid=0.0):
    g, o = _pair(oracle_lib, case, init_fields, lid)
    print(f"[curv] {case.name} {case.nx}x{case.ny} {case.storage} {case.collision} steps={steps}", flush=True)
    g.step(steps)
    o.step(steps)
    if case.grid2d and case.grid2d[0] == "annulus":
        e = _tc_errors(g.fields(), o.fields())
    else:
        e = G.field_errors(g.fields(), o.fields(), o, case.storage)
    print(case.name, case.storage, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < tol, (k, e)
    return g, o


def _wavy(nx, ny, storage="f64", **kw):
    return W.Case(f"wavy_{nx}x{ny}", nx, ny, "wall", "wall", flow="free", tau=0.9,
                  body_force=(1e-6, -5e-7), grid2d=("wavy", 0.3), v_wall=(0.004, -0.006), storage=storage, **kw)


def test_metric_2d_matches_oracle(oracle_lib):
    for case in [W.taylor_couette(n1=70, n2=6, R1=8.0, n_theta=20.0), _wavy(70, 45)]:
        g = B.Run(case)
        mt = W.wavy_metric(case.nx, case.ny, 0.3) if case.grid2d[0] == "wavy" else None
        o = oracle_lib.Model(case, metric2d=mt)
        for name, arr in zip(("h1", "h2", "th11", "th12", "th21", "th22"), g.metric_2d()):
            ref = getattr(o, name)
            assert np.allclose(arr, ref, rtol=1e-13, atol=1e-15 * np.max(np.abs(ref)) + 1e-300), name
        assert g.derived()["cs2"] == pytest.approx(o.lat.cs2, rel=1e-15)


@pytest.mark.parametrize("collision", ["central", "raw"])
def test_taylor_couette_sector_fp64(oracle_lib, collision):
    """The annular sector with both cylinders moving, 300 steps from rest:
    ragged strip (130 radial nodes), periodic azimuth."""
    case = W.taylor_couette(n1=130, n2=6, R1=16.0, n_theta=60 * (130 / 256), collision=collision)
    _check(oracle_lib, case, 300, 1e-12)


@pytest.mark.parametrize("collision", ["central", "raw", "srt"])
def test_wavy_grid_fp64(oracle_lib, collision):
    """Non-separable conformal grid (every theta_ij nonzero), walls on all
    faces with a moving lid and moving xi1 walls, body force, from smooth
    random fields: every curvature term of the stresses, the force and the
    corrections."""
    case = _wavy(70, 45, collision=collision)
    g, o = _pair(oracle_lib, case, W.smooth_fields(70, 45, seed=4, amp=0.01), lid=0.008)
    print(f"[curv] wavy {collision}", flush=True)
    g.step(200)
    o.step(200)
    e = G.field_errors(g.fields(), o.fields(), o, "f64")
    print(collision, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-12, (k, e)


@pytest.mark.parametrize("flags", [dict(gi_terms=0), dict(rho_terms=1), dict(lid_corners=0)])
def test_wavy_grid_reading_flags_fp64(oracle_lib, flags):
    case = _wavy(66, 40, **flags)
    g, o = _pair(oracle_lib, case, W.smooth_fields(66, 40, seed=8, amp=0.01), lid=0.008)
    g.step(100)
    o.step(100)
    e = G.field_errors(g.fields(), o.fields(), o, "f64")
    print(flags, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-12, (k, e)


def test_wavy_grid_periodic_fp64(oracle_lib):
    case = W.Case("wavy_p", 67, 41, "periodic", "periodic", flow="free", tau=0.8,
                  body_force=(2e-6, 1e-6), grid2d=("wavy", 0.2), storage="f64")
    g, o = _pair(oracle_lib, case, W.smooth_fields(67, 41, seed=9, amp=0.01))
    g.step(150)
    o.step(150)
    e = G.field_errors(g.fields(), o.fields(), o, "f64")
    for k, v in e.items():
        assert v < 1e-12, (k, e)


def test_taylor_couette_fp32_1000_steps(oracle_lib):
    case = W.taylor_couette(n1=128, n2=6, R1=16.0, n_theta=60 * 0.5, storage="f32")
    _check(oracle_lib, case, 1000, 1e-5)


def test_wavy_grid_fp32_1000_steps(oracle_lib):
    case = _wavy(96, 64, storage="f32")
    g, o = _pair(oracle_lib, case, W.smooth_fields(96, 64, seed=12, amp=0.01), lid=0.008)
    g.step(1000)
    o.step(1000)
    e = G.field_errors(g.fields(), o.fields(), o, "f32")
    print("wavy f32", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-5, (k, e)


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_wavy_grid_16bit_one_step(oracle_lib, storage):
    case = _wavy(96, 64, storage=storage)
    g, o = _pair(oracle_lib, case, W.smooth_fields(96, 64, seed=12, amp=0.01))
    g.step(1)
    o.step(1)
    e = G.field_errors(g.fields(), o.fields(), o, storage)
    print("wavy", storage, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 4 * G.UNIT[storage], (k, e)


def test_curvilinear_populations_roundtrip(oracle_lib):
    case = _wavy(70, 45)
    o = oracle_lib.Model(case, metric2d=W.wavy_metric(70, 45, 0.3)).init(*W.smooth_fields(70, 45, seed=2, amp=0.01))
    o.step(20)
    g = B.Run(case)
    g.set_populations(o.f, o.F)
    f, F, _ = g.populations()
    assert np.max(np.abs(f - o.f)) <= 2.3e-16 * np.max(np.abs(o.f))
    assert np.array_equal(F, o.F)
    g.step(50)
    o.step(50)
    e = G.field_errors(g.fields(), o.fields(), o, "f64")
    for k, v in e.items():
        assert v < 1e-12, (k, e)


@pytest.mark.parametrize("collision", ["central", "raw"])
def test_straight_grid_moving_xi1_walls_fp64(oracle_lib, collision):
    """The straight march with walls on the xi1 faces moving along xi2 (and a
    moving lid): clustered cavity, 300 steps."""
    case = W.Case("cxw", 127, 65, "wall", "wall", ("tanh", 1.5), ("tanh", 1.2), flow="free", tau=0.8,
                  body_force=(0.0, 0.0), v_wall=(0.01, -0.005), collision=collision, storage="f64")
    g, o = _pair(oracle_lib, case, lid=0.01)
    g.step(300)
    o.step(300)
    e = G.field_errors(g.fields(), o.fields(), o, "f64")
    print("straight xi1 walls", collision, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-12, (k, e)


def test_curvilinear_rejects_mhd():
    case = W.taylor_couette(n1=32, n2=6, R1=8.0, n_theta=20.0)
    g, m, p = B.derive(case)
    p.mhd = 1
    p.tau_m = 1.0
    with pytest.raises(B.GocError) as ei:
        B.Run(case, structs=(g, m, p))
    assert ei.value.code == B.GOC_EINVAL


@pytest.mark.parametrize("u_in,u_out", [(1.0, 2.0), (2.0, 1.0)])
def test_taylor_couette_paper_sector_against_closed_form(u_in, u_out):
    """The curvilinear benchmark at the paper's size: one of 60 sectors,
    256 radial x 6 azimuthal nodes, R1 = 32, R2 = R1 + 256, wall speeds in
    units of U0 = 0.01 (one case of each of its figures), FP64, started from
    the closed-form profile: after 2.4M steps the azimuthal speed matches
    u_theta(r) within 3e-3 (relative L2; about 7e-4 and 2.0e-3 measured), the
    radial speed -- a slowly damped mode of the density's adjustment to the
    centripetal pressure -- is below 1e-3 U0, and the flow is uniform in
    the azimuth."""
    from oracle import params
    U0 = 0.01
    case = W.taylor_couette(n1=256, n2=6, R1=32.0, n_theta=60, U_in=u_in * U0, U_out=u_out * U0)
    g = B.Run(case)
    r = params.annulus(256, 6, 32.0, 288.0, 60)["r"]
    ua = params.taylor_couette(r, 32.0, 288.0, u_in * U0 / 32.0, u_out * U0 / 288.0)
    U2 = np.ascontiguousarray(np.broadcast_to(ua[None, :], (6, 256)))
    g.init(np.ones((6, 256)), np.zeros((6, 256)), U2)
    for k in range(12):
        g.step(200000)
        print(f"[taylor-couette] {u_in}/{u_out}: {(k + 1) * 200000} steps", flush=True)
    fl = g.fields()
    err = np.linalg.norm(fl["U2"][2] - ua) / np.linalg.norm(ua)
    print(f"[taylor-couette] U_in {u_in} U0, U_out {u_out} U0: rel L2 {err:.2e}, "
          f"max |U1| / U0 {np.max(np.abs(fl['U1'])) / U0:.1e}", flush=True)
    assert err < 3e-3
    assert np.max(np.abs(fl["U1"])) < 1e-3 * U0
    assert np.max(np.abs(fl["U2"] - fl["U2"][:1])) < 1e-12 * U0   # azimuthally uniform


def test_curvilinear_batch_fp64(oracle_lib):
    """A batch of curvilinear runs (two annular sectors of different sizes and
    a conformal grid, walls and periodic axes mixed) in one handle: each run
    equals its own oracle run within 1e-12 after 150 steps."""
    runs = [W.taylor_couette(n1=70, n2=6, R1=8.0, n_theta=20.0),
            W.taylor_couette(n1=33, n2=5, R1=4.0, n_theta=9.0, U_in=0.004, U_out=-0.002),
            _wavy(40, 21)]
    g = B.Run(batch=runs)
    g.step(150)
    for r, case in enumerate(runs):
        mt = W.wavy_metric(case.nx, case.ny, 0.3) if case.grid2d[0] == "wavy" else None
        o = oracle_lib.Model(case, metric2d=mt).init()
        o.step(150)
        gf, of = g.fields(run=r), o.fields()
        e = _tc_errors(gf, of) if case.grid2d[0] == "annulus" else G.field_errors(gf, of, o, "f64")
        print(f"[curv batch] run {r} {case.nx}x{case.ny}", {k: f"{v:.1e}" for k, v in e.items()}, flush=True)
        for k, v in e.items():
            assert v < 1e-12, (r, k, e)


def test_curvilinear_checkpoint_resume_is_bitwise():
    case = _wavy(70, 45, storage="f32")
    a = B.Run(case)
    a.init(*W.smooth_fields(70, 45, seed=5, amp=0.01))
    a.step(23)
    blob = a.get_state()
    a.step(120)
    fa, Fa, _ = a.populations()
    b = B.Run(case)
    b.set_state(blob)
    b.step(120)
    fb, Fb, _ = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(Fa, Fb)
    assert b.derived()["step"] == 143
