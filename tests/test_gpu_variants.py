"""GPU parity of the two collision variants (raw-moment MRT and SRT) through
the C-ABI against the FP64 oracle's own implementations of them, at the
tolerances of the central-moment model: 1e-12 in FP64, 1e-5 after 1000 FP32
steps, 1e-3 after 1000 steps of the 16-bit storage.  The
oracle computes SRT in velocity space (f^eq and S as P^-1 of their moments,
with its own coefficients G_j, H_j); the library runs it as the raw-moment
body with equal rates."""
import numpy as np
import pytest

import test_gpu_parity as G
from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["raw", "srt"]


@pytest.mark.parametrize("collision", VARIANTS)
@pytest.mark.parametrize("nx,ny", [(127, 65), (63, 200)])
def test_variant_cavity_fp64_ragged(oracle_lib, collision, nx, ny):
    """Walled cavity with a moving lid and clustering on both axes, ragged
    strip and segment tails, 300 steps."""
    G.check(oracle_lib, G.cavity(nx, ny, "f64", collision=collision), 300, 1e-12)


@pytest.mark.parametrize("collision", VARIANTS)
def test_variant_periodic_random_fields_fp64(oracle_lib, collision):
    """Fully periodic, clustered in both directions, from smooth random
    fields with a body force: every equilibrium, correction and source term."""
    case = W.Case("p", 96, 70, "periodic", "periodic", ("tanh", 0.8), ("tanh", 1.2), flow="free",
                  tau=0.7, body_force=(1e-6, -2e-6), collision=collision, storage="f64")
    G.check(oracle_lib, case, 200, 1e-12, init_fields=W.smooth_fields(96, 70, seed=11, amp=0.02))


@pytest.mark.parametrize("collision", VARIANTS)
@pytest.mark.parametrize("flags", [dict(gi_terms=0), dict(lid_corners=0)])
def test_variant_reading_flags_fp64(oracle_lib, collision, flags):
    case = G.cavity(70, 45, "f64", collision=collision, **flags)
    G.check(oracle_lib, case, 100, 1e-12, init_fields=W.smooth_fields(70, 45, seed=5, amp=0.01))


def test_raw_printed_density_terms_fp64(oracle_lib):
    case = G.cavity(70, 45, "f64", collision="raw", rho_terms=1)
    G.check(oracle_lib, case, 100, 1e-12, init_fields=W.smooth_fields(70, 45, seed=6, amp=0.01))


@pytest.mark.parametrize("collision", VARIANTS)
def test_variant_mhd_fp64(oracle_lib, collision):
    """Coupled D2Q5 induction with the variant flow collision (Lorentz force
    through the sources), 300 steps."""
    case = W.Case("h64", 70, 40, "periodic", "wall", ("uniform", 0.0), ("tanh", 3.0),
                  flow="hartmann", Re=100.0, Ha=30.0, mhd=True, collision=collision, storage="f64")
    G.check(oracle_lib, case, 300, 1e-12)


@pytest.mark.parametrize("collision", VARIANTS)
def test_variant_cavity_fp32_1000_steps(oracle_lib, collision):
    """The 1024^2 Re = 1000 cavity's parameters on a 130x97 grid in FP32,
    1000 steps, within 1e-5."""
    case = W.cavity_1024().replace(name=f"cav32_{collision}", nx=130, ny=97,
                                   Re=1000.0 * 130 / 1024, collision=collision)
    G.check(oracle_lib, case, 1000, 1e-5)


def _developed(oracle_lib, collision, storage, nx=256, ny=128):
    case = W.hartmann_4096().replace(name=f"hd_{collision}_{storage}", nx=nx, ny=ny,
                                     storage=storage, collision=collision)
    g = B.Run(case)
    d = g.derived()
    init = W.hartmann_start(case, d["nu"], d["F1"], d["eta"], d["B0"])
    g.init(*init)
    o = oracle_lib.Model(case).init(*init)
    print(f"[parity] developed Hartmann {collision} {nx}x{ny} {storage}", flush=True)
    return g, o


@pytest.mark.parametrize("collision", VARIANTS)
def test_variant_fp32_developed_hartmann_1000_steps(oracle_lib, collision):
    g, o = _developed(oracle_lib, collision, "f32")
    g.step(1000)
    o.step(1000)
    e = G.field_errors(g.fields(), o.fields(), o, "f32")
    print(collision, "f32 developed", {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-5, (k, e)


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_raw_16bit_developed_hartmann_1000_steps(oracle_lib, storage):
    """The raw-moment body in the precision form: every field within 1e-3 of
    the FP64 oracle after 1000 steps from the developed Hartmann state."""
    g, o = _developed(oracle_lib, "raw", storage)
    g.step(1000)
    o.step(1000)
    e = G.field_errors(g.fields(), o.fields(), o, storage)
    print("raw", storage, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < 1e-3, (k, e)


@pytest.mark.parametrize("collision", VARIANTS)
def test_variant_batch_fp64(oracle_lib, collision):
    """Batched form with a variant collision: 4 uneven runs of the seeded
    batch in one launch per step, FP64, 300 steps, each within 1e-12 of its
    own oracle run."""
    runs = [c.replace(storage="f64", collision=collision) for c in W.batch_256(n=4)]
    g = B.Run(batch=runs)
    g.step(300)
    for r, case in enumerate(runs):
        o = oracle_lib.Model(case).init()
        o.step(300)
        e = G.field_errors(g.fields(run=r), o.fields(), o, "f64")
        print(f"[batch {collision}] run {r} {case.nx}x{case.ny}", {k: f"{v:.1e}" for k, v in e.items()},
              flush=True)
        for k, v in e.items():
            assert v < 1e-12, (r, k, e)


def test_srt_derived_viscosities_are_equal():
    """SRT relaxes every moment at 1/tau: the library reports zeta = nu."""
    g = B.Run(G.cavity(40, 30, "f64", collision="srt"))
    d = g.derived()
    assert d["zeta"] == pytest.approx(d["nu"], rel=1e-15)


def _survives(collision, N, Re, steps=200000, chunk=10000):
    """Run the beta = 1.2 clustered cavity (lid at Mach 0.1 of the GOC sound
    speed, bulk viscosity equal to the shear viscosity, full corrections)
    in FP64; True if after `steps` steps every population is finite and
    max |U| stays below twice the lid speed."""
    case = W.Case(f"stab_{collision}", N, N, "wall", "wall", ("tanh", 1.2), ("tanh", 1.2),
                  flow="cavity", Re=Re, Ma=0.1, u_lid=0.0, collision=collision, storage="f64")
    g, m, p = B.derive(case)
    p.omega[3] = p.omega[4]          # zeta = nu, the SRT model's own bulk viscosity
    run = B.Run(case, structs=(g, m, p))
    lid = float(g.u_wall_hi)
    done = 0
    try:
        while done < steps:
            try:
                run.step(chunk)
            except B.GocError as e:   # the watchdog found non-finite values
                if e.code != B.GOC_EUNSTABLE:
                    raise
                print(f"[stability] {collision} N={N} Re={Re:g}: watchdog at step {done + chunk}", flush=True)
                return False
            done += chunk
            dg = run.diagnostics()
            if dg[7] > 0 or not np.isfinite(dg[6]) or dg[6] > 2.0 * lid:
                print(f"[stability] {collision} N={N} Re={Re:g}: unstable at step {done}", flush=True)
                return False
        print(f"[stability] {collision} N={N} Re={Re:g}: stable for {steps} steps, "
              f"max|U| = {dg[6] / lid:.3f} U_lid", flush=True)
        return True
    finally:
        run.close()


def test_stability_ranking_on_clustered_cavity():
    """The stability ranking of the three collision models on a coarse
    clustered cavity (128^2, tanh beta = 1.2 toward all walls): all are
    stable at Re = 100; at Re = 200 the SRT model fails while both MRT
    models hold; at Re = 5000 the raw-moment model fails while the
    central-moment model holds.  Every model has the same shear and bulk
    viscosity, so only the collision differs."""
    assert all(_survives(c, 128, 100.0) for c in ("srt", "raw", "central"))
    assert not _survives("srt", 128, 200.0)
    assert _survives("raw", 128, 200.0) and _survives("central", 128, 200.0)
    assert not _survives("raw", 128, 5000.0)
    assert _survives("central", 128, 5000.0)
