"""Edge cases of the GPU path against the FP64 oracle: the smallest grids
the method allows (3 nodes per axis, where the one-sided wall differences
span the whole axis and a segment is a single partial group of rows), grids
one node past a 64-column strip or a 4-row group, each boundary combination,
MHD on the smallest channel (each in 64-column tiles and in 128 x 4 tiles,
including grids one node past a 128-column tile), the curvilinear step on
tiny grids, and zero steps."""
import numpy as np
import pytest

import test_gpu_parity as G
from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(oracle_lib, case, lid=0.0, metric2d=None, wide=False):
    gs, ms, ps = B.derive(case)
    gs.u_wall_hi = lid
    g = B.Run(case, structs=(gs, ms, ps))
    if wide:   # 128 x 4 tiles (two waves per tile row)
        g.set_tile(4, cols=128)
        assert g.launch_info()["tile_cols"] == 128
    o = oracle_lib.Model(case, metric2d=metric2d)
    if lid:
        o.lat.u_wall_hi = lid
        o.cfg = o._make_cfg()
    return g, o


def _run(oracle_lib, case, steps=60, lid=0.0, metric2d=None, amp=0.01, wide=False):
    g, o = _pair(oracle_lib, case, lid, metric2d, wide)
    init = W.smooth_fields(case.nx, case.ny, seed=21, amp=amp)
    if case.mhd:
        g.init(*init, np.zeros((case.ny, case.nx)), np.full((case.ny, case.nx), g.derived()["B0"]))
        o.init(*init, np.zeros((case.ny, case.nx)), np.full((case.ny, case.nx), o.lat.B0))
    else:
        g.init(*init)
        o.init(*init)
    print(f"[edge] {case.name} {case.nx}x{case.ny} {case.bc_x}/{case.bc_y} mhd={case.mhd} wide={wide} steps={steps}",
          flush=True)
    g.step(steps)
    o.step(steps)
    f, F, gg = g.populations()
    scale = np.max(np.abs(o.f))
    assert np.max(np.abs(f - o.f)) < 1e-12 * scale, np.max(np.abs(f - o.f)) / scale
    # (F is a sum of pressure and stress terms of order h theta P0 that cancel
    # to a much smaller force: compared at the rounding of those terms)
    assert np.max(np.abs(F - o.F)) <= 1e-12 * np.max(np.abs(o.F)) + 1e-15 * o.lat.cs2 * o.lat.rho0
    if case.mhd:
        assert np.max(np.abs(gg - o.g)) < 1e-12 * np.max(np.abs(o.g))


@pytest.mark.parametrize("nx,ny,bcx,bcy", [
    (3, 3, "wall", "wall"), (3, 3, "periodic", "periodic"), (3, 3, "periodic", "wall"), (3, 3, "wall", "periodic"),
    (3, 7, "wall", "wall"), (7, 3, "wall", "wall"), (65, 5, "wall", "wall"), (64, 9, "periodic", "wall"),
    (66, 3, "periodic", "periodic"), (3, 70, "periodic", "wall"), (129, 5, "wall", "wall"),
    (130, 9, "periodic", "wall"),
])
@pytest.mark.parametrize("collision", ["central", "raw"])
@pytest.mark.parametrize("wide", [False, True], ids=["tile64", "tile128x4"])
def test_smallest_and_edge_sizes_fp64(oracle_lib, nx, ny, bcx, bcy, collision, wide):
    case = W.Case(f"edge_{nx}x{ny}", nx, ny, bcx, bcy, ("tanh", 1.0) if bcx == "wall" else ("uniform", 0.0),
                  ("tanh", 1.2) if bcy == "wall" else ("uniform", 0.0), flow="free", tau=0.8,
                  body_force=(1e-6, 5e-7), v_wall=(0.003, -0.002), collision=collision, storage="f64")
    _run(oracle_lib, case, lid=0.01 if bcy == "wall" else 0.0, wide=wide)


@pytest.mark.parametrize("nx,ny", [(3, 3), (3, 5), (65, 4), (129, 5)])
@pytest.mark.parametrize("wide", [False, True], ids=["tile64", "tile128x4"])
def test_smallest_mhd_channels_fp64(oracle_lib, nx, ny, wide):
    # (mild clustering: with tanh beta = 1.5 over three rows the channel
    # diverges within 60 steps in the oracle too, which then amplifies
    # rounding differences)
    case = W.Case(f"edge_mhd_{nx}x{ny}", nx, ny, "periodic", "wall", ("uniform", 0.0), ("tanh", 0.5),
                  flow="hartmann", Re=2.0, Ha=2.0, Ma=0.1, mhd=True, storage="f64")
    _run(oracle_lib, case, wide=wide)


@pytest.mark.parametrize("nx,ny,bcx,bcy", [(3, 3, "wall", "wall"), (3, 4, "wall", "periodic"),
                                           (65, 5, "periodic", "periodic")])
def test_curvilinear_smallest_sizes_fp64(oracle_lib, nx, ny, bcx, bcy):
    case = W.Case(f"edge_wavy_{nx}x{ny}", nx, ny, bcx, bcy, flow="free", tau=0.9, body_force=(1e-6, 0.0),
                  grid2d=("wavy", 0.2), v_wall=(0.002, -0.003), storage="f64")
    _run(oracle_lib, case, lid=0.004 if bcy == "wall" else 0.0, metric2d=W.wavy_metric(nx, ny, 0.2))


def test_zero_steps_leave_the_state(oracle_lib):
    case = W.Case("zero", 70, 33, "periodic", "wall", ("uniform", 0.0), ("tanh", 1.5), flow="channel",
                  Re=10.0, tau=0.8, storage="f32")
    g = B.Run(case)
    g.init(*W.smooth_fields(70, 33, seed=1, amp=0.01))
    before = g.populations()
    g.step(0)
    after = g.populations()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert g.derived()["step"] == 0
