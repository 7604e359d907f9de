"""The paper's channel validations on the GPU, through the C-ABI, against
their closed forms (Sec. 7.1 and 7.2), at the strip sizes the paper uses:
steady body-force Poiseuille flow on a tanh-clustered 3 x 40 strip (and its
second-order convergence), plane Couette flow with the momentum-augmented
bounce-back of App. C (exact on a uniform grid, second order on a clustered
one) and its start-up transient on the 6 x 50 Roberts grid against the
series solution.  The node positions come from the grid maps of the oracle
(test infrastructure); every value compared comes from the library."""
import math

import numpy as np
import pytest

from oracle import params
from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ycoords(n, stretch):
    kind, p = stretch
    xi = np.arange(n) + 0.5
    if kind == "tanh":
        return params.tanh_two_wall_y(n, p, xi)
    if kind == "roberts":
        return params.roberts_y(n, p, xi)
    return xi


def _run(case, lid=0.0):
    gs, ms, ps = B.derive(case)
    gs.u_wall_hi = lid
    return B.Run(case, structs=(gs, ms, ps)).init()


def _steady(r, field="U1", col=1, chunk=2000, tol=1e-13, maxit=500):
    prev = None
    for _ in range(maxit):
        r.step(chunk)
        u = r.fields()[field][:, col]
        if prev is not None and np.max(np.abs(u - prev)) <= tol * max(np.max(np.abs(u)), 1e-30):
            return u
        prev = u
    raise AssertionError("no steady state")


def test_poiseuille_3x40_steady_second_order(oracle_lib):
    errs = []
    for N in (20, 40):
        case = W.Case("p", 3, N, "periodic", "wall", ("uniform", 0.0), ("tanh", 1.5), flow="channel", Re=10.0,
                      tau=1.0, storage="f64")
        r = _run(case)
        u = _steady(r)
        U = oracle_lib.Model(case).lat.extra["U"]   # centreline speed of the paper's Re
        y = _ycoords(N, case.stretch_y)
        ua = 4 * U * (y / N) * (1 - y / N)
        errs.append(float(np.linalg.norm(u - ua) / np.linalg.norm(ua)))
        r.close()
    print("Poiseuille 3xN, N = 20, 40:", errs, flush=True)
    assert errs[1] < 5e-3
    assert math.log2(errs[0] / errs[1]) > 1.8


def test_couette_steady_exact_and_second_order():
    def steady(N, stretch):
        case = W.Case("c", 3, N, "periodic", "wall", ("uniform", 0.0), stretch, flow="free", tau=1.0,
                      storage="f64")
        r = _run(case, lid=0.02)
        u = _steady(r, tol=1e-14)
        r.close()
        ua = 0.02 * _ycoords(N, stretch) / N
        return float(np.linalg.norm(u - ua) / np.linalg.norm(ua))

    e0 = steady(20, ("uniform", 0.0))
    e1, e2 = steady(20, ("tanh", 1.0)), steady(40, ("tanh", 1.0))
    print("Couette uniform", e0, "tanh N = 20, 40:", e1, e2, flush=True)
    assert e0 < 1e-10
    assert e2 < 2e-3 and math.log2(e1 / e2) > 1.8


def test_couette_6x50_roberts_transient_matches_series():
    case = W.Case("c", 6, 50, "periodic", "wall", ("uniform", 0.0), ("roberts", 1.06), flow="free", tau=1.0,
                  storage="f64")
    r = _run(case, lid=0.02)
    nu, H, U = r.derived()["nu"], 50.0, 0.02
    steps = int(round(0.02 * H * H / nu))
    r.step(steps)
    y = _ycoords(50, case.stretch_y)
    ua = U * y / H
    for n in range(1, 20000):
        ua -= 2 * U / (math.pi * n) * math.exp(-(n * math.pi) ** 2 * nu * steps / H ** 2) * np.sin(
            n * math.pi * (1 - y / H))
    un = r.fields()["U1"][:, 2]
    err = float(np.linalg.norm(un - ua) / np.linalg.norm(ua))
    print("Couette 6x50 Roberts transient at", steps, "steps:", err, flush=True)
    assert err < 5e-3
    r.close()
