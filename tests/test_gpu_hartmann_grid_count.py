"""The grid saving of the GOC scheme on the Hartmann channel (Sec. 7.4 and
its grid-count table): 3 x Ny periodic strips with the coupled D2Q5
induction scheme, FP64, Roberts gamma = 1.05 toward both plates against the
uniform grid (the same kernel at h = 1, the standard LBM), Re = 100, Pm = 1,
run from the closed-form profiles for up to 2M steps (tests/hartmann_grid_count.py).

The saving factor K at the error of a GOC grid of N rows is the ratio of the
uniform rows needed for the same relative L2 error to N.  It is bracketed
between uniform grids of K_lo N and K_hi N rows: the first has the larger
error, the second the smaller.  Measured brackets (u_x; B_x):

    Ha = 50,  N = 200, error 2.4e-4 (1.6e-4): 8 < K_u < 16, 4 < K_B < 8
    Ha = 100, N = 360, error 9.2e-4 (2.0e-4): 6.1 < K_u < 12.2, 3.05 < K_B < 6.1

so at these errors the GOC grid saves more than the paper's K = 2.9 and
3.05 (printed for a 1e-5 error, which neither grid reaches at the printed
row counts under these settings; the GOC error falls at second order in N).
"""
import pytest

import hartmann_grid_count as HG

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

STEPS = 2000000


def _run(Ha, ny, scheme):
    print(f"[hartmann-K] Ha {Ha:g} {scheme} 3x{ny}", flush=True)
    r = HG.run_one(Ha, ny, scheme, 100.0, STEPS)
    print(f"[hartmann-K] {r}", flush=True)
    return r


@pytest.mark.parametrize("Ha,n_goc,uniform,u_bracket,b_bracket,u_err,b_err", [
    # uniform rows tried; (K_lo, K_hi) rows for u_x and for B_x; GOC errors
    (50.0, 200, (800, 1600, 3200), (1600, 3200), (800, 1600), 2.4e-4, 1.6e-4),
    (100.0, 360, (1100, 2200, 4400), (2200, 4400), (1100, 2200), 9.2e-4, 2.0e-4),
])
def test_hartmann_grid_saving_factor(Ha, n_goc, uniform, u_bracket, b_bracket, u_err, b_err):
    goc = _run(Ha, n_goc, "goc")
    assert goc["change"] < 2e-6   # (u_x change over the last 20000 steps, relative)
    assert goc["err_u"] == pytest.approx(u_err, rel=0.05)
    assert goc["err_b"] == pytest.approx(b_err, rel=0.05)
    std = {n: _run(Ha, n, "std") for n in uniform}
    # the uniform error falls monotonically with the row count
    errs = [std[n]["err_u"] for n in uniform]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    lo, hi = u_bracket
    assert std[lo]["err_u"] > goc["err_u"] > std[hi]["err_u"], (lo / n_goc, hi / n_goc)
    lo, hi = b_bracket
    assert std[lo]["err_b"] > goc["err_b"] > std[hi]["err_b"], (lo / n_goc, hi / n_goc)
    # and K exceeds the paper's factor at this error
    paper_k = {50.0: 2.9, 100.0: 3.05}[Ha]
    assert u_bracket[0] / n_goc > paper_k


def test_hartmann_wall_error_follows_the_third_order_rates():
    """At 3 x 360, Ha = 100 the error is that of the half-way bounce-back
    walls, which depends on the free third-order rates omega6 = omega7: at
    1.6 instead of 1 the u_x error falls from 9.2e-4 to 1.35e-4 and the B_x
    error from 2.0e-4 to 1.0e-4; the fourth-order rate omega8 plays no part
    in this flow."""
    r = HG.run_one(100.0, 360, "goc", 100.0, STEPS, w3=1.6)
    print(f"[hartmann-K] {r}", flush=True)
    assert r["err_u"] == pytest.approx(1.345e-4, rel=0.05)
    assert r["err_b"] == pytest.approx(1.01e-4, rel=0.05)
    r8 = HG.run_one(100.0, 360, "goc", 100.0, STEPS, w3=1.6, w4=1.6)
    assert r8["err_u"] == pytest.approx(r["err_u"], rel=1e-6)
