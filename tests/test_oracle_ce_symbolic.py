"""Symbolic Chapman-Enskog pin of the equilibrium corrections (Sec. 4-5).

The oracle's correction coefficients D3k, C3, D4k, C4 are checked against the
constraints they must satisfy for the scheme to recover the GOC
Navier-Stokes stresses: with the first-order non-equilibrium moments
obtained from the O(eps) moment system (fluxes taken as moments of
f^eq = P^-1 m^eq by definition, time derivatives eliminated with the
O(eps) conservation laws), the combinations

  -1/2 (1 - w3/2) n3^(1) -/+ 1/2 (1 - w4/2) n4^(1) - w3/4 n3^eq(1) -/+ w4/4 n4^eq(1)

must equal (h2/h1) tau11 and (h1/h2) tau22 (Sec. 4, momentum-flux matching).
The check uses a general curvilinear metric (all four theta_ij non-zero),
smooth analytic fields, sympy derivatives and high-precision evaluation.
"""
import numpy as np
import pytest
import sympy as sp

import refimpl as R


def _setup(uniform_rho=False):
    x1, x2 = sp.symbols("xi1 xi2", real=True)
    h1 = sp.Rational(13, 10) + sp.Rational(2, 10) * sp.sin(sp.Rational(7, 10) * x1 + sp.Rational(3, 10) * x2)
    h2 = sp.Rational(8, 10) + sp.Rational(15, 100) * sp.cos(sp.Rational(4, 10) * x1 - sp.Rational(5, 10) * x2)
    rho = 1 + sp.Rational(5, 100) * sp.sin(sp.Rational(3, 10) * x1 + sp.Rational(11, 10) * x2)
    if uniform_rho:
        rho = sp.Integer(1) + 0 * x1
    U1 = sp.Rational(3, 100) * sp.cos(sp.Rational(9, 10) * x1 - sp.Rational(2, 10) * x2) + sp.Rational(1, 100)
    U2 = sp.Rational(2, 100) * sp.sin(sp.Rational(5, 10) * x1 + sp.Rational(6, 10) * x2)
    F1 = sp.Rational(1, 1000) * sp.sin(x1 + x2)
    F2 = sp.Rational(2, 1000) * sp.cos(x1 - 2 * x2)
    return x1, x2, h1, h2, rho, U1, U2, F1, F2


def _residuals(o, cs2v, w3v, w45v, rho_terms, uniform_rho):
    x1, x2, h1, h2, rho, U1, U2, F1, F2 = _setup(uniform_rho)
    cs2, w3, w4 = cs2v, w3v, w45v
    # equilibrium populations from the Sec. 3 raw equilibria (by definition)
    P = sp.Matrix(R.P_matrix().astype(int))
    Pinv = P.inv()
    meq = sp.Matrix([
        h1 * h2 * rho, h2 * rho * U1, h1 * rho * U2,
        h2 / h1 * (rho * U1**2 + rho * cs2), h1 / h2 * (rho * U2**2 + rho * cs2),
        rho * U1 * U2, rho * (cs2 + U1**2) * U2 / h1, rho * (cs2 + U2**2) * U1 / h2,
        rho * cs2**2 + rho * cs2 * (U1**2 + U2**2) + rho * U1**2 * U2**2])
    feq = Pinv * meq
    ex = [int(v) for v in R.EX]
    ey = [int(v) for v in R.EY]

    def mom(w):  # sum_a w_a feq_a
        return sum(w[a] * feq[a] for a in range(9))

    # conserved O(eps) laws -> time derivatives of rho, M1 = rho U1, M2 = rho U2
    rho_t, M1, M2 = sp.symbols("rho_t M1 M2")
    dt_rho = -(sp.diff(mom(ex), x1) + sp.diff(mom(ey), x2)) / (h1 * h2)
    dt_M1 = (F1 - sp.diff(mom([ex[a] * ex[a] for a in range(9)]), x1)
             - sp.diff(mom([ex[a] * ey[a] for a in range(9)]), x2)) / h2
    dt_M2 = (F2 - sp.diff(mom([ey[a] * ex[a] for a in range(9)]), x1)
             - sp.diff(mom([ey[a] * ey[a] for a in range(9)]), x2)) / h1

    def dt0(expr_of):  # expr_of(rho, M1, M2) -> time derivative by the chain rule
        r, m1, m2 = sp.symbols("r m1 m2")
        e = expr_of(r, m1, m2)
        subs = {r: rho, m1: rho * U1, m2: rho * U2}
        return (sp.diff(e, r).subs(subs) * dt_rho + sp.diff(e, m1).subs(subs) * dt_M1
                + sp.diff(e, m2).subs(subs) * dt_M2)

    n3eq = lambda r, m1, m2: h2 / h1 * m1**2 / r + h1 / h2 * m2**2 / r + (h2 / h1 + h1 / h2) * r * cs2
    n4eq = lambda r, m1, m2: h2 / h1 * m1**2 / r - h1 / h2 * m2**2 / r + (h2 / h1 - h1 / h2) * r * cs2
    T3 = [ex[a] ** 2 + ey[a] ** 2 for a in range(9)]
    T4 = [ex[a] ** 2 - ey[a] ** 2 for a in range(9)]
    flux = lambda T, e: mom([T[a] * e[a] for a in range(9)])
    Psi3 = 2 * (F1 * U1 / h1 + F2 * U2 / h2)
    Psi4 = 2 * (F1 * U1 / h1 - F2 * U2 / h2)
    n3unc = (-dt0(n3eq) - sp.diff(flux(T3, ex), x1) - sp.diff(flux(T3, ey), x2) + Psi3) / w3
    n4unc = (-dt0(n4eq) - sp.diff(flux(T4, ex), x1) - sp.diff(flux(T4, ey), x2) + Psi4) / w4

    nu = cs2 * (1 / w4 - sp.Rational(1, 2))
    zeta = cs2 * (1 / w3 - sp.Rational(1, 2))
    th11 = sp.diff(h1, x1) / h1**2
    th12 = sp.diff(h1, x2) / (h1 * h2)
    th21 = sp.diff(h2, x1) / (h1 * h2)
    th22 = sp.diff(h2, x2) / h2**2
    d1U1, d2U2 = sp.diff(U1, x1), sp.diff(U2, x2)
    tc11 = rho * (zeta + nu) * U2 * th12 + rho * (zeta - nu) * U1 * th21
    tc22 = rho * (zeta + nu) * U1 * th21 + rho * (zeta - nu) * U2 * th12
    tau11 = rho * (zeta + nu) * d1U1 / h1 + rho * (zeta - nu) * d2U2 / h2 + tc11
    tau22 = rho * (zeta + nu) * d2U2 / h2 + rho * (zeta - nu) * d1U1 / h1 + tc22

    omega = [1.0, 1.0, 1.0, float(w3), float(w4), float(w4), 1.0, 1.0, 1.0]
    cfg = o.bare_cfg(cs2=float(cs2), omega=omega, nu=float(nu), zeta=float(zeta), gi_terms=1,
                     rho_terms=rho_terms)
    res = []
    for pt in [(0.3, 0.7), (1.9, -0.4), (-2.2, 3.1)]:
        sub = {x1: sp.Float(pt[0], 40), x2: sp.Float(pt[1], 40)}
        ev = lambda e: float(sp.N(e.subs(sub), 30))
        metric = [ev(h1), ev(h2), ev(th11), ev(th12), ev(th21), ev(th22)]
        flow = [ev(rho), ev(U1), ev(U2), ev(d1U1), ev(d2U2), ev(sp.diff(rho, x1)),
                ev(sp.diff(rho, x2))]
        out = o.collide_node(cfg, np.ones(9), metric, flow, [0.0, 0.0])
        n3c, n4c = out["n3"], out["n4"]
        n3 = ev(n3unc) + n3c
        n4 = ev(n4unc) + n4c
        a3, a4 = 1 - float(w3) / 2, 1 - float(w4) / 2
        lhs11 = -0.5 * a3 * n3 - 0.5 * a4 * n4 - float(w3) / 4 * n3c - float(w4) / 4 * n4c
        lhs22 = -0.5 * a3 * n3 + 0.5 * a4 * n4 - float(w3) / 4 * n3c + float(w4) / 4 * n4c
        rhs11 = ev(h2 / h1 * tau11)
        rhs22 = ev(h1 / h2 * tau22)
        scale = abs(rhs11) + abs(rhs22) + abs(n3c) + abs(n4c)
        res.append(max(abs(lhs11 - rhs11), abs(lhs22 - rhs22)) / scale)
    return max(res)


CASES = [(sp.Rational(1, 20), 1, sp.Rational(3, 2)),
         (sp.Rational(1, 7), sp.Rational(17, 10), sp.Rational(9, 10))]


@pytest.mark.parametrize("cs2v,w3v,w45v", CASES)
def test_corrections_satisfy_ce_constraints(oracle_lib, cs2v, w3v, w45v):
    """Default coefficients: the constraints hold to rounding on a general
    curvilinear metric with non-uniform density."""
    assert _residuals(oracle_lib, cs2v, w3v, w45v, 0, False) < 1e-10


def test_printed_density_terms_break_constraints_only_through_grad_rho(oracle_lib):
    """The printed density-gradient coefficients satisfy the constraints when
    grad rho = 0 and miss them otherwise: the printed deviation terms E3, E4
    disagree with the paper's own O(eps) moment system in their U d(rho)
    cubic terms, which is why the default follows the derivation."""
    cs2v, w3v, w45v = CASES[0]
    assert _residuals(oracle_lib, cs2v, w3v, w45v, 1, True) < 1e-10
    assert _residuals(oracle_lib, cs2v, w3v, w45v, 1, False) > 1e-5
