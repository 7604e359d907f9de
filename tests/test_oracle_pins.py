"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
the definition of a moment set, a matrix built from monomials, an
independently written textbook scheme, an invariant or a closed form.
"""
import math

import numpy as np
import pytest

import refimpl as R


def rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ moment maps ----

def test_P_and_Pinv_match_monomial_matrix(oracle_lib):
    o = oracle_lib
    P = R.P_matrix()
    Pinv = np.linalg.inv(P)
    r = rng(1)
    for _ in range(20):
        f = r.normal(size=9)
        assert np.allclose(o.moment_map(0, f), P @ f, atol=1e-14, rtol=0)
        m = r.normal(size=9)
        assert np.allclose(o.moment_map(3, m), Pinv @ m, atol=1e-14, rtol=0)


def test_frame_transform_is_central_moment_definition(oracle_lib):
    o = oracle_lib
    r = rng(2)
    for _ in range(20):
        f = r.uniform(0.01, 1.0, size=9)
        U1, U2 = r.normal(scale=0.3, size=2)
        m = R.P_matrix() @ f
        kc = o.moment_map(1, m, U1, U2)
        assert np.allclose(kc, R.central_by_definition(f, U1, U2), atol=1e-13, rtol=0)
        # F^-1 = F(-U): the inverse map returns the raw moments
        assert np.allclose(o.moment_map(2, kc, U1, U2), m, atol=1e-13, rtol=0)


def test_central_equilibria_are_binomial_transform_of_raw(oracle_lib):
    """App. E builds the central equilibria from the Sec. 3 raw equilibria by
    the binomial transform (k22 is chosen freely as cs2^2 rho)."""
    o = oracle_lib
    r = rng(3)
    cs2 = 0.05
    cfg = o.bare_cfg(cs2=cs2)
    Pinv = np.linalg.inv(R.P_matrix())
    for _ in range(30):
        h1, h2 = r.uniform(0.2, 3.0, size=2)
        rho = r.uniform(0.8, 1.2)
        U1, U2 = r.normal(scale=0.05, size=2)
        eq, _ = o.central_eq(cfg, h1, h2, rho, U1, U2)
        kc = R.central_by_definition(Pinv @ R.raw_eq_sec3(rho, U1, U2, h1, h2, cs2), U1, U2)
        comb = [kc[0], kc[1], kc[2], kc[3] + kc[4], kc[3] - kc[4], kc[5], kc[6], kc[7]]
        assert np.allclose(eq[:8], comb, rtol=1e-12, atol=1e-15)
        assert eq[8] == pytest.approx(cs2 * cs2 * rho, rel=1e-15)


def test_printed_third_order_coefficients_differ_in_sign(oracle_lib):
    """The printed q21, q12 have the opposite sign of the binomial transform;
    the oracle's default follows the binomial transform, the flag the print."""
    o = oracle_lib
    cs2 = 0.05
    h1, h2, rho, U1, U2 = 1.7, 0.4, 1.0, 0.03, -0.02
    eq_b, _ = o.central_eq(o.bare_cfg(cs2=cs2, q3_sign=0), h1, h2, rho, U1, U2)
    eq_p, _ = o.central_eq(o.bare_cfg(cs2=cs2, q3_sign=1), h1, h2, rho, U1, U2)
    base21 = (1 - h2) * rho * cs2 * U2 / h1
    base12 = (1 - h1) * rho * cs2 * U1 / h2
    assert (eq_b[6] - base21) == pytest.approx(-(eq_p[6] - base21), rel=1e-12)
    assert (eq_b[7] - base12) == pytest.approx(-(eq_p[7] - base12), rel=1e-12)
    assert abs(eq_b[6] - eq_p[6]) > 1e-9


def test_central_sources_are_binomial_transform_of_raw(oracle_lib):
    o = oracle_lib
    r = rng(4)
    cfg = o.bare_cfg()
    Pinv = np.linalg.inv(R.P_matrix())
    for _ in range(30):
        h1, h2 = r.uniform(0.2, 3.0, size=2)
        U1, U2 = r.normal(scale=0.05, size=2)
        F1, F2 = r.normal(scale=1e-3, size=2)
        _, src = o.central_eq(cfg, h1, h2, 1.0, U1, U2, F1, F2)
        sc = R.central_by_definition(Pinv @ R.raw_src_sec3(F1, F2, U1, U2, h1, h2), U1, U2)
        comb = [sc[0], sc[1], sc[2], sc[3] + sc[4], sc[3] - sc[4], sc[5]]
        assert np.allclose(src[:6], comb, rtol=1e-12, atol=1e-18)
        assert np.all(src[6:] == 0.0)


# ------------------------------------------------------- node collision ----

def _random_node(r, straight=False):
    h1, h2 = r.uniform(0.3, 2.5, size=2)
    th = r.normal(scale=0.05, size=4)
    if straight:
        th[1] = th[2] = 0.0
    metric = np.array([h1, h2, th[0], th[1], th[2], th[3]])
    cs2 = r.uniform(0.02, 0.3)
    rho = r.uniform(0.9, 1.1)
    U1, U2 = r.normal(scale=0.03, size=2)
    feq = np.linalg.inv(R.P_matrix()) @ R.raw_eq_sec3(rho, U1, U2, h1, h2, cs2)
    f = feq * (1 + r.normal(scale=0.02, size=9))
    grads = r.normal(scale=1e-3, size=4)
    force = r.normal(scale=1e-5, size=2)
    omega = r.uniform(0.5, 1.8, size=9)
    return metric, cs2, rho, U1, U2, f, grads, force, omega


def test_node_collision_equals_matrix_form(oracle_lib):
    """App. E collision equals the explicit product P^-1 F^-1 [...] with
    matrices built from their definitions, for random inputs with rho and U
    taken from f and a lagged force (as in the time step)."""
    o = oracle_lib
    r = rng(6)
    for _ in range(200):
        metric, cs2, _, _, _, f, grads, force, omega = _random_node(r)
        h1, h2 = metric[0], metric[1]
        Fp = r.normal(scale=1e-5, size=2)
        m = R.P_matrix() @ f
        rho = m[0] / (h1 * h2)
        U1 = (m[1] + Fp[0] / 2) / (rho * h2)
        U2 = (m[2] + Fp[1] / 2) / (rho * h1)
        nu = cs2 * (1 / omega[4] - 0.5)
        cfg = o.bare_cfg(cs2=cs2, omega=omega, nu=nu)
        out = o.collide_node(cfg, f, metric, [rho, U1, U2, *grads], force)
        ref = R.cm_collision_matrix_form(f, rho, U1, U2, h1, h2, cs2, omega, out["F"][0],
                                         out["F"][1], out["n3"], out["n4"])
        assert np.max(np.abs(out["ft"] - ref)) < 1e-13 * np.max(np.abs(f))
        # collision conserves the zeroth moment
        assert abs(out["ft"].sum() - f.sum()) < 1e-14 * abs(f.sum())


def test_local_shear_stress_solves_implicit_equation(oracle_lib):
    """App. A: tau12 = -(1 - w5/2) (k'11 + sigma'11/2 - rho U1 U2) with
    sigma'11 built from the full effective force F = F~ + 2 h theta tau12,
    and F equals the full effective-force expressions of Sec. 2.2."""
    o = oracle_lib
    r = rng(7)
    for _ in range(100):
        metric, cs2, rho, U1, U2, f, grads, force, omega = _random_node(r)
        h1, h2, t11, t12, t21, t22 = metric
        nu = cs2 * (1 / omega[4] - 0.5)
        zeta = cs2 * (1 / omega[3] - 0.5)
        cfg = o.bare_cfg(cs2=cs2, omega=omega, nu=nu)
        out = o.collide_node(cfg, f, metric, [rho, U1, U2, *grads], force)
        F1, F2 = out["F"]
        tau12 = out["tau12"]
        k11 = (R.P_matrix() @ f)[5]
        s11 = F1 * U2 / h2 + F2 * U1 / h1
        resid = tau12 + (1 - omega[5] / 2) * (k11 + 0.5 * s11 - rho * U1 * U2)
        assert abs(resid) < 1e-15 + 1e-12 * abs(tau12)
        d1U1, d2U2 = grads[0], grads[1]
        tc11 = rho * (zeta + nu) * U2 * t12 + rho * (zeta - nu) * U1 * t21
        tc22 = rho * (zeta + nu) * U1 * t21 + rho * (zeta - nu) * U2 * t12
        tau11 = rho * (zeta + nu) * d1U1 / h1 + rho * (zeta - nu) * d2U2 / h2 + tc11
        tau22 = rho * (zeta + nu) * d2U2 / h2 + rho * (zeta - nu) * d1U1 / h1 + tc22
        P = rho * cs2
        F1ref = h2 * (force[0] + (t21 - t11) * P + t11 * (tau11 - rho * U1 * U1)
                      + 2 * t12 * (tau12 - rho * U1 * U2) - t21 * (tau22 - rho * U2 * U2))
        F2ref = h1 * (force[1] + (t12 - t22) * P + t22 * (tau22 - rho * U2 * U2)
                      + 2 * t21 * (tau12 - rho * U1 * U2) - t12 * (tau11 - rho * U1 * U1))
        assert F1 == pytest.approx(F1ref, rel=1e-11, abs=1e-18)
        assert F2 == pytest.approx(F2ref, rel=1e-11, abs=1e-18)


def test_corrections_vanish_at_unit_metric_low_mach(oracle_lib):
    """App. B(ii) at h1 = h2 = 1, theta = 0, cs2 = 1/3: all correction
    coefficients are zero, so the GOC model is the uniform-grid one."""
    o = oracle_lib
    r = rng(8)
    for _ in range(50):
        omega = r.uniform(0.6, 1.9, size=9)
        cfg = o.bare_cfg(cs2=1 / 3, omega=omega, nu=(1 / 3) * (1 / omega[4] - 0.5), gi_terms=0)
        f = r.uniform(0.01, 0.5, size=9)
        out = o.collide_node(cfg, f, [1, 1, 0, 0, 0, 0], [1.0, 0.05, -0.04, *r.normal(size=4)],
                             [1e-4, 0])
        # zero up to the rounding of c_s^2 = 1/3 in the coefficient sums
        assert abs(out["n3"]) < 1e-15 and abs(out["n4"]) < 1e-15


def test_full_corrections_at_unit_metric_are_cubic(oracle_lib):
    """With the full coefficients at h = 1 the corrections are the cubic
    Galilean-invariance terms: they scale as U^2 * gradient (Ma^3)."""
    o = oracle_lib
    cfg = o.bare_cfg(cs2=1 / 3, omega=[1, 1, 1, 1, 1.5, 1.5, 1, 1, 1],
                     nu=(1 / 3) * (1 / 1.5 - 0.5), gi_terms=1)
    f = np.full(9, 0.1)
    vals = []
    for s in [1e-2, 5e-3]:
        out = o.collide_node(cfg, f, [1, 1, 0, 0, 0, 0], [1.0, s, s / 2, s, s, s * s, s * s],
                             [0, 0])
        vals.append(abs(out["n3"]) + abs(out["n4"]))
    assert vals[0] / vals[1] == pytest.approx(8.0, rel=0.05)


# ------------------------------------------------------------- metric ----

def test_tanh_metric_is_derivative_of_mapping(oracle_lib):
    from oracle import params
    for n, beta in [(64, 1.5), (1024, 2.0), (1024, 3.0), (50, 0.7)]:
        h, dh, th, lo, hi = params.tanh_two_wall(n, beta)
        xi = np.arange(n) + 0.5
        eps = 1e-5
        hfd = (params.tanh_two_wall_y(n, beta, xi + eps) - params.tanh_two_wall_y(n, beta, xi - eps)) / (2 * eps)
        assert np.allclose(h, hfd, rtol=1e-8)
        # walls map to 0 and L, so the node-centred midpoint sum of h is L to O(1/n^2)
        assert params.tanh_two_wall_y(n, beta, 0.0) == pytest.approx(0.0, abs=1e-12)
        assert params.tanh_two_wall_y(n, beta, float(n)) == pytest.approx(n, rel=1e-14)
        # theta = (1/h^2) dh/dxi against a finite difference of h
        hp = params.tanh_two_wall(n, beta)[0]
        x2 = xi[1:-1]
        hfd2 = (np.interp(x2 + 1, xi, hp) - np.interp(x2 - 1, xi, hp)) / 2
        assert np.allclose(dh[1:-1], hfd2, rtol=0.05, atol=1e-3 * np.max(np.abs(dh)))
        assert np.allclose(th, dh / h**2)
        # the paper's printed curvature formula with L_y = n
        u = beta * (1 - 2 * xi / n)
        th_paper = 4 * math.tanh(beta) / n * np.tanh(u) / (1 / np.cosh(u) ** 2)
        assert np.allclose(th, th_paper, rtol=1e-12)


def test_roberts_metric_is_derivative_of_mapping(oracle_lib):
    from oracle import params
    for n, gamma in [(40, 1.06), (360, 1.05)]:
        h, dh, th, lo, hi = params.roberts(n, gamma)
        xi = np.arange(n) + 0.5
        eps = 1e-5
        hfd = (params.roberts_y(n, gamma, xi + eps) - params.roberts_y(n, gamma, xi - eps)) / (2 * eps)
        assert np.allclose(h, hfd, rtol=1e-7)
        assert params.roberts_y(n, gamma, 0.0) == pytest.approx(0.0, abs=1e-10)
        assert params.roberts_y(n, gamma, float(n)) == pytest.approx(n, rel=1e-12)
        lam = (gamma + 1) / (gamma - 1)
        s = (xi / n - 0.5) / 0.5
        th_paper = (1 / n) * (2 / (2 * gamma)) * (lam ** (-s) - lam**s)
        assert np.allclose(th, th_paper, rtol=1e-10)


def test_sound_speed_values():
    """Sec. 3.2.1 at the benchmark grids: q = min h."""
    from oracle import params
    h = params.tanh_two_wall(64, 1.5)[0]
    assert params.sound_speed_sq(np.ones(64), h) == pytest.approx(h.min() ** 2 / 3)
    assert h.min() == pytest.approx(0.3124, abs=2e-4)
    assert params.tanh_two_wall(1024, 3.0)[0].min() == pytest.approx(0.0299, abs=1e-4)
