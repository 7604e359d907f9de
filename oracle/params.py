"""Oracle-side grid metric and lattice-parameter relations, in FP64.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  Written from
the paper independently of the HIP library's own parameter code.

Node convention (reading of Sec. 6 against the half-way bounce-back of
Sec. 7): node j sits at xi = j + 1/2 of a computational length L_xi = N, the
walls at xi = 0 and xi = N map onto y = 0 and y = L_y = N, so the mean metric
factor is one.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- metric ----

def tanh_two_wall(n: int, beta: float):
    """Sec. 6.1, hyperbolic stretching clustered at both walls.

    y(xi) = (L/2) {1 - tanh[beta (1 - 2 xi/L)] / tanh beta},  L = n.
    Returns (h, dh, theta, h_face_lo, h_face_hi) with h = dy/dxi and
    dh = dh/dxi at the node centres xi = j + 1/2, theta = dh/(h^2) (the
    diagonal curvature element of Sec. 2.1) and h on the two wall faces.
    beta = 0 is the uniform grid h = 1.
    """
    xi = np.arange(n, dtype=np.float64) + 0.5
    if beta == 0.0:
        one = np.ones(n)
        return one, np.zeros(n), np.zeros(n), 1.0, 1.0
    L = float(n)
    u = beta * (1.0 - 2.0 * xi / L)
    sech2 = 1.0 / np.cosh(u) ** 2
    c = beta / math.tanh(beta)
    h = c * sech2
    # d/dxi of c sech^2(u) = c * (-2 sech^2 tanh) * du/dxi, du/dxi = -2 beta / L
    dh = c * sech2 * np.tanh(u) * (4.0 * beta / L)
    theta = dh / h**2
    hf = c / math.cosh(beta) ** 2
    return h, dh, theta, hf, hf


def tanh_two_wall_y(n: int, beta: float, xi):
    """Physical coordinate y(xi) of the same mapping (used by the pins)."""
    L = float(n)
    if beta == 0.0:
        return np.asarray(xi, dtype=np.float64)
    return 0.5 * L * (1.0 - np.tanh(beta * (1.0 - 2.0 * np.asarray(xi) / L)) / math.tanh(beta))


def roberts(n: int, gamma: float, alpha: float = 0.5):
    """Sec. 6.2, Roberts boundary-layer transformation.

    y = L [A l - B] / [C (1 + l)], l = lambda^s, s = (xi/L - alpha)/(1 - alpha),
    A = gamma + 2 alpha, B = gamma - 2 alpha, C = 2 alpha + 1.
    reading: lambda = (gamma + 1)/(gamma - 1) (the printed ratio is one).
    Returns (h, dh, theta, h_face_lo, h_face_hi) at node centres.
    """
    lam = (gamma + 1.0) / (gamma - 1.0)
    L = float(n)
    A, B, C = gamma + 2 * alpha, gamma - 2 * alpha, 2 * alpha + 1
    k = math.log(lam) / (L * (1.0 - alpha))

    def h_dh(x):
        s = (np.asarray(x, dtype=np.float64) / L - alpha) / (1.0 - alpha)
        l = lam**s
        h = (L / C) * (A + B) * k * l / (1 + l) ** 2
        dh = (L / C) * (A + B) * k * k * l * (1 - l) / (1 + l) ** 3
        return h, dh

    xi = np.arange(n, dtype=np.float64) + 0.5
    h, dh = h_dh(xi)
    theta = dh / h**2
    return h, dh, theta, float(h_dh(0.0)[0]), float(h_dh(L)[0])


def roberts_y(n: int, gamma: float, xi, alpha: float = 0.5):
    """Physical coordinate y(xi) of the Roberts mapping (used by the pins)."""
    lam = (gamma + 1.0) / (gamma - 1.0)
    L = float(n)
    s = (np.asarray(xi, dtype=np.float64) / L - alpha) / (1.0 - alpha)
    l = lam**s
    return L * ((gamma + 2 * alpha) * l - gamma + 2 * alpha) / ((2 * alpha + 1) * (1 + l))


def annulus(n1: int, n2: int, a: float, Ro: float, n_theta: float):
    """Conformal map of an annular sector (the Taylor-Couette section):
    Z = a exp(pi W / N_theta), shifted and scaled so that xi1 in [0, n1]
    spans the radii a..Ro and xi2 in [0, n2] the polar angles
    -pi/N_theta..pi/N_theta (node-centred reading: L_xi = n).  With
    k = ln(Ro/a)/n1: r(xi1) = a exp(k xi1), h1 = a k exp(k xi1),
    h2 = (2 pi a/(N_theta n2)) exp(k xi1), theta11 = theta21 = k/h1 =
    exp(-k xi1)/a, theta12 = theta22 = 0.  Returns a dict of [n2, n1]
    node arrays h1, h2, th11, th12, th21, th22, the radius r, and the
    face values h1 on the xi1 = 0 / n1 walls per row and h2 beside them."""
    k = math.log(Ro / a) / n1
    xi1 = np.arange(n1, dtype=np.float64) + 0.5
    e = np.exp(k * xi1)
    h1 = a * k * e
    h2 = 2.0 * math.pi * a / (n_theta * n2) * e
    th = np.exp(-k * xi1) / a
    rep = lambda v: np.ascontiguousarray(np.broadcast_to(v[None, :], (n2, n1)))
    zero = np.zeros((n2, n1))
    h2w = 2.0 * math.pi * a / (n_theta * n2)
    return dict(h1=rep(h1), h2=rep(h2), th11=rep(th), th12=zero.copy(), th21=rep(th), th22=zero.copy(),
                r=a * e, h1_face_lo=np.full(n2, a * k), h1_face_hi=np.full(n2, Ro * k),
                h2_face_xlo=np.full(n2, h2w), h2_face_xhi=np.full(n2, h2w * Ro / a))


def taylor_couette(r, R1: float, R2: float, Omega1: float, Omega2: float):
    """Azimuthal speed u_theta(r) of steady circular Couette flow between
    cylinders of radii R1 < R2 rotating at Omega1, Omega2."""
    q = (R1 / R2) ** 2
    r = np.asarray(r, dtype=np.float64)
    return ((Omega2 - Omega1 * q) * r + R1 * R1 / r * (Omega1 - Omega2)) / (1.0 - q)


def metric_from_arrays(h1, h2, periodic_x: bool = False, periodic_y: bool = False):
    """Curvature elements of a 2-D orthogonal metric given at the nodes
    ([ny, nx] arrays, unit node spacing), Sec. 2.1: theta11 = d1h1/h1^2,
    theta12 = d2h1/(h1 h2), theta21 = d1h2/(h1 h2), theta22 = d2h2/h2^2,
    with second-order differences: central inside, wrapped along a periodic
    axis, one-sided second order at the ends of a walled one."""
    def d(f, axis, periodic):
        if periodic:
            return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))
        return np.gradient(f, axis=axis, edge_order=2)
    d1h1, d2h1 = d(h1, 1, periodic_x), d(h1, 0, periodic_y)
    d1h2, d2h2 = d(h2, 1, periodic_x), d(h2, 0, periodic_y)
    return dict(th11=d1h1 / h1**2, th12=d2h1 / (h1 * h2), th21=d1h2 / (h1 * h2), th22=d2h2 / h2**2)


# ------------------------------------------------------------ parameters ----

def sound_speed_sq(h1, h2):
    """Sec. 3.2.1: c_s = q / sqrt(3) with q the minimum metric factor of the domain."""
    q = min(float(np.min(h1)), float(np.min(h2)))
    return q * q / 3.0


def viscosity_from_tau(cs2: float, tau: float) -> float:
    """Shear viscosity nu = c_s^2 (1/omega - 1/2) with omega = 1/tau (Sec. 4)."""
    return cs2 * (tau - 0.5)


def omega_from_viscosity(cs2: float, nu: float) -> float:
    """Inverse of nu = c_s^2 (1/omega - 1/2)."""
    return 1.0 / (nu / cs2 + 0.5)


def poiseuille(H: float, nu: float, Re: float, rho0: float = 1.0):
    """Sec. 7.1: Re = U (H/2)/nu and U = F (H/2)^2 / (2 nu); returns (U, F)."""
    U = Re * nu / (H / 2.0)
    F = 2.0 * nu * U * rho0 / (H / 2.0) ** 2
    return U, F


def hartmann(H: float, Ha: float, Re: float, Pm: float, Uc: float, rho0: float = 1.0,
             mu_m: float = 1.0):
    """Sec. 7.4 Hartmann flow between plates 2H apart.

    reading: Re = U_c H / nu with U_c the analytic centre-line velocity;
    eta = nu / Pm; Ha = B0 H sqrt(sigma/(rho nu)) with sigma = 1/(eta mu_m);
    U_r = H^2 F/(rho nu) and u(0) = U_r (1 - sech Ha)/(Ha tanh Ha).
    Returns dict(nu, eta, B0, F, Ur, Br).
    """
    nu = Uc * H / Re
    eta = nu / Pm
    sigma = 1.0 / (eta * mu_m)
    B0 = Ha / (H * math.sqrt(sigma / (rho0 * nu))) if Ha > 0 else 0.0
    if Ha > 0:
        shape = (1.0 - 1.0 / math.cosh(Ha)) / (Ha * math.tanh(Ha))
    else:
        shape = 0.5  # Poiseuille limit of the same profile: u(0) = H^2 F/(2 rho nu)
    F = Uc * rho0 * nu / (H * H * shape)
    Ur = H * H * F / (rho0 * nu)
    Br = H * H * F * mu_m * math.sqrt(sigma / (rho0 * nu))
    return dict(nu=nu, eta=eta, B0=B0, F=F, Ur=Ur, Br=Br, sigma=sigma)


def hartmann_profile(ystar, Ha: float, Ur: float, Br: float):
    """Closed-form u_x(y*) and B_x(y*) of Sec. 7.4, y* in [-1, 1] from the centre."""
    y = np.asarray(ystar, dtype=np.float64)
    u = Ur * (1.0 / (Ha * math.tanh(Ha))) * (1.0 - np.cosh(Ha * y) / math.cosh(Ha))
    b = Br * (-y / Ha + (1.0 / (Ha * math.tanh(Ha))) * np.sinh(Ha * y) / math.cosh(Ha))
    return u, b
