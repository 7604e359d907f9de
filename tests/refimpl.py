"""Independent brute-force references used to pin the oracle.

Nothing here is shared with the oracle or the HIP library.  The matrices are
built from their definitions (monomials of the lattice velocities), central
moments are taken as explicit sums over populations, inverses come from
numpy.linalg, and the textbook schemes at h = 1 are written from the
standard uniform-grid formulations the paper reduces to.
"""
from __future__ import annotations

import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
# bare moment exponents (m, n) in the order k00 k10 k01 k20 k02 k11 k21 k12 k22
EXPS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def P_matrix():
    """Rows are the monomials e1^m e2^n over the nine lattice velocities."""
    return np.array([[EX[a] ** m * EY[a] ** n for a in range(9)] for (m, n) in EXPS])


def Mc_matrix(U1, U2):
    """Central-moment matrix: rows (e1-U1)^m (e2-U2)^n."""
    return np.array([[(EX[a] - U1) ** m * (EY[a] - U2) ** n for a in range(9)] for (m, n) in EXPS])


def F_matrix(U1, U2):
    """Frame transformation from raw to central moments, built numerically as
    Mc(U) P^-1 (the definition of central moments), not from the expansion."""
    return Mc_matrix(U1, U2) @ np.linalg.inv(P_matrix())


def B_matrix():
    """Combination of the bare second-order diagonal moments into (k20+k02, k20-k02)."""
    B = np.eye(9)
    B[3, 3], B[3, 4] = 1.0, 1.0
    B[4, 3], B[4, 4] = 1.0, -1.0
    return B


def central_by_definition(f, U1, U2):
    return Mc_matrix(U1, U2) @ np.asarray(f)


def raw_eq_sec3(rho, U1, U2, h1, h2, cs2):
    """Bare raw-moment equilibria of the base GOC model (Sec. 3)."""
    P = rho * cs2
    return np.array([
        h1 * h2 * rho,
        h2 * rho * U1,
        h1 * rho * U2,
        h2 / h1 * (rho * U1 * U1 + P),
        h1 / h2 * (rho * U2 * U2 + P),
        rho * U1 * U2,
        rho * (cs2 + U1 * U1) * U2 / h1,
        rho * (cs2 + U2 * U2) * U1 / h2,
        rho * cs2 * cs2 + rho * cs2 * (U1 * U1 + U2 * U2) + rho * U1 * U1 * U2 * U2,
    ])


def raw_src_sec3(F1, F2, U1, U2, h1, h2):
    """Bare raw source moments of the base GOC model (Sec. 3)."""
    return np.array([0.0, F1, F2, 2 * F1 * U1 / h1, 2 * F2 * U2 / h2,
                     F1 * U2 / h2 + F2 * U1 / h1, 0.0, 0.0, 0.0])


def cm_collision_matrix_form(f, rho, U1, U2, h1, h2, cs2, omega, F1, F2, n3, n4):
    """Whole central-moment collision as the explicit matrix product
    f~ = P^-1 F^-1 [m^c + B^-1 L (B m^c,eq - B m^c) + B^-1 (I - L/2) B Phi^c].

    m^c,eq and Phi^c are the central moments (by definition) of the Sec. 3
    raw equilibria and sources; k22^eq is replaced by cs2^2 rho (the paper's
    free choice) and the corrections n3, n4 are added to the combined
    second-order slots."""
    P = P_matrix()
    Pinv = np.linalg.inv(P)
    Fm = F_matrix(U1, U2)
    Finv = np.linalg.inv(Fm)
    B = B_matrix()
    Binv = np.linalg.inv(B)
    L = np.diag(omega)
    mc = Fm @ (P @ f)
    feq = Pinv @ raw_eq_sec3(rho, U1, U2, h1, h2, cs2)
    mceq = Mc_matrix(U1, U2) @ feq
    mceq[8] = cs2 * cs2 * rho
    Beq = B @ mceq
    Beq[3] += n3
    Beq[4] += n4
    S = Pinv @ raw_src_sec3(F1, F2, U1, U2, h1, h2)
    phic = Mc_matrix(U1, U2) @ S
    phic[6:] = 0.0   # third and higher order source central moments are zero
    mct = mc + Binv @ (L @ (Beq - B @ mc)) + Binv @ ((np.eye(9) - L / 2) @ (B @ phic))
    return Pinv @ (Finv @ mct)


# ---------------------------------------------------------------- textbook ----

def textbook_cm_step(f, Fprev, omega, cs2, Fext, bc="periodic"):
    """One step of a textbook D2Q9 central-moment MRT LBM on a uniform
    periodic grid with a constant body force (trapezoidal forcing in the
    'bar' variables).  f[9, ny, nx]; returns (f_new, F_used)."""
    nine, ny, nx = f.shape
    rho = f.sum(axis=0)
    U1 = ((f * EX[:, None, None]).sum(axis=0) + 0.5 * Fprev[0]) / rho
    U2 = ((f * EY[:, None, None]).sum(axis=0) + 0.5 * Fprev[1]) / rho
    B = B_matrix()
    Binv = np.linalg.inv(B)
    L = np.diag(omega)
    ft = np.empty_like(f)
    for j in range(ny):
        for i in range(nx):
            u1, u2, r = U1[j, i], U2[j, i], rho[j, i]
            M = Mc_matrix(u1, u2)
            k = M @ f[:, j, i]
            keq = np.array([r, 0, 0, r * cs2, r * cs2, 0, 0, 0, r * cs2 * cs2])
            s = np.array([0, Fext[0], Fext[1], 0, 0, 0, 0, 0, 0], dtype=float)
            kt = k + Binv @ (L @ (B @ keq - B @ k)) + Binv @ ((np.eye(9) - L / 2) @ (B @ s))
            ft[:, j, i] = np.linalg.solve(M, kt)
    fn = np.empty_like(f)
    for a in range(9):
        fn[a] = np.roll(np.roll(ft[a], int(EY[a]), axis=0), int(EX[a]), axis=1)
    Fused = np.empty((2, ny, nx))
    Fused[0] = Fext[0]
    Fused[1] = Fext[1]
    return fn, Fused


def textbook_cm_init(rho, U1, U2, cs2):
    """Equilibrium populations of the textbook central-moment model."""
    ny, nx = rho.shape
    f = np.empty((9, ny, nx))
    for j in range(ny):
        for i in range(nx):
            r = rho[j, i]
            keq = np.array([r, 0, 0, r * cs2, r * cs2, 0, 0, 0, r * cs2 * cs2])
            f[:, j, i] = np.linalg.solve(Mc_matrix(U1[j, i], U2[j, i]), keq)
    return f


E5X = np.array([0, 1, 0, -1, 0], dtype=float)
E5Y = np.array([0, 0, 1, 0, -1], dtype=float)


def textbook_mhd_step(f, g, Fprev, omega, cs2, Fext, tau_m, mu_m=1.0):
    """One step of a textbook uniform-grid MHD LBM on a periodic grid: the
    central-moment D2Q9 flow solver above coupled to a D2Q5 vector
    distribution for B (Dellar's scheme: g^eq = w [B_i + e_j (u_j B_i -
    B_j u_i)/cs2], w0 = 1/3, w1..4 = 1/6 at cs2 = 1/3), with the current
    density from the non-equilibrium first moments
    dB_i/dx_j = -Lambda^(1)_ji / (cs2 tau_m) and the Lorentz force J x B."""
    nine, ny, nx = f.shape
    rho = f.sum(axis=0)
    U1 = ((f * EX[:, None, None]).sum(axis=0) + 0.5 * Fprev[0]) / rho
    U2 = ((f * EY[:, None, None]).sum(axis=0) + 0.5 * Fprev[1]) / rho
    w = np.array([1 - 2 * cs2, cs2 / 2, cs2 / 2, cs2 / 2, cs2 / 2])
    g = g.reshape(2, 5, ny, nx)
    B = g.sum(axis=1)                      # [2, ny, nx]
    U = np.stack([U1, U2])
    geq = np.empty_like(g)
    for c in range(2):
        for a in range(5):
            e = (E5X[a], E5Y[a])
            adv = sum(e[j] * (U[j] * B[c] - B[j] * U[c]) for j in range(2))
            geq[c, a] = w[a] * (B[c] + adv / cs2)
    dB = np.empty((2, 2, ny, nx))         # dB[j, c] = d B_c / d x_j
    for c in range(2):
        neq = g[c] - geq[c]
        dB[0, c] = -(neq * E5X[:, None, None]).sum(axis=0) / (cs2 * tau_m)
        dB[1, c] = -(neq * E5Y[:, None, None]).sum(axis=0) / (cs2 * tau_m)
    J3 = (dB[0, 1] - dB[1, 0]) / mu_m
    FL1 = -J3 * B[1]
    FL2 = J3 * B[0]
    # flow collision with the Lorentz force added to the body force
    Bm = B_matrix()
    Binv = np.linalg.inv(Bm)
    L = np.diag(omega)
    ft = np.empty_like(f)
    for j in range(ny):
        for i in range(nx):
            u1, u2, r = U1[j, i], U2[j, i], rho[j, i]
            M = Mc_matrix(u1, u2)
            k = M @ f[:, j, i]
            keq = np.array([r, 0, 0, r * cs2, r * cs2, 0, 0, 0, r * cs2 * cs2])
            s = np.array([0, Fext[0] + FL1[j, i], Fext[1] + FL2[j, i], 0, 0, 0, 0, 0, 0])
            kt = k + Binv @ (L @ (Bm @ keq - Bm @ k)) + Binv @ ((np.eye(9) - L / 2) @ (Bm @ s))
            ft[:, j, i] = np.linalg.solve(M, kt)
    gt = g - (g - geq) / tau_m
    fn = np.empty_like(f)
    for a in range(9):
        fn[a] = np.roll(np.roll(ft[a], int(EY[a]), axis=0), int(EX[a]), axis=1)
    gn = np.empty_like(gt)
    for c in range(2):
        for a in range(5):
            gn[c, a] = np.roll(np.roll(gt[c, a], int(E5Y[a]), axis=0), int(E5X[a]), axis=1)
    Fused = np.stack([Fext[0] + FL1, Fext[1] + FL2])
    return fn, gn.reshape(10, ny, nx), Fused


# ------------------------------------------------------- collision variants ----

def raw_collision_matrix_form(f, rho, U1, U2, h1, h2, cs2, omega, F1, F2, n3, n4):
    """Raw-moment MRT collision as the explicit matrix product
    f~ = P^-1 [m + B^-1 L (B m^eq + c - B m) + B^-1 (I - L/2) B sigma]
    with the Sec. 3 raw equilibria and sources and the corrections
    c = (0, 0, 0, n3, n4, 0, 0, 0, 0) on the combined diagonal slots."""
    P = P_matrix()
    Pinv = np.linalg.inv(P)
    B = B_matrix()
    Binv = np.linalg.inv(B)
    L = np.diag(omega)
    m = P @ f
    Beq = B @ raw_eq_sec3(rho, U1, U2, h1, h2, cs2)
    Beq[3] += n3
    Beq[4] += n4
    sig = raw_src_sec3(F1, F2, U1, U2, h1, h2)
    mt = m + Binv @ (L @ (Beq - B @ m)) + Binv @ ((np.eye(9) - L / 2) @ (B @ sig))
    return Pinv @ mt


def product_equilibrium(rho, U1, U2, cs2):
    """Factorised D2Q9 equilibrium: rho times the product over both axes of
    the one-dimensional three-velocity populations that carry the moments
    1, u, cs2 + u^2 of a Maxwellian (phi_0 = 1 - cs2 - u^2,
    phi_+-1 = (cs2 + u^2 +- u)/2).  Arrays of any common shape."""
    def phi(e, u):
        if e == 0:
            return 1.0 - cs2 - u * u
        return 0.5 * (cs2 + u * u + e * u)
    return np.stack([rho * phi(int(EX[a]), U1) * phi(int(EY[a]), U2) for a in range(9)])


def _stream_periodic(ft):
    fn = np.empty_like(ft)
    for a in range(9):
        fn[a] = np.roll(np.roll(ft[a], int(EY[a]), axis=0), int(EX[a]), axis=1)
    return fn


def textbook_product_bgk_step(f, tau, cs2):
    """One step of a uniform periodic D2Q9 BGK LBM with the factorised
    equilibrium and no force."""
    rho = f.sum(axis=0)
    U1 = (f * EX[:, None, None]).sum(axis=0) / rho
    U2 = (f * EY[:, None, None]).sum(axis=0) / rho
    feq = product_equilibrium(rho, U1, U2, cs2)
    return _stream_periodic(f + (feq - f) / tau)


def textbook_raw_mrt_step(f, omega, cs2):
    """One step of a uniform periodic D2Q9 raw-moment MRT LBM (moments of
    the monomial basis, diagonal second moments combined as k20 +- k02) with
    the factorised equilibrium and no force."""
    nine, ny, nx = f.shape
    rho = f.sum(axis=0)
    U1 = (f * EX[:, None, None]).sum(axis=0) / rho
    U2 = (f * EY[:, None, None]).sum(axis=0) / rho
    feq = product_equilibrium(rho, U1, U2, cs2)
    P = P_matrix()
    B = B_matrix()
    Binv = np.linalg.inv(B)
    L = np.diag(omega)
    Pinv = np.linalg.inv(P)
    ft = np.empty_like(f)
    for j in range(ny):
        for i in range(nx):
            m = P @ f[:, j, i]
            meq = P @ feq[:, j, i]
            ft[:, j, i] = Pinv @ (m + Binv @ (L @ (B @ meq - B @ m)))
    return _stream_periodic(ft)
