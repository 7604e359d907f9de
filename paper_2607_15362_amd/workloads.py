"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds only problem descriptions and seeded random draws: grid
sizes, boundary types, stretching parameters, the physical parameters
(Re, Ha, Pm, Ma, tau, lid speed) and smooth random initial fields.  It holds
none of the method's arithmetic; the HIP library and the oracle each derive
their lattice parameters and metric factors from these descriptions with
their own code.

The workloads follow the paper's benchmark families (Sec. 7): the
body-force channel of Sec. 7.1, the lid-driven cavity of Sec. 7.3 and the
Hartmann flow of Sec. 7.4, all on tanh-clustered grids (Sec. 6.1).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

STORAGES = ("f64", "f32", "f16dev", "bf16dev")


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    bc_x: str = "periodic"            # "periodic" | "wall"
    bc_y: str = "wall"
    stretch_x: tuple = ("uniform", 0.0)   # ("uniform", 0) | ("tanh", beta) | ("roberts", gamma)
    stretch_y: tuple = ("uniform", 0.0)
    flow: str = "channel"             # "channel" | "cavity" | "hartmann" | "free"
    Re: float = 10.0
    Ha: float = 0.0
    Pm: float = 1.0
    Ma: float = 0.1
    tau: float = 0.8                  # channel / free flows: shear relaxation time
    u_lid: float = 0.0                # cavity: top-wall speed (<= 0: Ma * c_s)
    tau_max: float = 0.0              # Hartmann / cavity: cap on the shear relaxation time (0: none)
    rho0: float = 1.0
    mu_m: float = 1.0
    mhd: bool = False
    storage: str = "f32"
    steps: int = 100
    gi_terms: int = 1
    q3_sign: int = 0
    lid_corners: int = 1
    rho_terms: int = 0
    collision: str = "central"        # "central" | "raw" (moment MRT) | "srt"
    grid2d: tuple | None = None       # general 2-D metric: ("annulus", a, Ro, n_theta) or
                                      # ("wavy", eps) (node arrays from wavy_metric)
    v_wall: tuple = (0.0, 0.0)        # xi2 velocity of the walls at xi1 = 0 and xi1 = nx
    body_force: tuple = (0.0, 0.0)    # "free" flows: explicit force density
    init_seed: int | None = None      # smooth random initial fields when set
    init_amp: float = 0.0

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


# ---- the five benchmark configurations -------------------------------------

def channel_64() -> Case:
    """Plain channel, FP64: 64x64, periodic x, walls in y, tanh beta = 1.5,
    Re = 10, tau = 0.8, 2000 steps (Poiseuille start-up)."""
    return Case("channel_64", 64, 64, "periodic", "wall", ("uniform", 0.0), ("tanh", 1.5),
                flow="channel", Re=10.0, tau=0.8, storage="f64", steps=2000)


def cavity_1024() -> Case:
    """Lid-driven cavity, FP32: 1024^2, tanh beta = 2 toward all walls,
    Re = 1000, 50k steps (parity at 1000).  The lid speed is Mach 0.1 of
    the GOC sound speed lowered so that the shear relaxation time stays at
    most 1 (Re kept): here U_lid = 3.5e-3, Mach 0.041.  The literal lid
    speed 0.05 is Mach 0.59 and the FP64 oracle diverges within 150 steps;
    Mach 0.1 gives tau = 1.7, where the oracle diverges after 10^4 steps."""
    return Case("cavity_1024", 1024, 1024, "wall", "wall", ("tanh", 2.0), ("tanh", 2.0),
                flow="cavity", Re=1000.0, u_lid=0.0, Ma=0.1, tau_max=1.0, storage="f32", steps=50000)


def hartmann_4096() -> Case:
    """Coupled MHD Hartmann channel, FP32: 4096x1024, tanh beta = 3 in y,
    Ha = 100, Re = 100, Pm = 1, applied B2.  Centre-line speed Mach 0.1
    lowered so that the shear relaxation time stays at most 1 (Re kept):
    on tanh beta = 3 grids the scheme amplifies x-varying perturbations for
    tau above about 1.2 (an x-homogeneous start never excites them, a
    perturbed one does), and Mach 0.1 would give tau = 30."""
    return Case("hartmann_4096x1024", 4096, 1024, "periodic", "wall", ("uniform", 0.0),
                ("tanh", 3.0), flow="hartmann", Re=100.0, Ha=100.0, Pm=1.0, Ma=0.1,
                tau_max=1.0, mhd=True, storage="f32", steps=1000)


def hartmann_4096_precision(storage: str) -> Case:
    return hartmann_4096().replace(name=f"hartmann_4096x1024_{storage}", storage=storage)


def batch_256(seed: int = 15362, n: int = 256):
    """256 independent stretched channel / Hartmann runs: grids 128x64 .. 1024x512,
    beta in [1, 3], Re in [10, 500], Ha in [0, 200], FP32."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(128, 1025, n)
    ny = rng.integers(64, 513, n)
    beta = rng.uniform(1.0, 3.0, n)
    Re = rng.uniform(10.0, 500.0, n)
    Ha = rng.uniform(0.0, 200.0, n)
    runs = []
    for k in range(n):
        runs.append(Case(f"batch_{k}", int(nx[k]), int(ny[k]), "periodic", "wall",
                         ("uniform", 0.0), ("tanh", float(beta[k])), flow="hartmann",
                         Re=float(Re[k]), Ha=float(Ha[k]), Pm=1.0, Ma=0.1, tau_max=1.0,
                         mhd=True, storage="f32", steps=1000))
    return runs


def taylor_couette(n1: int = 256, n2: int = 6, R1: float = 32.0, n_theta: int = 60,
                   U_in: float = 0.01, U_out: float = 0.015, tau: float = 1.0,
                   storage: str = "f64", collision: str = "central") -> Case:
    """Circular Couette flow in one annular sector on the conformal grid of
    the curvilinear section: n1 radial nodes between the inner radius R1
    and R2 = R1 + n1 (walls moving at the linear speeds U_in, U_out),
    n2 periodic azimuthal nodes over 2 pi / n_theta, shear relaxation time
    tau (the paper's sector: 256 x 6, R1 = 32, n_theta = 60, U0 = 0.01)."""
    return Case(f"tc_{n1}x{n2}", n1, n2, "wall", "periodic", flow="free", tau=tau,
                body_force=(0.0, 0.0), grid2d=("annulus", R1, R1 + n1, n_theta),
                v_wall=(U_in, U_out), storage=storage, collision=collision, steps=0)


def wavy_metric(nx: int, ny: int, eps: float):
    """Node metric of the conformal map Z = W + eps (2L/pi) sin(pi W / (2L)),
    L = max(nx, ny), W = xi1 + i xi2 at the nodes xi = (i + 1/2, j + 1/2):
    h1 = h2 = |1 + eps cos(pi W / (2L))|, a non-separable orthogonal grid
    (|h - 1| <= 2.6 eps over the domain).  Returns [ny, nx] arrays (h1, h2)."""
    L = float(max(nx, ny))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    W = x[None, :] + 1j * y[:, None]
    h = np.abs(1.0 + eps * np.cos(0.5 * np.pi * W / L))
    return np.ascontiguousarray(h), np.ascontiguousarray(h.copy())


# ---- seeded smooth random fields ---------------------------------------------

def smooth_fields(nx: int, ny: int, seed: int, amp: float, rho0: float = 1.0, modes: int = 3):
    """Smooth periodic random fields (rho, U1, U2) of shape [ny, nx]:
    rho = rho0 (1 + amp r), U = amp (u, v) with r, u, v sums of a few random
    low Fourier modes of unit amplitude."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)

    def field_():
        out = np.zeros((ny, nx))
        for _ in range(modes):
            kx, ky = rng.integers(1, 4, 2)
            ph = rng.uniform(0, 2 * np.pi, 2)
            out += np.sin(2 * np.pi * kx * X + ph[0]) * np.cos(2 * np.pi * ky * Y + ph[1])
        return out / modes

    r, u, v = field_(), field_(), field_()
    return rho0 * (1.0 + amp * r), amp * u, amp * v


def hartmann_start(case: Case, nu: float, F1: float, eta: float = 0.0, B0: float = 0.0):
    """Developed Hartmann flow as an initial state (rho, U1, U2, B1, B2) of
    shape [ny, nx], from the closed forms between the plates (Sec. 7.4):
    rho = rho0, u(y*) = U_r (cosh Ha - cosh(Ha y*)) / (Ha sinh Ha),
    B1(y*) = B_r (sinh(Ha y*) / (Ha tanh(Ha) cosh(Ha)) - y* / Ha), B2 = B0,
    with U_r = H^2 F1 / (rho0 nu), B_r = H^2 F1 mu_m sqrt(sigma / (rho0 nu)),
    sigma = 1 / (eta mu_m), half-height H = ny / 2 in lattice units of the
    physical domain [0, ny], and y* in [-1, 1] the node's wall-normal
    position on the tanh-clustered grid of Sec. 6.1 (node centres at
    xi = j + 1/2): y* = tanh(beta (2 xi / ny - 1)) / tanh(beta).
    nu, F1, eta, B0 are the run's lattice viscosity, body force, magnetic
    diffusivity and applied field (B1 = 0 when eta or Ha is zero)."""
    kind, beta = case.stretch_y
    if kind not in ("tanh", "uniform"):
        raise ValueError("hartmann_start needs a tanh or uniform wall-normal grid")
    xi = (np.arange(case.ny) + 0.5) / case.ny
    ys = np.tanh(beta * (2 * xi - 1)) / np.tanh(beta) if kind == "tanh" and beta > 0 else 2 * xi - 1
    H = 0.5 * case.ny
    Ur = H * H * F1 / (case.rho0 * nu)
    Ha = case.Ha
    if Ha > 0:
        u = Ur * (np.cosh(Ha) - np.cosh(Ha * ys)) / (Ha * np.sinh(Ha))
    else:
        u = 0.5 * Ur * (1 - ys * ys)
    b = np.zeros_like(ys)
    if Ha > 0 and eta > 0:
        sigma = 1.0 / (eta * case.mu_m)
        Br = H * H * F1 * case.mu_m * np.sqrt(sigma / (case.rho0 * nu))
        b = Br * (np.sinh(Ha * ys) / (Ha * np.tanh(Ha) * np.cosh(Ha)) - ys / Ha)
    rep = lambda v: np.repeat(v[:, None], case.nx, axis=1)
    U1 = rep(u)
    return (np.full((case.ny, case.nx), case.rho0), U1, np.zeros_like(U1), rep(b),
            np.full((case.ny, case.nx), B0))


def sample_nodes(nx: int, ny: int, count: int, seed: int):
    """Seeded node sample that always includes the corners and wall rows."""
    rng = np.random.default_rng(seed)
    ix = list(rng.integers(0, nx, count))
    iy = list(rng.integers(0, ny, count))
    for (i, j) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0),
                   (nx // 2, ny - 1), (0, ny // 2), (nx - 1, ny // 2), (1, 1), (nx - 2, ny - 2)]:
        ix.append(i)
        iy.append(j)
    return np.asarray(ix, dtype=np.int32), np.asarray(iy, dtype=np.int32)
