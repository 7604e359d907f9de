"""FP64 CPU oracle of the GOC-LBM hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does, and the HIP library shares no code with it.

The arithmetic lives in goc_oracle.c (plain loops, FP64, optionally OpenMP
over rows); this module compiles it with gcc, mirrors its configuration
struct with ctypes and derives the lattice parameters from a workload
description with the relations in params.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import params

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "goc_oracle.c")
LIB = os.path.join(HERE, "libgoc_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle shared library (gcc -O3, FP64, no fast-math: the
    optimiser keeps the source's order of floating-point operations)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        P = C.POINTER(C.c_double)
        cfgp = C.POINTER(OracleCfg)
        _lib.oracle_step.argtypes = [cfgp, P, P, P, C.c_int]
        _lib.oracle_step_sample.argtypes = [cfgp, P, P, P, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int32), C.c_int, P, P, P]
        _lib.oracle_fields.argtypes = [cfgp, P, P, P, P, P, P, P, P]
        _lib.oracle_init.argtypes = [cfgp, P, P, P, P, P, P, P, P]
        _lib.oracle_collide_node.argtypes = [cfgp, P, P]
        _lib.oracle_moment_map.argtypes = [C.c_int, P, C.c_double, C.c_double, P]
        _lib.oracle_central_eq.argtypes = [cfgp] + [C.c_double] * 7 + [P, P]
        _lib.oracle_mie_node.argtypes = [cfgp, P, P, P, P]
        _lib.oracle_threads.restype = C.c_int
        _lib.oracle_set_threads.argtypes = [C.c_int]
        _lib.oracle_set_threads.restype = C.c_int
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """Use n OpenMP threads in the oracle's loops; returns the number in use."""
    return int(lib().oracle_set_threads(int(n)))


class OracleCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc_x", C.c_int32), ("bc_y", C.c_int32),
        ("gi_terms", C.c_int32), ("q3_sign", C.c_int32), ("lid_corners", C.c_int32),
        ("rho_terms", C.c_int32), ("mhd", C.c_int32),
        ("u_wall_lo", C.c_double), ("u_wall_hi", C.c_double), ("cs2", C.c_double),
        ("omega", C.c_double * 9), ("nu", C.c_double), ("zeta", C.c_double),
        ("rho0", C.c_double), ("Fext", C.c_double * 2),
        ("csm2", C.c_double), ("tau_m", C.c_double), ("eta", C.c_double),
        ("mu_m", C.c_double), ("B0", C.c_double),
        ("h1", C.POINTER(C.c_double)), ("h2", C.POINTER(C.c_double)),
        ("th11", C.POINTER(C.c_double)), ("th12", C.POINTER(C.c_double)),
        ("th21", C.POINTER(C.c_double)), ("th22", C.POINTER(C.c_double)),
        ("h2_face_lo", C.POINTER(C.c_double)), ("h2_face_hi", C.POINTER(C.c_double)),
        ("h1_face_ylo", C.POINTER(C.c_double)), ("h1_face_yhi", C.POINTER(C.c_double)),
        ("h1_face_lo", C.POINTER(C.c_double)), ("h1_face_hi", C.POINTER(C.c_double)),
        ("h2_face_xlo", C.POINTER(C.c_double)), ("h2_face_xhi", C.POINTER(C.c_double)),
        ("collision", C.c_int32),
        ("v_wall_lo", C.c_double), ("v_wall_hi", C.c_double),
    ]


COLLISIONS = {"central": 0, "raw": 1, "srt": 2}


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def metric_1d(n: int, stretch):
    """(h, dh, theta, face_lo, face_hi) for a stretching descriptor."""
    kind, p = stretch
    if kind == "uniform" or (kind == "tanh" and p == 0.0):
        return np.ones(n), np.zeros(n), np.zeros(n), 1.0, 1.0
    if kind == "tanh":
        return params.tanh_two_wall(n, float(p))
    if kind == "roberts":
        return params.roberts(n, float(p))
    raise ValueError(kind)


@dataclass
class Lattice:
    """Lattice parameters of one run (all FP64)."""
    cs2: float
    omega: np.ndarray
    nu: float
    zeta: float
    rho0: float
    Fext: tuple
    u_wall_lo: float
    u_wall_hi: float
    mhd: bool
    csm2: float = 0.0
    tau_m: float = 1.0
    eta: float = 0.0
    mu_m: float = 1.0
    B0: float = 0.0
    extra: dict = None


def derive(case, h1, h2) -> Lattice:
    """Lattice parameters of a workload (Sec. 3.2.1, Sec. 4, App. G, Sec. 7).

    reading: omega_0,1,2,6,7,8 = 1 and omega_3 = 1 (bulk viscosity
    zeta = c_s^2/2); omega_4 = omega_5 from the shear viscosity.  The SRT
    model relaxes every moment at omega = 1/tau, so zeta = nu.
    """
    cs2 = params.sound_speed_sq(h1, h2)
    rho0 = case.rho0
    extra = {}
    u_lo = u_hi = 0.0
    Fext = (0.0, 0.0)
    B0 = 0.0
    eta = 0.0
    tau_m = 1.0
    if case.flow == "channel":
        nu = params.viscosity_from_tau(cs2, case.tau)
        U, F = params.poiseuille(float(case.ny), nu, case.Re, rho0)
        Fext = (F, 0.0)
        extra.update(U=U)
    elif case.flow == "cavity":
        u_hi = case.u_lid if case.u_lid > 0 else case.Ma * np.sqrt(cs2)
        nu = u_hi * case.nx / case.Re
        tmax = getattr(case, "tau_max", 0.0)
        if case.u_lid <= 0 and tmax > 0 and params.viscosity_from_tau(cs2, tmax) < nu:
            # reading: cap the shear relaxation time (Re = U_lid L / nu kept)
            nu = params.viscosity_from_tau(cs2, tmax)
            u_hi = nu * case.Re / case.nx
    elif case.flow == "hartmann":
        H = case.ny / 2.0
        Uc = case.Ma * np.sqrt(cs2)
        tmax = getattr(case, "tau_max", 0.0)
        if tmax > 0 and params.viscosity_from_tau(cs2, tmax) < Uc * H / case.Re:
            # reading: cap the shear relaxation time (Re = Uc H / nu kept)
            Uc = params.viscosity_from_tau(cs2, tmax) * case.Re / H
        hp = params.hartmann(H, case.Ha, case.Re, case.Pm, Uc, rho0, case.mu_m)
        nu, eta, B0 = hp["nu"], hp["eta"], hp["B0"]
        Fext = (hp["F"], 0.0)
        extra.update(hp, Uc=Uc)
    elif case.flow == "free":
        nu = params.viscosity_from_tau(cs2, case.tau)
        Fext = tuple(case.body_force)
    else:
        raise ValueError(case.flow)
    w45 = params.omega_from_viscosity(cs2, nu)
    omega = np.ones(9)
    omega[4] = omega[5] = w45
    if getattr(case, "collision", "central") == "srt":
        omega[:] = w45
    zeta = cs2 * (1.0 / omega[3] - 0.5)
    csm2 = cs2
    if case.mhd:
        tau_m = eta / csm2 + 0.5
    return Lattice(cs2, omega, nu, zeta, rho0, Fext, u_lo, u_hi, case.mhd, csm2, tau_m, eta,
                   case.mu_m, B0, extra)


class Model:
    """One oracle run: metric, lattice parameters and the FP64 state.

    The metric is the straight one of case.stretch_x / stretch_y, or a
    general 2-D one: case.grid2d = ("annulus", a, Ro, n_theta) (the conformal
    annular sector), or node arrays metric2d = (h1, h2) ([ny, nx]) whose
    curvature elements come from second-order differences (reading: face
    values are those of the adjacent nodes)."""

    def __init__(self, case, lattice: Lattice | None = None, metric2d=None):
        self.case = case
        nx, ny = case.nx, case.ny
        self.nx, self.ny = nx, ny
        g2 = getattr(case, "grid2d", None)
        if g2 is None and metric2d is None:
            h1, dh1, th1, h1lo, h1hi = metric_1d(nx, case.stretch_x)
            h2, dh2, th2, h2lo, h2hi = metric_1d(ny, case.stretch_y)
            self.h1_1d, self.h2_1d = h1, h2
            self.dh1_1d, self.dh2_1d = dh1, dh2
            # 2-D metric arrays (straight grid: theta12 = theta21 = 0)
            self.h1 = np.ascontiguousarray(np.broadcast_to(h1[None, :], (ny, nx)))
            self.h2 = np.ascontiguousarray(np.broadcast_to(h2[:, None], (ny, nx)))
            self.th11 = np.ascontiguousarray(np.broadcast_to(th1[None, :], (ny, nx)))
            self.th22 = np.ascontiguousarray(np.broadcast_to(th2[:, None], (ny, nx)))
            self.th12 = np.zeros((ny, nx))
            self.th21 = np.zeros((ny, nx))
            self.h2_face_lo = np.full(nx, h2lo)
            self.h2_face_hi = np.full(nx, h2hi)
            self.h1_face_ylo = h1.copy()
            self.h1_face_yhi = h1.copy()
            self.h1_face_lo = np.full(ny, h1lo)
            self.h1_face_hi = np.full(ny, h1hi)
            self.h2_face_xlo = h2.copy()
            self.h2_face_xhi = h2.copy()
        else:
            if metric2d is not None:
                h1a, h2a = (np.ascontiguousarray(x, dtype=np.float64) for x in metric2d)
                m = dict(h1=h1a, h2=h2a, **params.metric_from_arrays(h1a, h2a, case.bc_x == "periodic",
                                                                      case.bc_y == "periodic"))
                m.update(h1_face_lo=h1a[:, 0].copy(), h1_face_hi=h1a[:, -1].copy(),
                         h2_face_xlo=h2a[:, 0].copy(), h2_face_xhi=h2a[:, -1].copy())
            elif g2[0] == "annulus":
                m = params.annulus(nx, ny, float(g2[1]), float(g2[2]), float(g2[3]))
                self.radius = m["r"]
            else:
                raise ValueError(g2)
            for k in ("h1", "h2", "th11", "th12", "th21", "th22"):
                setattr(self, k, np.ascontiguousarray(m[k], dtype=np.float64))
            self.h2_face_lo = self.h2[0].copy()
            self.h2_face_hi = self.h2[-1].copy()
            self.h1_face_ylo = self.h1[0].copy()
            self.h1_face_yhi = self.h1[-1].copy()
            for k in ("h1_face_lo", "h1_face_hi", "h2_face_xlo", "h2_face_xhi"):
                setattr(self, k, np.ascontiguousarray(m[k], dtype=np.float64))
            h1, h2 = self.h1, self.h2
        self.lat = lattice if lattice is not None else derive(case, h1, h2)
        self.cfg = self._make_cfg()
        self.N = nx * ny
        self.f = np.zeros((9, ny, nx))
        self.F = np.zeros((2, ny, nx))
        self.g = np.zeros((10, ny, nx)) if self.lat.mhd else np.zeros((10, 1, 1))

    def _make_cfg(self):
        c = OracleCfg()
        case, lat = self.case, self.lat
        c.nx, c.ny = case.nx, case.ny
        c.bc_x = 0 if case.bc_x == "periodic" else 1
        c.bc_y = 0 if case.bc_y == "periodic" else 1
        c.gi_terms, c.q3_sign, c.lid_corners = case.gi_terms, case.q3_sign, case.lid_corners
        c.rho_terms = getattr(case, "rho_terms", 0)
        c.collision = COLLISIONS[getattr(case, "collision", "central")]
        c.mhd = 1 if lat.mhd else 0
        c.u_wall_lo, c.u_wall_hi = lat.u_wall_lo, lat.u_wall_hi
        c.v_wall_lo, c.v_wall_hi = (float(v) for v in getattr(case, "v_wall", (0.0, 0.0)))
        c.cs2 = lat.cs2
        for k in range(9):
            c.omega[k] = float(lat.omega[k])
        c.nu, c.zeta, c.rho0 = lat.nu, lat.zeta, lat.rho0
        c.Fext[0], c.Fext[1] = lat.Fext
        c.csm2, c.tau_m, c.eta, c.mu_m, c.B0 = lat.csm2, lat.tau_m, lat.eta, lat.mu_m, lat.B0
        for name in ["h1", "h2", "th11", "th12", "th21", "th22", "h2_face_lo", "h2_face_hi",
                     "h1_face_ylo", "h1_face_yhi", "h1_face_lo", "h1_face_hi", "h2_face_xlo",
                     "h2_face_xhi"]:
            setattr(c, name, _ptr(getattr(self, name)))
        return c

    # -- state --------------------------------------------------------------
    def init(self, rho=None, U1=None, U2=None, B1=None, B2=None):
        """Initial state from node fields [ny][nx] (None: rho0, U = 0 and the
        applied field B = (0, B0))."""
        ny, nx = self.ny, self.nx
        rho = np.full((ny, nx), self.lat.rho0) if rho is None else np.ascontiguousarray(rho, float)
        U1 = np.zeros((ny, nx)) if U1 is None else np.ascontiguousarray(U1, float)
        U2 = np.zeros((ny, nx)) if U2 is None else np.ascontiguousarray(U2, float)
        if (B1 is None) != (B2 is None):
            raise ValueError("give both B1 and B2 or neither")
        Bp = [None, None] if B1 is None else [np.ascontiguousarray(B1, float), np.ascontiguousarray(B2, float)]
        self.f = np.zeros((9, ny, nx))
        self.F = np.zeros((2, ny, nx))
        self.g = np.zeros((10, ny, nx)) if self.lat.mhd else np.zeros((10, 1, 1))
        lib().oracle_init(C.byref(self.cfg), _ptr(rho), _ptr(U1), _ptr(U2),
                          None if Bp[0] is None else _ptr(Bp[0]), None if Bp[1] is None else _ptr(Bp[1]),
                          _ptr(self.f), _ptr(self.F), _ptr(self.g))
        return self

    def set_state(self, f, F, g=None):
        self.f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx).copy()
        self.F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, self.ny, self.nx).copy()
        if self.lat.mhd:
            self.g = np.ascontiguousarray(g, dtype=np.float64).reshape(10, self.ny, self.nx).copy()

    def step(self, n: int = 1):
        rc = lib().oracle_step(C.byref(self.cfg), _ptr(self.f), _ptr(self.F), _ptr(self.g), int(n))
        if rc != 0:
            raise MemoryError("oracle_step")
        return self

    def fields(self):
        ny, nx = self.ny, self.nx
        out = [np.zeros((ny, nx)) for _ in range(5)]
        lib().oracle_fields(C.byref(self.cfg), _ptr(self.f), _ptr(self.F), _ptr(self.g),
                            *[_ptr(o) for o in out])
        rho, U1, U2, B1, B2 = out
        d = dict(rho=rho, U1=U1, U2=U2)
        if self.lat.mhd:
            d.update(B1=B1, B2=B2)
        return d

    def step_sample(self, ix, iy):
        """One step evaluated at sampled nodes only: (f[9,ns], F[2,ns], g[10,ns])."""
        ix = np.ascontiguousarray(ix, dtype=np.int32)
        iy = np.ascontiguousarray(iy, dtype=np.int32)
        ns = len(ix)
        fo = np.zeros((9, ns))
        Fo = np.zeros((2, ns))
        go = np.zeros((10, ns))
        rc = lib().oracle_step_sample(C.byref(self.cfg), _ptr(self.f), _ptr(self.F), _ptr(self.g),
                                      ix.ctypes.data_as(C.POINTER(C.c_int32)),
                                      iy.ctypes.data_as(C.POINTER(C.c_int32)), ns, _ptr(fo),
                                      _ptr(Fo), _ptr(go))
        if rc != 0:
            raise MemoryError("oracle_step_sample")
        return fo, Fo, go

    def mass(self):
        return float(self.f.sum())


# ---- single-node helpers for the unit pins ---------------------------------

def collide_node(cfg: OracleCfg, f, metric, flow, force):
    """Oracle collision at one node.  metric = (h1,h2,th11,th12,th21,th22),
    flow = (rho,U1,U2,d1U1,d2U2,d1rho,d2rho), force = external (F1,F2).
    Returns dict(ft, F, tau12, n3, n4, Ft)."""
    vin = np.zeros(24)
    vin[0:9] = f
    vin[9:15] = metric
    vin[15:22] = flow
    vin[22:24] = force
    out = np.zeros(16)
    lib().oracle_collide_node(C.byref(cfg), _ptr(vin), _ptr(out))
    return dict(ft=out[0:9].copy(), F=out[9:11].copy(), tau12=out[11], n3=out[12], n4=out[13],
                Ft=out[14:16].copy())


def moment_map(which: int, v, U1=0.0, U2=0.0):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(9)
    lib().oracle_moment_map(int(which), _ptr(v), float(U1), float(U2), _ptr(out))
    return out


def central_eq(cfg, h1, h2, rho, U1, U2, F1=0.0, F2=0.0):
    eq = np.zeros(9)
    src = np.zeros(9)
    lib().oracle_central_eq(C.byref(cfg), h1, h2, rho, U1, U2, F1, F2, _ptr(eq), _ptr(src))
    return eq, src


def mie_node(cfg, gb, U, metric):
    gb = np.ascontiguousarray(gb, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    met = np.ascontiguousarray(metric, dtype=np.float64)
    out = np.zeros(19)
    lib().oracle_mie_node(C.byref(cfg), _ptr(gb), _ptr(U), _ptr(met), _ptr(out))
    return dict(B=out[0:2].copy(), dB=out[2:6].copy(), J3=out[6], FL=out[7:9].copy(),
                gt=out[9:19].copy())


def bare_cfg(cs2=1.0 / 3.0, omega=None, nu=0.1, zeta=None, gi_terms=1, q3_sign=0, csm2=None,
             tau_m=1.0, eta=None, mu_m=1.0, B0=0.0, rho_terms=0, collision="central"):
    """A configuration for single-node calls (no grid pointers)."""
    c = OracleCfg()
    c.collision = COLLISIONS[collision]
    c.cs2 = cs2
    om = np.ones(9) if omega is None else np.asarray(omega, float)
    for k in range(9):
        c.omega[k] = float(om[k])
    c.nu = nu
    c.zeta = cs2 * (1.0 / om[3] - 0.5) if zeta is None else zeta
    c.gi_terms, c.q3_sign, c.rho_terms = gi_terms, q3_sign, rho_terms
    c.csm2 = cs2 if csm2 is None else csm2
    c.tau_m = tau_m
    c.eta = c.csm2 * (tau_m - 0.5) if eta is None else eta
    c.mu_m, c.B0 = mu_m, B0
    c.rho0 = 1.0
    return c
