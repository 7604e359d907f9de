"""The lid-driven cavity at the paper's settings, run on the GPU to steady
state, and the vortex centres of its stream function.

Test infrastructure (used by tests/test_gpu_cavity_paper.py and runnable on
its own for the long cases):

    python tests/cavity_paper.py N Re STEPS

Settings: tanh clustering beta = 1.2 toward all four walls (Sec. 6.1), the
lid on the xi2 = N wall at Mach 0.1 of the GOC sound speed, the
central-moment model with the bulk viscosity equal to the shear viscosity
(omega3 = omega4; with the default omega3 = 1 the corrections destabilise
the MRT models at Re >= 1000 on such grids), FP64.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import params  # noqa: E402  (node coordinates of the tanh map)
from paper_2607_15362_amd import binding as B  # noqa: E402
from paper_2607_15362_amd import workloads as W  # noqa: E402

BETA = 1.2


def golden():
    with open(os.path.join(HERE, "golden", "cavity_vortex_centres.json")) as fh:
        return json.load(fh)


def make_run(N: int, Re: float, Ma: float = 0.1, storage: str = "f64"):
    case = W.Case("cav_paper", N, N, "wall", "wall", ("tanh", BETA), ("tanh", BETA), flow="cavity", Re=Re,
                  Ma=Ma, u_lid=0.0, storage=storage)
    g, m, p = B.derive(case)
    p.omega[3] = p.omega[4]
    return B.Run(case, structs=(g, m, p)), float(g.u_wall_hi)


def run_steady(run, lid: float, max_steps: int, chunk: int = 50000, tol: float = 1e-9, log=None):
    """Step until the largest change of U1 over a chunk is below tol * lid
    (or max_steps); returns (steps, last change / lid)."""
    prev, done, ch = None, 0, float("inf")
    while done < max_steps:
        run.step(chunk)
        done += chunk
        u = run.fields()["U1"]
        if not np.all(np.isfinite(u)):
            raise FloatingPointError(f"non-finite velocity after {done} steps")
        if prev is not None:
            ch = float(np.max(np.abs(u - prev)) / lid)
            if log and done % (10 * chunk) == 0:
                log(f"[cavity] {done} steps, change {ch:.2e}")
            if ch < tol:
                break
        prev = u.copy()
    return done, ch


def stream_function(U1, N: int):
    """psi(x_i, y_j) = integral of u from the bottom wall (u = 0 there) to y_j
    on the physical node positions, trapezoidal; x, y in units of the side."""
    x = params.tanh_two_wall_y(N, BETA, np.arange(N) + 0.5) / N
    yy = np.concatenate([[0.0], x])
    uu = np.concatenate([np.zeros((1, N)), U1], axis=0)
    psi = np.cumsum(0.5 * (uu[1:] + uu[:-1]) * np.diff(yy)[:, None], axis=0)
    return x, psi


def _refine(x, psi, jj, ii):
    """Extremum of the quadratic fitted to the 3 x 3 nodes around (jj, ii)."""
    X, Y, Z = [], [], []
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            X.append(x[ii + di])
            Y.append(x[jj + dj])
            Z.append(psi[jj + dj, ii + di])
    X, Y, Z = map(np.asarray, (X, Y, Z))
    A = np.stack([np.ones(9), X, Y, X * X, X * Y, Y * Y], axis=1)
    c = np.linalg.lstsq(A, Z, rcond=None)[0]
    M = np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]])
    return [float(v) for v in np.linalg.solve(M, -np.array([c[1], c[2]]))]


def vortex_centres(U1, N: int):
    """Primary vortex (extremum of psi, negative for a lid moving in +x) and
    the corner vortices: the first secondary ones (positive extrema) top-left,
    bottom-left and bottom-right, and the second secondary ones (negative
    extrema) in the two bottom corners.  None where a region has no interior
    extremum of the expected sign."""
    x, psi = stream_function(U1, N)
    out = {}
    core = np.full_like(psi, np.inf)
    core[2:-2, 2:-2] = psi[2:-2, 2:-2]
    jj, ii = np.unravel_index(np.argmin(core), psi.shape)
    out["primary"] = _refine(x, psi, jj, ii)
    regions = {"TL": (x < 0.3, x > 0.7, 1), "BL": (x < 0.35, x < 0.35, 1), "BR": (x > 0.6, x < 0.4, 1),
               "BL2": (x < 0.05, x < 0.05, -1), "BR2": (x > 0.93, x < 0.07, -1)}
    for name, (mx, my, sign) in regions.items():
        sub = np.where(my[:, None] & mx[None, :], sign * psi, -np.inf)
        jj, ii = np.unravel_index(np.argmax(sub), sub.shape)
        if not sub[jj, ii] > 0 or jj in (0, N - 1) or ii in (0, N - 1):
            out[name] = None
            continue
        out[name] = _refine(x, psi, jj, ii)
    return out


def main():
    N, Re, steps = int(sys.argv[1]), float(sys.argv[2]), int(sys.argv[3])
    t0 = time.time()
    run, lid = make_run(N, Re)
    done, ch = run_steady(run, lid, steps, log=lambda s: print(s, flush=True))
    c = vortex_centres(run.fields()["U1"], N)
    ref = golden()
    key = str(int(Re))
    print(json.dumps({"N": N, "Re": Re, "steps": done, "change": ch, "seconds": round(time.time() - t0, 1),
                      "centres": {k: (None if v is None else [round(a, 4) for a in v]) for k, v in c.items()},
                      "paper_goc_lbm_primary": ref["primary"]["goc_lbm"].get(key),
                      "paper_goc_lbm_secondary": ref["secondary_goc_lbm"].get(key)}), flush=True)


if __name__ == "__main__":
    main()
