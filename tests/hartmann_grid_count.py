"""Grid points needed to resolve the Hartmann layers: the GOC grid (Roberts
clustering gamma = 1.05 toward both plates) against the uniform grid (the
same kernel at h = 1, i.e. the standard LBM), the experiment behind the
paper's grid-savings table for the MHD channel.

Test infrastructure: tests/test_gpu_hartmann_grid_count.py brackets the
saving factor with it, and it runs on its own for sweeps (minutes of GPU
time):

    python tests/hartmann_grid_count.py HA NY1,NY2,... goc|std [Re] [max_steps]

Each run is a 3 x Ny periodic strip with the coupled D2Q5 induction scheme,
FP64, Pm = 1, Re = U_c H / nu (default 100), U_c at Mach 0.1 lowered by the
relaxation-time cap tau <= 1, started from the closed-form Hartmann profiles
(u_x, B_x) at the node positions and run until u changes by less than 1e-12
(relative) over 20000 steps or max_steps (default 2M).  It prints the
relative L2 errors of u_x and B_x against the closed forms (Sec. 7.4) and
the last 20000-step change of u_x relative to its maximum.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import params  # noqa: E402  (closed forms and grid positions)
from paper_2607_15362_amd import binding as B  # noqa: E402
from paper_2607_15362_amd import workloads as W  # noqa: E402


def run_one(Ha: float, Ny: int, scheme: str, Re: float = 100.0, max_steps: int = 2000000,
            w3: float = 1.0, w4: float = 1.0, tau_max: float = 1.0):
    """w3: the third-order relaxation rates omega6 = omega7, w4: the
    fourth-order rate omega8 (free parameters of the model, 1 by default);
    tau_max: the cap on the shear relaxation time."""
    st = ("roberts", 1.05) if scheme == "goc" else ("uniform", 0.0)
    case = W.Case("hgc", 3, Ny, "periodic", "wall", ("uniform", 0.0), st, flow="hartmann", Re=Re, Ha=Ha,
                  Pm=1.0, Ma=0.1, tau_max=tau_max, mhd=True, storage="f64")
    gs, ms, ps = B.derive(case)
    ps.omega[6] = ps.omega[7] = w3
    ps.omega[8] = w4
    g = B.Run(case, structs=(gs, ms, ps))
    d = g.derived()
    H = Ny / 2.0
    nu, F1, eta, B0 = d["nu"], d["F1"], d["eta"], d["B0"]
    sigma = 1.0 / eta
    Ur = H * H * F1 / nu
    Br = H * H * F1 * math.sqrt(sigma / nu)
    xi = np.arange(Ny) + 0.5
    y = params.roberts_y(Ny, 1.05, xi) if scheme == "goc" else xi
    ua, ba = params.hartmann_profile(2.0 * y / Ny - 1.0, Ha, Ur, Br)
    rep = lambda v: np.ascontiguousarray(np.repeat(v[:, None], 3, axis=1))
    g.init(np.ones((Ny, 3)), rep(ua), np.zeros((Ny, 3)), rep(ba), np.full((Ny, 3), B0))
    prev, done, change = None, 0, float("inf")
    while done < max_steps:
        g.step(20000)
        done += 20000
        u = g.fields()["U1"][:, 1]
        if prev is not None:
            change = float(np.max(np.abs(u - prev)) / np.max(np.abs(u)))
            if change < 1e-12:
                break
        prev = u
    fl = g.fields()
    out = dict(Ha=Ha, scheme=scheme, Ny=Ny, steps=done, change=change, tau=nu / d["cs2"] + 0.5, w3=w3, w4=w4,
               err_u=float(np.linalg.norm(fl["U1"][:, 1] - ua) / np.linalg.norm(ua)),
               err_b=float(np.linalg.norm(fl["B1"][:, 1] - ba) / np.linalg.norm(ba)))
    g.close()
    return out


def main():
    Ha = float(sys.argv[1])
    nys = [int(v) for v in sys.argv[2].split(",")]
    scheme = sys.argv[3]
    Re = float(sys.argv[4]) if len(sys.argv) > 4 else 100.0
    steps = int(sys.argv[5]) if len(sys.argv) > 5 else 2000000
    for ny in nys:
        t0 = time.time()
        r = run_one(Ha, ny, scheme, Re, steps)
        r["seconds"] = round(time.time() - t0, 1)
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
