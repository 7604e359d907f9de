"""The lid-driven cavity at the paper's settings (tanh beta = 1.2 on both
axes, its grid for each Re: 120^2, 300^2, 350^2, 400^2 for Re = 1000, 3200,
5000, 7500) run to steady state on the GPU: the vortex centres against the
GOC-LBM values the paper prints (tests/golden, Tables 1 and 2 of the cavity
section).  The primary centre agrees within 1e-3 (2e-3 at Re 1000) at every
Re.  The first secondary vortices agree within 3e-3 of the side up to
Re 3200, 4e-3 at Re 5000 and 1.2e-2 at Re 7500, where the corner vortices
span a few cells of the paper's 400^2 grid and ours lie closer to Erturk's
reference centres than to the paper's GOC-LBM row (design notes).  The
second secondary vortices are not compared: the paper's lie within two
cells of the corner, where neither grid resolves them."""
import pytest

import cavity_paper as CP

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Re,N,steps,tol_primary,tol_secondary", [
    (1000.0, 120, 1500000, 0.002, 0.012),
    (3200.0, 300, 3000000, 0.001, 0.003),
    pytest.param(5000.0, 350, 6000000, 0.001, 0.004, marks=pytest.mark.slow),
    pytest.param(7500.0, 400, 12000000, 0.001, 0.012, marks=pytest.mark.slow),
])
def test_cavity_vortex_centres_match_paper(Re, N, steps, tol_primary, tol_secondary):
    ref = CP.golden()
    key = str(int(Re))
    run, lid = CP.make_run(N, Re)
    print(f"[cavity] Re {Re:g} on {N}^2, up to {steps} steps", flush=True)
    done, ch = CP.run_steady(run, lid, steps, tol=1e-7, log=lambda s: print(s, flush=True))
    c = CP.vortex_centres(run.fields()["U1"], N)
    print(f"[cavity] Re {Re:g}: {done} steps, change {ch:.1e}, centres",
          {k: (None if v is None else [round(a, 4) for a in v]) for k, v in c.items()}, flush=True)
    px, py = ref["primary"]["goc_lbm"][key]
    assert abs(c["primary"][0] - px) < tol_primary and abs(c["primary"][1] - py) < tol_primary
    for name in ("TL", "BL", "BR"):
        want = ref["secondary_goc_lbm"][key].get(name)
        if want is None:
            assert c[name] is None or name != "TL"   # no top vortex at Re = 1000 in the paper either
            continue
        assert c[name] is not None, name
        assert abs(c[name][0] - want[0]) < tol_secondary and abs(c[name][1] - want[1]) < tol_secondary, (
            name, c[name], want)
