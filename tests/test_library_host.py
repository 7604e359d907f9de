"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point its header declares, and its host-only parameter
derivation agrees with the oracle's independent one."""
import math
import os
import re

import numpy as np
import pytest

from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols(header="goc_lbm.h", prefix="goc_lbm_"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2607_15362_amd import build
        build.build(force=True)
    return B.lib()


def test_library_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in goc_lbm.h but not exported"
        assert s in B.SIGNATURES, f"{s} has no binding signature"


def test_instrument_library_exports_every_declared_symbol():
    from paper_2607_15362_amd import ceiling as CL
    if not os.path.exists(CL.LIB_PATH):
        from paper_2607_15362_amd import build
        build.build_ceiling(force=True)
    L = CL.lib()
    syms = _declared_symbols("goc_ceiling.h", "goc_ceiling_")
    assert syms == sorted(CL.SIGNATURES)
    for s in syms:
        assert hasattr(L, s), f"{s} declared in goc_ceiling.h but not exported"


def test_instrument_rejects_bad_arguments():
    """Argument checks run on the host, before any device call."""
    import ctypes as C
    from paper_2607_15362_amd import ceiling as CL
    L = CL.lib()
    out = C.c_double(0.0)
    assert L.goc_ceiling_pattern(4096, 1024, 1, 8, 64, 4, 1, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_pattern(4096, 1024, 1, 4, 64, 5, 1, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_pattern(4096, 1024, 1, 4, 96, 4, 1, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_pattern(4096, 1024, 1, 4, 128, 8, 1, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_pattern(2, 1024, 1, 4, 64, 4, 1, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_pattern(4096, 1024, 1, 4, 64, 4, 1, 10, None, None) == B.GOC_EINVAL
    assert L.goc_ceiling_copy(100, 10, None, C.byref(out)) == B.GOC_EINVAL
    assert L.goc_ceiling_copy(1 << 20, 0, None, C.byref(out)) == B.GOC_EINVAL
    for args in [(100, 1, 1, 0, 0, 32, 10),        # not a multiple of 16
                 (1 << 20, 3, 1, 0, 0, 32, 10),    # reads beyond 2
                 (1 << 20, 1, -1, 0, 0, 32, 10),   # negative writes
                 (1 << 20, 0, 0, 0, 0, 32, 10),    # nothing moved
                 (1 << 20, 1, 1, 2, 0, 32, 10),    # store policy neither 0 nor 1
                 (1 << 20, 1, 1, 0, 2, 32, 10),    # sweep order neither 0 nor 1
                 (1 << 20, 1, 1, 0, 0, 0, 10),     # work-groups per CU outside 1 .. 64
                 (1 << 20, 1, 1, 0, 0, 65, 10),
                 (1 << 20, 1, 1, 0, 0, 32, 0)]:    # no timed launch
        assert L.goc_ceiling_mix(*args, None, C.byref(out)) == B.GOC_EINVAL, args
    assert L.goc_ceiling_mix(1 << 20, 1, 1, 0, 0, 32, 10, None, None) == B.GOC_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        B.lib()


@pytest.mark.parametrize("case", [W.channel_64(), W.cavity_1024(), W.hartmann_4096(),
                                  W.Case("r", 6, 50, "periodic", "wall", ("uniform", 0), ("roberts", 1.06),
                                         flow="free", tau=1.0, body_force=(1e-6, 0.0))])
def test_derive_matches_oracle(lib, oracle_lib, case):
    g, m, p = B.derive(case)
    o = oracle_lib
    h1 = o.metric_1d(case.nx, case.stretch_x)[0]
    h2 = o.metric_1d(case.ny, case.stretch_y)[0]
    lat = o.derive(case, h1, h2)
    assert p.omega[4] == pytest.approx(lat.omega[4], rel=1e-13)
    assert p.omega[5] == pytest.approx(lat.omega[5], rel=1e-13)
    for k in (0, 1, 2, 3, 6, 7, 8):
        assert p.omega[k] == 1.0
    assert p.F_ext[0] == pytest.approx(lat.Fext[0], rel=1e-12, abs=1e-300)
    assert p.F_ext[1] == pytest.approx(lat.Fext[1], rel=1e-12, abs=1e-300)
    assert g.u_wall_hi == pytest.approx(lat.u_wall_hi)
    if case.mhd:
        assert p.mhd == 1
        assert p.B0 == pytest.approx(lat.B0, rel=1e-12)
        assert p.tau_m == pytest.approx(lat.tau_m, rel=1e-12)


def test_derive_rejects_bad_input(lib):
    case = W.channel_64()
    g, m, ph = B.case_structs(case)
    p = B.Params()
    g.nx = 2
    assert lib.goc_lbm_derive(g, m, ph, p) == B.GOC_EINVAL
    assert "3" in lib.goc_lbm_last_error().decode()
    g, m, ph = B.case_structs(case)
    ph.tau = 0.4
    assert lib.goc_lbm_derive(g, m, ph, p) == B.GOC_EINVAL
    g, m, ph = B.case_structs(case)
    m.kind_y, m.param_y = B.STRETCH["tanh"], -1.0
    assert lib.goc_lbm_derive(g, m, ph, p) == B.GOC_EINVAL
    g, m, ph = B.case_structs(case)
    m.kind_y = B.STRETCH["array"]   # array kind without arrays
    assert lib.goc_lbm_derive(g, m, ph, p) == B.GOC_EINVAL


def test_create_rejects_bad_input_before_touching_the_device(lib):
    case = W.channel_64()
    g, m, p = B.derive(case)
    h = B.VP()
    p.omega[4] = 2.5
    assert lib.goc_lbm_create(B.C.byref(h), g, m, p, 1, None) == B.GOC_EINVAL
    assert not h.value
    assert lib.goc_lbm_create(None, g, m, p, 1, None) == B.GOC_EINVAL
    g, m, p = B.derive(case)
    assert lib.goc_lbm_create(B.C.byref(h), g, m, p, 7, None) == B.GOC_EINVAL


def test_create_rejects_bad_collision_choice_before_touching_the_device(lib):
    """Collision selector: an unknown model, the SRT model with the printed
    density coefficients, and a batch that mixes models are refused."""
    case = W.channel_64()
    h = B.VP()
    g, m, p = B.derive(case)
    p.collision = 3
    assert lib.goc_lbm_create(B.C.byref(h), g, m, p, 1, None) == B.GOC_EINVAL
    assert "collision" in lib.goc_lbm_last_error().decode()
    g, m, p = B.derive(case.replace(collision="srt", rho_terms=1))
    assert lib.goc_lbm_create(B.C.byref(h), g, m, p, 1, None) == B.GOC_EINVAL
    assert "SRT" in lib.goc_lbm_last_error().decode()
    structs = [B.derive(case.replace(collision=c)) for c in ("raw", "central")]
    G = (B.Grid * 2)(*[s[0] for s in structs])
    M = (B.Metric * 2)(*[s[1] for s in structs])
    P = (B.Params * 2)(*[s[2] for s in structs])
    assert lib.goc_lbm_create_batch(B.C.byref(h), 2, G, M, P, 1, None) == B.GOC_EINVAL
    assert "share one collision" in lib.goc_lbm_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("nx,ny,storage,mhd,ok", [
    (8192, 4096, 1, 1, True),      # FP32 with the D2Q5 slots in the slot pool's rows: 2.7 GB
    (8192, 8192, 1, 1, False),     # the same at 8192 rows: 5.4 GB, above the 4 GiB of 32-bit offsets
    (8192, 4096, 0, 1, False),     # FP64 with the D2Q5 slots: 5.4 GB
    (8192, 8192, 0, 0, False),     # FP64 plain: 4.9 GB
    (12288, 12288, 2, 0, True),    # 16-bit: 2.7 GB
    (16384, 16384, 1, 0, False),   # FP32: 9.7 GB
    (65536, 65536, 2, 0, False),   # beyond 2^31 nodes
])
def test_create_checks_size_limits_before_touching_the_device(lib, nx, ny, storage, mhd, ok):
    """Sizes beyond the per-run limits are refused with GOC_EINVAL and a
    message, before any device call; sizes within them pass validation (on a
    host without a GPU they then fail at the device, with GOC_EDEVICE)."""
    case = W.Case("big", nx, ny, "periodic", "wall", flow="free", tau=0.8, storage="f32", mhd=bool(mhd))
    g, m, p = B.derive(case.replace(nx=64, ny=64))   # derive checks the grid too
    g.nx, g.ny = nx, ny
    p.mhd = mhd
    p.tau_m = 1.0
    h = B.VP()
    rc = lib.goc_lbm_create(B.C.byref(h), g, m, p, storage, None)
    if ok:
        assert rc != B.GOC_EINVAL
    else:
        assert rc == B.GOC_EINVAL
        assert "too large" in lib.goc_lbm_last_error().decode()
    if h.value:
        lib.goc_lbm_destroy(h)


def test_committed_profiles_cover_the_current_kernels():
    """The counter summaries under profiles/ were taken on the current kernel
    sources, for the tiled forms of the FP32 headline the autotuner picks or
    that sit next to its pick, so the benchmark reports measured traffic."""
    import json
    import bench
    sha = bench.kernel_source_hash()
    for form in ("tiled128x4nt", "tiled8nt", "tiled4nt"):
        path = os.path.join(ROOT, "profiles", f"tile_step_kernel_hartmann_4096x1024_{form}_pmc.json")
        with open(path) as fh:
            d = json.load(fh)
        assert d["kernel_source_sha"] == sha, path
        t = bench.measured_traffic("goc::tile_step_kernel", "hartmann_4096x1024", form)
        assert t == d["hbm_bytes_per_launch"]
        assert 1.0 <= t / d["algorithmic_bytes_per_launch"] < 1.1
