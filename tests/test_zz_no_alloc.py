"""goc_lbm_diagnostics_noalloc, the entry point for callers that cannot
allocate, against goc_lbm_diagnostics_run through the C-ABI: the same eight
outputs, bit for bit (the same kernels over the same grid), on two calls in a
row, the second on a smaller run (the static scratch keeps the first call's
partials, which the second must not pick up); its argument checks."""
import ctypes as C

import numpy as np
import pytest

from paper_2607_15362_amd import binding as B
from paper_2607_15362_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(run, k, out):
    return B.lib().goc_lbm_diagnostics_noalloc(run.h, int(k), C.c_void_p(out.data_ptr()))


def test_noalloc_diagnostics_equal_the_allocating_entry_point():
    torch = pytest.importorskip("torch")
    big = W.hartmann_4096().replace(name="na_big", nx=600, ny=260)
    a = B.Run(big)
    d = a.derived()
    a.init(*W.hartmann_start(big, d["nu"], d["F1"], d["eta"], d["B0"]))
    a.step(40)
    small = W.Case("na_small", 70, 45, "wall", "wall", ("tanh", 2.0), ("tanh", 1.5), flow="cavity", Re=100.0,
                   Ma=0.1, storage="f64")
    b = B.Run(small)
    b.init(*W.smooth_fields(70, 45, seed=4, amp=0.01))
    b.step(30)
    print("[no-alloc] 600x260 FP32 MHD, then 70x45 FP64 cavity", flush=True)
    for run in (a, b):
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        assert _noalloc(run, 0, out) == B.GOC_OK, B.lib().goc_lbm_last_error().decode()
        run.synchronize()
        got = out.cpu().numpy()
        ref = run.diagnostics(run=0)
        print("[no-alloc]", got, ref, flush=True)
        assert np.array_equal(got, ref)
        assert ref[0] > 0 and ref[7] == 0
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    assert _noalloc(b, 1, out) == B.GOC_EINVAL
    assert B.lib().goc_lbm_diagnostics_noalloc(b.h, 0, None) == B.GOC_EINVAL
    a.close()
    b.close()


def test_noalloc_diagnostics_of_batch_runs():
    torch = pytest.importorskip("torch")
    runs = W.batch_256(n=4)
    g = B.Run(batch=runs)
    g.step(25)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    for r in (3, 0, 2, 1):   # (larger and smaller runs in turn)
        assert _noalloc(g, r, out) == B.GOC_OK
        g.synchronize()
        assert np.array_equal(out.cpu().numpy(), g.diagnostics(run=r)), r
    g.close()
