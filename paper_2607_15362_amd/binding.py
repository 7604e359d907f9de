"""ctypes binding of libgoclbm.so (argument marshalling only).

Every step of the method runs in the HIP library; this module converts a
workload description into the C structs of include/goc_lbm.h, moves numpy /
torch buffers in and out and turns status codes into exceptions.  It fails
loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoclbm.so")

GOC_OK, GOC_EINVAL, GOC_ENOMEM, GOC_EDEVICE, GOC_EUNSTABLE, GOC_ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f64": 0, "f32": 1, "f16dev": 2, "bf16dev": 3}
STRETCH = {"array": 0, "uniform": 1, "tanh": 2, "roberts": 3, "annulus": 4, "array2d": 5}
FLOW = {"channel": 0, "cavity": 1, "hartmann": 2, "free": 3}
BC = {"periodic": 0, "wall": 1}
COLLISION = {"central": 0, "raw": 1, "srt": 2}


class GocError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"goc_lbm error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc_x", C.c_int32), ("bc_y", C.c_int32),
                ("u_wall_lo", C.c_double), ("u_wall_hi", C.c_double),
                ("v_wall_lo", C.c_double), ("v_wall_hi", C.c_double)]


class Metric(C.Structure):
    _fields_ = [("kind_x", C.c_int32), ("kind_y", C.c_int32), ("param_x", C.c_double),
                ("param_y", C.c_double), ("h1", C.POINTER(C.c_double)), ("h2", C.POINTER(C.c_double)),
                ("dh1", C.POINTER(C.c_double)), ("dh2", C.POINTER(C.c_double)),
                ("h1_face", C.c_double * 2), ("h2_face", C.c_double * 2),
                ("n_theta", C.c_double),
                ("h1_2d", C.POINTER(C.c_double)), ("h2_2d", C.POINTER(C.c_double)),
                ("d1h1", C.POINTER(C.c_double)), ("d2h1", C.POINTER(C.c_double)),
                ("d1h2", C.POINTER(C.c_double)), ("d2h2", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("omega", C.c_double * 9), ("rho0", C.c_double), ("F_ext", C.c_double * 2),
                ("gi_terms", C.c_int32), ("q3_sign", C.c_int32), ("rho_terms", C.c_int32),
                ("lid_corners", C.c_int32), ("mhd", C.c_int32), ("tau_m", C.c_double),
                ("mu_m", C.c_double), ("B0", C.c_double), ("collision", C.c_int32)]


class Physics(C.Structure):
    _fields_ = [("flow", C.c_int32), ("Re", C.c_double), ("Ha", C.c_double), ("Pm", C.c_double),
                ("Ma", C.c_double), ("tau", C.c_double), ("tau_max", C.c_double),
                ("u_lid", C.c_double), ("rho0", C.c_double),
                ("mu_m", C.c_double), ("F_ext", C.c_double * 2)]


_lib = None
P_D = C.POINTER(C.c_double)
VP = C.c_void_p

# exported symbols and their signatures (the names of include/goc_lbm.h)
SIGNATURES = {
    "goc_lbm_derive": (C.c_int, [C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Physics), C.POINTER(Params)]),
    "goc_lbm_create": (C.c_int, [C.POINTER(VP), C.POINTER(Grid), C.POINTER(Metric), C.POINTER(Params),
                                 C.c_int32, VP]),
    "goc_lbm_create_batch": (C.c_int, [C.POINTER(VP), C.c_int32, C.POINTER(Grid), C.POINTER(Metric),
                                       C.POINTER(Params), C.c_int32, VP]),
    "goc_lbm_init": (C.c_int, [VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_init_mhd": (C.c_int, [VP, VP, VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_init_run": (C.c_int, [VP, C.c_int32, VP, VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_derived_run": (C.c_int, [VP, C.c_int32, P_D]),
    "goc_lbm_step": (C.c_int, [VP, C.c_int64]),
    "goc_lbm_moments": (C.c_int, [VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_moments_run": (C.c_int, [VP, C.c_int32, VP, VP, VP, C.c_int32]),
    "goc_lbm_diagnostics": (C.c_int, [VP, P_D]),
    "goc_lbm_diagnostics_run": (C.c_int, [VP, C.c_int32, P_D]),
    "goc_lbm_diagnostics_noalloc": (C.c_int, [VP, C.c_int32, VP]),
    "goc_lbm_set_watchdog": (C.c_int, [VP, C.c_int64]),
    "goc_lbm_get_populations": (C.c_int, [VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_get_populations_run": (C.c_int, [VP, C.c_int32, VP, VP, VP, C.c_int32]),
    "goc_lbm_set_populations": (C.c_int, [VP, VP, VP, VP, C.c_int32]),
    "goc_lbm_get_state": (C.c_int, [VP, VP, C.POINTER(C.c_size_t)]),
    "goc_lbm_set_state": (C.c_int, [VP, VP, C.c_size_t]),
    "goc_lbm_derived": (C.c_int, [VP, P_D]),
    "goc_lbm_metric": (C.c_int, [VP, P_D, P_D, P_D, P_D]),
    "goc_lbm_metric_2d": (C.c_int, [VP, C.c_int32, P_D, P_D, P_D, P_D, P_D, P_D]),
    "goc_lbm_destroy": (None, [VP]),
    "goc_lbm_last_error": (C.c_char_p, []),
    "goc_lbm_num_runs": (C.c_int32, [VP]),
    "goc_lbm_set_launch": (C.c_int, [VP, C.c_double]),
    "goc_lbm_launch_info": (C.c_int, [VP, P_D]),
    "goc_lbm_tune": (C.c_int, [VP, C.c_int32, P_D]),
    "goc_lbm_set_tile": (C.c_int, [VP, C.c_int32, C.c_int32]),
    "goc_lbm_set_tile_shape": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32]),
}


def lib():
    """Load libgoclbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_2607_15362_amd.build.build() (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != GOC_OK:
        raise GocError(rc, lib().goc_lbm_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(P_D)


def _vptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()   # torch tensor


def case_structs(case):
    """Grid, Metric and Physics structs of a workload description."""
    vw = getattr(case, "v_wall", (0.0, 0.0))
    g = Grid(case.nx, case.ny, BC[case.bc_x], BC[case.bc_y], 0.0, 0.0, float(vw[0]), float(vw[1]))
    m = Metric()
    m.kind_x, m.param_x = STRETCH[case.stretch_x[0]], float(case.stretch_x[1])
    m.kind_y, m.param_y = STRETCH[case.stretch_y[0]], float(case.stretch_y[1])
    g2 = getattr(case, "grid2d", None)
    if g2 is not None:
        if g2[0] == "annulus":
            m.kind_x = STRETCH["annulus"]
            m.param_x, m.param_y, m.n_theta = float(g2[1]), float(g2[2]), float(g2[3])
        elif g2[0] == "wavy":
            from . import workloads as W
            h1, h2 = W.wavy_metric(case.nx, case.ny, float(g2[1]))
            m.kind_x = STRETCH["array2d"]
            m.h1_2d, m.h2_2d = _dptr(h1), _dptr(h2)
            m._keep = (h1, h2)     # the arrays must outlive the create call
        else:
            raise ValueError(f"unknown 2-D grid {g2[0]}")
    ph = Physics()
    ph.flow = FLOW[case.flow]
    ph.Re, ph.Ha, ph.Pm, ph.Ma = case.Re, case.Ha, case.Pm, case.Ma
    ph.tau, ph.u_lid, ph.rho0, ph.mu_m = case.tau, case.u_lid, case.rho0, case.mu_m
    ph.tau_max = getattr(case, "tau_max", 0.0)
    ph.F_ext[0], ph.F_ext[1] = case.body_force
    return g, m, ph


def derive(case):
    g, m, ph = case_structs(case)
    p = Params()
    _check(lib().goc_lbm_derive(C.byref(g), C.byref(m), C.byref(ph), C.byref(p)))
    p.gi_terms, p.q3_sign, p.rho_terms, p.lid_corners = (case.gi_terms, case.q3_sign,
                                                         case.rho_terms, case.lid_corners)
    p.collision = COLLISION[getattr(case, "collision", "central")]
    if not case.mhd:
        p.mhd = 0
    return g, m, p


_hip = None


def hip():
    """The HIP runtime (stream and event calls only)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipStreamCreate.argtypes = [C.POINTER(VP)]
        _hip.hipStreamDestroy.argtypes = [VP]
        _hip.hipStreamSynchronize.argtypes = [VP]
        _hip.hipEventCreate.argtypes = [C.POINTER(VP)]
        _hip.hipEventRecord.argtypes = [VP, VP]
        _hip.hipEventSynchronize.argtypes = [VP]
        _hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), VP, VP]
        _hip.hipEventDestroy.argtypes = [VP]
    return _hip


class Stream:
    """A HIP stream at the default priority, owned by the binding (a
    non-NULL stream so that blocks of steps can be captured in graphs)."""

    def __init__(self):
        self.handle = VP()
        if hip().hipStreamCreate(C.byref(self.handle)) != 0:
            raise GocError(GOC_EDEVICE, "hipStreamCreate failed")

    def synchronize(self):
        if hip().hipStreamSynchronize(self.handle) != 0:
            raise GocError(GOC_EDEVICE, "hipStreamSynchronize failed")

    def __del__(self):
        try:
            if self.handle:
                hip().hipStreamDestroy(self.handle)
        except Exception:
            pass


class Event:
    def __init__(self):
        self.handle = VP()
        if hip().hipEventCreate(C.byref(self.handle)) != 0:
            raise GocError(GOC_EDEVICE, "hipEventCreate failed")

    def record(self, stream):
        hip().hipEventRecord(self.handle, stream.handle if isinstance(stream, Stream) else stream)

    def elapsed_ms(self, end) -> float:
        hip().hipEventSynchronize(end.handle)
        ms = C.c_float(0)
        hip().hipEventElapsedTime(C.byref(ms), self.handle, end.handle)
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle:
                hip().hipEventDestroy(self.handle)
        except Exception:
            pass


def default_stream():
    s = Stream()
    return s, s.handle.value


class Run:
    """One GOC-LBM run (or a batch) living on the GPU."""

    def __init__(self, case=None, *, structs=None, storage=None, stream=None, batch=None):
        self._keep = []
        self.stream_obj = None
        if stream is None:
            self.stream_obj, stream = default_stream()
        self.stream = stream
        h = VP()
        if batch is not None:
            n = len(batch)
            grids = (Grid * n)()
            metrics = (Metric * n)()
            params = (Params * n)()
            for k, c in enumerate(batch):
                g, m, p = derive(c)
                self._keep.append(m)
                grids[k], metrics[k], params[k] = g, m, p
            st = STORAGE[storage or batch[0].storage]
            _check(lib().goc_lbm_create_batch(C.byref(h), n, grids, metrics, params, st, stream))
            self.cases = list(batch)
            self.case = batch[0]
        else:
            if structs is None:
                structs = derive(case)
            g, m, p = structs
            self.grid, self.metric, self.params = g, m, p
            st = STORAGE[storage or case.storage]
            _check(lib().goc_lbm_create(C.byref(h), C.byref(g), C.byref(m), C.byref(p), st, stream))
            self.cases = [case]
            self.case = case
        self.h = h
        self.nx, self.ny = self.case.nx, self.case.ny

    def close(self):
        if self.h:
            lib().goc_lbm_destroy(self.h)
            self.h = None

    def synchronize(self):
        if self.stream_obj is not None:
            self.stream_obj.synchronize()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls ---------------------------------------------------------
    def init_run(self, run, rho, u1, u2, b1=None, b2=None):
        """Initial fields of one run of a batch (the others are unchanged)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, u1, u2)]
        bs = [None, None] if b1 is None else [np.ascontiguousarray(a, dtype=np.float64) for a in (b1, b2)]
        ptr = [a.ctypes.data for a in arrs] + [None if b is None else b.ctypes.data for b in bs]
        _check(lib().goc_lbm_init_run(self.h, int(run), *ptr, 0))
        return self

    def init(self, rho=None, u1=None, u2=None, b1=None, b2=None):
        if rho is None:
            _check(lib().goc_lbm_init(self.h, None, None, None, 0))
            return self
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, u1, u2)]
        if b1 is None and b2 is None:
            _check(lib().goc_lbm_init(self.h, *[a.ctypes.data for a in arrs], 0))
            return self
        arrs += [np.ascontiguousarray(a, dtype=np.float64) for a in (b1, b2)]
        _check(lib().goc_lbm_init_mhd(self.h, *[a.ctypes.data for a in arrs], 0))
        return self

    def step(self, n=1):
        _check(lib().goc_lbm_step(self.h, int(n)))
        return self

    def fields(self, run=0):
        case = self.cases[run]
        N = case.nx * case.ny
        rho = np.zeros(N)
        u = np.zeros(2 * N)
        B = np.zeros(2 * N)
        _check(lib().goc_lbm_moments_run(self.h, run, rho.ctypes.data, u.ctypes.data, B.ctypes.data, 0))
        sh = (case.ny, case.nx)
        d = dict(rho=rho.reshape(sh), U1=u[:N].reshape(sh), U2=u[N:].reshape(sh))
        if case.mhd:
            d.update(B1=B[:N].reshape(sh), B2=B[N:].reshape(sh))
        return d

    def fields_device(self, rho, u, B=None):
        """Write the fields into torch device tensors (no host copy)."""
        _check(lib().goc_lbm_moments(self.h, _vptr(rho), _vptr(u), _vptr(B), 1))

    def populations(self, run=0):
        case = self.cases[run]
        N = case.nx * case.ny
        f = np.zeros(9 * N)
        F = np.zeros(2 * N)
        g = np.zeros(10 * N)
        _check(lib().goc_lbm_get_populations_run(self.h, run, f.ctypes.data, F.ctypes.data,
                                                 g.ctypes.data, 0))
        sh = (case.ny, case.nx)
        return f.reshape((9,) + sh), F.reshape((2,) + sh), g.reshape((10,) + sh)

    def set_populations(self, f, F, g=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.float64)
        gp = None
        if g is not None:
            g = np.ascontiguousarray(g, dtype=np.float64)
            gp = g.ctypes.data
        _check(lib().goc_lbm_set_populations(self.h, f.ctypes.data, F.ctypes.data, gp, 0))

    def diagnostics(self, run=None):
        """The eight global sums (run 0, or run `run` of a batch)."""
        out = np.zeros(8)
        if run is None:
            _check(lib().goc_lbm_diagnostics(self.h, _dptr(out)))
        else:
            _check(lib().goc_lbm_diagnostics_run(self.h, int(run), _dptr(out)))
        return out

    def set_watchdog(self, every):
        _check(lib().goc_lbm_set_watchdog(self.h, int(every)))

    def get_state(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().goc_lbm_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().goc_lbm_get_state(self.h, C.cast(buf, VP), C.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().goc_lbm_set_state(self.h, C.cast(buf, VP), len(blob)))

    def derived(self, run=0):
        out = np.zeros(16)
        _check(lib().goc_lbm_derived_run(self.h, int(run), _dptr(out)))
        keys = ["cs2", "nu", "zeta", "q", "csm2", "eta", "tau_m", "B0", "F1", "F2", "hw_lo", "hw_hi",
                "step", "bytes_per_node", "nx", "ny"]
        return dict(zip(keys, out))

    def num_runs(self):
        return int(lib().goc_lbm_num_runs(self.h))

    def set_launch(self, waves_per_cu):
        _check(lib().goc_lbm_set_launch(self.h, float(waves_per_cu)))
        return self

    def set_tile(self, rows, nontemporal=None, cols=64):
        """The tiled step with tiles of `cols` x `rows` nodes (64 x 4, 8 or
        16; 128 x 4) and non-temporal (1) or plain (0) stores (None: as now)."""
        nt = self.launch_info()["nontemporal"] if nontemporal is None else int(nontemporal)
        if int(cols) == 64:
            _check(lib().goc_lbm_set_tile(self.h, int(rows), int(nt)))
        else:
            _check(lib().goc_lbm_set_tile_shape(self.h, int(cols), int(rows), int(nt)))
        return self

    def launch_info(self):
        out = np.zeros(6)
        _check(lib().goc_lbm_launch_info(self.h, _dptr(out)))
        return dict(waves_per_cu=out[0], blocks=int(out[1]), rows_per_segment=out[2], strips=int(out[3]),
                    nontemporal=int(out[4]), tile_cols=int(out[5]))

    def tune(self, trial_steps=20):
        """Autotune the launch plan (the state does not change)."""
        out = np.zeros(4)
        _check(lib().goc_lbm_tune(self.h, int(trial_steps), _dptr(out)))
        return dict(waves_per_cu=out[0], us_per_step=out[1], us_before=out[2], candidates=int(out[3]))

    def metric_2d(self, run=0):
        """Node metric (h1, h2, th11, th12, th21, th22), each [ny, nx] FP64."""
        c = self.cases[run]
        out = [np.zeros((c.ny, c.nx)) for _ in range(6)]
        _check(lib().goc_lbm_metric_2d(self.h, int(run), *[_dptr(o) for o in out]))
        return tuple(out)

    def metric_arrays(self):
        h1, t1 = np.zeros(self.nx), np.zeros(self.nx)
        h2, t2 = np.zeros(self.ny), np.zeros(self.ny)
        _check(lib().goc_lbm_metric(self.h, _dptr(h1), _dptr(t1), _dptr(h2), _dptr(t2)))
        return h1, t1, h2, t2
