"""ctypes binding of libmpstep.so: the calls of include/mp.h under the same names.

Argument marshalling only; every step of the path runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpstep.so")

MP_OK = 0
MP_E_PARAM, MP_E_UNSTABLE, MP_E_NULLPTR, MP_E_UNBOUND, MP_E_HIP, MP_E_NONFINITE, MP_E_STATE = (
    -1, -2, -3, -4, -5, -6, -7)
MP_BC_PERIODIC, MP_BC_NOFLUX = 0, 1
MP_FP64, MP_FP32 = 0, 1
MP_WELL, MP_OBSTACLE, MP_OBSTACLE_ACTIVE, MP_THETA = 0, 1, 2, 3
POTENTIALS = {"well": MP_WELL, "obstacle": MP_OBSTACLE, "obstacle_active": MP_OBSTACLE_ACTIVE, "theta": MP_THETA}
MP_GP, MP_KKS = 0, 1
MODELS = {"gp": MP_GP, "kks": MP_KKS}

ERROR_NAMES = {
    MP_E_PARAM: "MP_E_PARAM", MP_E_UNSTABLE: "MP_E_UNSTABLE", MP_E_NULLPTR: "MP_E_NULLPTR",
    MP_E_UNBOUND: "MP_E_UNBOUND", MP_E_HIP: "MP_E_HIP", MP_E_NONFINITE: "MP_E_NONFINITE",
    MP_E_STATE: "MP_E_STATE",
}

# Every symbol the header declares (checked by the ABI test).
EXPORTS = [
    "mp_dt_limit", "mp_create", "mp_state_bytes", "mp_workspace_bytes", "mp_bind", "mp_step",
    "mp_current", "mp_set_step", "mp_diagnostics", "mp_set_tile", "mp_get_tile", "mp_destroy",
    "mp_last_error", "mp_set_graph", "mp_create_batch", "mp_instance_count", "mp_instance_offset",
    "mp_diagnostics_batch", "mp_step_ckpt", "mp_adjoint_work_bytes", "mp_adjoint",
    "mp_tune_candidates", "mp_tune", "mp_set_fusion", "mp_get_fusion",
    "mp_set_antitrapping", "mp_get_antitrapping", "mp_diagnostics_static", "mp_front_row", "mp_shift",
    "mp_step_diag",
]

# Layout of the parameter gradient filled by mp_adjoint.
GRAD_NAMES = ["gamma01", "gamma02", "gamma12", "D00", "D01", "D10", "D11", "D20", "D21", "tau"]


class mp_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("bc", C.c_int32 * 3), ("n", C.c_int64 * 3), ("dx", C.c_double)]


class mp_params(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("potential", C.c_int32),
        ("eps", C.c_double), ("tau", C.c_double), ("dt", C.c_double),
        ("gamma", (C.c_double * 3) * 3), ("gamma3", C.c_double), ("delta", (C.c_double * 3) * 3),
        ("A", (C.c_double * 2) * 3), ("B", (C.c_double * 2) * 3), ("C", C.c_double * 3),
        ("s", C.c_double * 3), ("D", (C.c_double * 2) * 3),
        ("Te", C.c_double), ("T0", C.c_double), ("G", C.c_double), ("V", C.c_double),
        ("y0", C.c_double),
        ("Bt", (C.c_double * 2) * 3), ("Ct", C.c_double * 3), ("A01", C.c_double * 3), ("D01", C.c_double * 3),
        ("tau_ab", (C.c_double * 3) * 3),
        ("model", C.c_int32), ("reserved", C.c_int32), ("Mphi", C.c_double),
        ("theta", C.c_double * 3), ("theta_ab", (C.c_double * 3) * 3), ("theta3", C.c_double),
    ]


class mp_diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("nonfinite", C.c_int64), ("max_sum_dev", C.c_double),
        ("mass", C.c_double * 2), ("volume", C.c_double * 3), ("min_chi", C.c_double * 2),
    ]


class MPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2404_01035_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mp_dt_limit.restype = C.c_double
        L.mp_dt_limit.argtypes = [C.POINTER(mp_grid), C.c_int, C.c_int, C.POINTER(mp_params)]
        L.mp_create.restype = C.c_int
        L.mp_create.argtypes = [C.POINTER(mp_grid), C.c_int, C.c_int, C.POINTER(mp_params),
                                C.POINTER(vp)]
        L.mp_state_bytes.restype = C.c_size_t
        L.mp_state_bytes.argtypes = [vp]
        L.mp_workspace_bytes.restype = C.c_size_t
        L.mp_workspace_bytes.argtypes = [vp]
        L.mp_bind.restype = C.c_int
        L.mp_bind.argtypes = [vp, vp, vp, vp]
        L.mp_step.restype = C.c_int
        L.mp_step.argtypes = [vp, C.c_int64, vp]
        L.mp_current.restype = C.c_int
        L.mp_current.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.mp_set_step.restype = C.c_int
        L.mp_set_step.argtypes = [vp, C.c_int64, C.c_int]
        L.mp_diagnostics.restype = C.c_int
        L.mp_diagnostics.argtypes = [vp, C.POINTER(mp_diag), vp]
        L.mp_step_diag.restype = C.c_int
        L.mp_step_diag.argtypes = [vp, C.c_int64, C.POINTER(mp_diag), vp]
        L.mp_diagnostics_static.restype = C.c_int
        L.mp_diagnostics_static.argtypes = [vp, vp, C.c_int64, C.POINTER(mp_diag), vp]
        L.mp_front_row.restype = C.c_int
        L.mp_front_row.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.mp_shift.restype = C.c_int
        L.mp_shift.argtypes = [vp, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64), vp]
        L.mp_set_tile.restype = C.c_int
        L.mp_set_tile.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.mp_get_tile.restype = C.c_int
        L.mp_get_tile.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.mp_destroy.restype = None
        L.mp_destroy.argtypes = [vp]
        L.mp_last_error.restype = C.c_char_p
        L.mp_last_error.argtypes = []
        L.mp_set_graph.restype = C.c_int
        L.mp_set_graph.argtypes = [vp, C.c_int]
        L.mp_create_batch.restype = C.c_int
        L.mp_create_batch.argtypes = [C.c_int, C.POINTER(mp_grid), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(mp_params), C.POINTER(vp)]
        L.mp_instance_count.restype = C.c_int
        L.mp_instance_count.argtypes = [vp, C.POINTER(C.c_int)]
        L.mp_instance_offset.restype = C.c_int
        L.mp_instance_offset.argtypes = [vp, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.mp_diagnostics_batch.restype = C.c_int
        L.mp_diagnostics_batch.argtypes = [vp, C.POINTER(mp_diag), vp]
        L.mp_step_ckpt.restype = C.c_int
        L.mp_step_ckpt.argtypes = [vp, C.c_int64, C.c_int64, vp, vp]
        L.mp_adjoint_work_bytes.restype = C.c_size_t
        L.mp_adjoint_work_bytes.argtypes = [vp, C.c_int64]
        L.mp_adjoint.restype = C.c_int
        L.mp_adjoint.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_int64, vp, vp,
                                 C.POINTER(C.c_double), vp, vp]
        L.mp_set_fusion.restype = C.c_int
        L.mp_set_fusion.argtypes = [vp, C.c_int]
        L.mp_get_fusion.restype = C.c_int
        L.mp_get_fusion.argtypes = [vp, C.POINTER(C.c_int)]
        L.mp_set_antitrapping.restype = C.c_int
        L.mp_set_antitrapping.argtypes = [vp, C.c_int]
        L.mp_get_antitrapping.restype = C.c_int
        L.mp_get_antitrapping.argtypes = [vp, C.POINTER(C.c_int)]
        L.mp_tune_candidates.restype = C.c_int
        L.mp_tune_candidates.argtypes = [vp, C.POINTER(C.c_int32), C.c_int]
        L.mp_tune.restype = C.c_int
        L.mp_tune.argtypes = [vp, C.POINTER(C.c_int32), C.c_int, C.c_int, C.POINTER(C.c_double),
                              C.POINTER(C.c_int), vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != MP_OK:
        raise MPError(rc, lib().mp_last_error().decode())
    return rc


def mp_last_error() -> str:
    return lib().mp_last_error().decode()


def to_grid(p) -> mp_grid:
    g = mp_grid()
    g.dim = int(p.dim)
    for i in range(3):
        g.bc[i] = int(p.bc[i])
        g.n[i] = int(p.n[i])
    g.dx = float(p.dx)
    return g


def to_params(p) -> mp_params:
    c = mp_params()
    c.precision = MP_FP64 if p.precision == "f64" else MP_FP32
    c.potential = POTENTIALS[p.potential]
    c.eps, c.tau, c.dt = float(p.eps), float(p.tau), float(p.dt)
    c.gamma3 = float(p.gamma3)
    g = np.asarray(p.gamma, dtype=np.float64)
    d = np.asarray(p.delta, dtype=np.float64)
    A, B, Dm = (np.asarray(x, dtype=np.float64) for x in (p.A, p.B, p.D))
    for a in range(3):
        c.C[a] = float(p.C[a])
        c.s[a] = float(p.s[a])
        for b in range(3):
            c.gamma[a][b] = float(g[a, b])
            c.delta[a][b] = float(d[a, b])
        for k in range(2):
            c.A[a][k] = float(A[a, k])
            c.B[a][k] = float(B[a, k])
            c.D[a][k] = float(Dm[a, k])
    c.Te, c.T0, c.G, c.V, c.y0 = (float(x) for x in (p.Te, p.T0, p.G, p.V, p.y0))
    Bt, tab = np.asarray(p.Bt, dtype=np.float64), np.asarray(p.tau_ab, dtype=np.float64)
    for a in range(3):
        c.Ct[a] = float(p.Ct[a])
        c.A01[a] = float(p.A01[a])
        c.D01[a] = float(p.D01[a])
        for k in range(2):
            c.Bt[a][k] = float(Bt[a, k])
        for b in range(3):
            c.tau_ab[a][b] = float(tab[a, b])
    c.model = MODELS[getattr(p, "model", "gp")]
    c.Mphi = float(getattr(p, "Mphi", 1.0))
    th = np.asarray(getattr(p, "theta", np.zeros(3)), dtype=np.float64)
    thab = np.asarray(getattr(p, "theta_ab", np.zeros((3, 3))), dtype=np.float64)
    for a in range(3):
        c.theta[a] = float(th[a])
        for b in range(3):
            c.theta_ab[a][b] = float(thab[a, b])
    c.theta3 = float(getattr(p, "theta3", 0.0))
    return c


def mp_dt_limit(p) -> float:
    g, c = to_grid(p), to_params(p)
    return lib().mp_dt_limit(C.byref(g), int(p.nphases), int(p.ncomp), C.byref(c))


def mp_create(p) -> int:
    """Validate and create a state for the problem ``p`` (an inputs.Params); returns a handle."""
    g, c = to_grid(p), to_params(p)
    h = C.c_void_p()
    _check(lib().mp_create(C.byref(g), int(p.nphases), int(p.ncomp), C.byref(c), C.byref(h)))
    return h.value


def mp_state_bytes(st) -> int:
    return int(lib().mp_state_bytes(st))


def mp_workspace_bytes(st) -> int:
    return int(lib().mp_workspace_bytes(st))


def mp_bind(st, buf0: int, buf1: int, workspace: int):
    _check(lib().mp_bind(st, buf0, buf1, workspace))


def mp_step(st, nsteps: int, stream: int = 0):
    _check(lib().mp_step(st, int(nsteps), stream))


def mp_current(st):
    w, s = C.c_int(), C.c_int64()
    _check(lib().mp_current(st, C.byref(w), C.byref(s)))
    return w.value, s.value


def mp_set_step(st, step: int, which_buf: int):
    _check(lib().mp_set_step(st, int(step), int(which_buf)))


def _diag_dict(d) -> dict:
    return {
        "step": d.step, "nonfinite": d.nonfinite, "max_sum_dev": d.max_sum_dev,
        "mass": list(d.mass), "volume": list(d.volume), "min_chi": list(d.min_chi),
    }


def mp_diagnostics(st, stream: int = 0, allow_nonfinite: bool = False) -> dict:
    d = mp_diag()
    rc = lib().mp_diagnostics(st, C.byref(d), stream)
    if rc != MP_OK and not (allow_nonfinite and rc == MP_E_NONFINITE):
        _check(rc)
    return _diag_dict(d)


def mp_step_diag(st, nsteps: int, stream: int = 0, allow_nonfinite: bool = False) -> list:
    """nsteps steps, then the diagnostics of the state reached, their partial
    sums formed by the last step launch; one dict per instance."""
    n = mp_instance_count(st)
    arr = (mp_diag * n)()
    rc = lib().mp_step_diag(st, int(nsteps), arr, stream)
    if rc != MP_OK and not (allow_nonfinite and rc == MP_E_NONFINITE):
        _check(rc)
    return [_diag_dict(arr[i]) for i in range(n)]


def mp_diagnostics_batch(st, stream: int = 0, allow_nonfinite: bool = False) -> list:
    n = mp_instance_count(st)
    arr = (mp_diag * n)()
    rc = lib().mp_diagnostics_batch(st, arr, stream)
    if rc != MP_OK and not (allow_nonfinite and rc == MP_E_NONFINITE):
        _check(rc)
    return [_diag_dict(arr[i]) for i in range(n)]


def mp_diagnostics_static(st, state_buf: int, step: int, stream: int = 0,
                          allow_nonfinite: bool = False) -> list:
    """Diagnostics of the state in device buffer ``state_buf`` at time level
    ``step``, reduced in the library's static scratch (no workspace); one dict
    per instance."""
    n = mp_instance_count(st)
    arr = (mp_diag * n)()
    rc = lib().mp_diagnostics_static(st, state_buf, int(step), arr, stream)
    if rc != MP_OK and not (allow_nonfinite and rc == MP_E_NONFINITE):
        _check(rc)
    return [_diag_dict(arr[i]) for i in range(n)]


def mp_front_row(st, stream: int = 0) -> int:
    """Highest row holding a cell with liquid fraction below 1/2 (-1 if none)."""
    r = C.c_int64()
    _check(lib().mp_front_row(st, C.byref(r), stream))
    return r.value


def mp_shift(st, rows: int, mu_melt, stream: int = 0) -> int:
    """Shift the frame up by ``rows`` with melt at ``mu_melt``; returns the total offset."""
    m = (C.c_double * 2)(*([float(v) for v in mu_melt] + [0.0, 0.0])[:2])
    off = C.c_int64()
    _check(lib().mp_shift(st, int(rows), m, C.byref(off), stream))
    return off.value


def mp_create_batch(plist) -> int:
    """One batched state for a list of 2D problems (inputs.Params); returns a handle."""
    n = len(plist)
    grids = (mp_grid * n)(*[to_grid(p) for p in plist])
    params = (mp_params * n)(*[to_params(p) for p in plist])
    nph = (C.c_int * n)(*[int(p.nphases) for p in plist])
    ncp = (C.c_int * n)(*[int(p.ncomp) for p in plist])
    h = C.c_void_p()
    _check(lib().mp_create_batch(n, grids, nph, ncp, params, C.byref(h)))
    return h.value


def mp_instance_count(st) -> int:
    n = C.c_int()
    _check(lib().mp_instance_count(st, C.byref(n)))
    return n.value


def mp_instance_offset(st, i: int):
    off, nb = C.c_size_t(), C.c_size_t()
    _check(lib().mp_instance_offset(st, int(i), C.byref(off), C.byref(nb)))
    return off.value, nb.value


def mp_set_fusion(st, steps: int):
    _check(lib().mp_set_fusion(st, int(steps)))


def mp_get_fusion(st) -> int:
    v = C.c_int()
    _check(lib().mp_get_fusion(st, C.byref(v)))
    return v.value


def mp_set_antitrapping(st, on):
    """on: False/0 off, True/1 on (folded into the 2D step), 2 on with the separate correction kernel."""
    _check(lib().mp_set_antitrapping(st, int(on)))


def mp_get_antitrapping(st) -> int:
    v = C.c_int()
    _check(lib().mp_get_antitrapping(st, C.byref(v)))
    return v.value


def mp_set_graph(st, chunk: int):
    _check(lib().mp_set_graph(st, int(chunk)))


def mp_set_tile(st, bx: int = 0, seg: int = 0, vec: int = 0):
    _check(lib().mp_set_tile(st, int(bx), int(seg), int(vec)))


def mp_get_tile(st):
    bx, seg, vec = C.c_int(), C.c_int(), C.c_int()
    _check(lib().mp_get_tile(st, C.byref(bx), C.byref(seg), C.byref(vec)))
    return bx.value, seg.value, vec.value


def mp_destroy(st):
    if st:
        lib().mp_destroy(st)


def mp_step_ckpt(st, nsteps: int, every: int, ckpt_buf: int, stream: int = 0):
    _check(lib().mp_step_ckpt(st, int(nsteps), int(every), ckpt_buf, stream))


def mp_adjoint_work_bytes(st, every: int) -> int:
    return int(lib().mp_adjoint_work_bytes(st, int(every)))


def mp_adjoint(st, ckpt_buf: int, nsteps: int, every: int, n0: int, lam_final: int,
               lam_initial: int, work: int, stream: int = 0) -> dict:
    """Adjoint sweep; returns the parameter gradient as a dict keyed by GRAD_NAMES."""
    g = (C.c_double * 10)()
    _check(lib().mp_adjoint(st, ckpt_buf, int(nsteps), int(every), int(n0), lam_final,
                            lam_initial, g, work, stream))
    return dict(zip(GRAD_NAMES, list(g)))


def mp_tune_candidates(st):
    """The (bx, seg, vec, steps per launch) candidates the library accepts for this state."""
    L = lib()
    n = L.mp_tune_candidates(st, None, 0)
    _check(min(n, 0))
    buf = (C.c_int32 * (4 * n))()
    _check(min(L.mp_tune_candidates(st, buf, n), 0))
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(n)]


def mp_tune(st, cand, reps: int, stream: int = 0):
    """Time each candidate; returns (ms per step list, index of the fastest, now set)."""
    n = len(cand)
    buf = (C.c_int32 * (4 * n))(*[int(v) for tri in cand for v in tri])
    ms = (C.c_double * n)()
    best = C.c_int(-1)
    _check(lib().mp_tune(st, buf, n, int(reps), ms, C.byref(best), stream))
    return list(ms), best.value
