"""MI355X (gfx950) right-hand side and Runge-Kutta march of the OpenCFD-SCU
finite-difference solver for compressible turbulence (Dang et al.,
arXiv:2209.15333, Section 2).

The numerics live in the HIP library libocfd.so (C ABI: include/ocfd.h).  This
package only marshals arguments: the functions below carry the names of the C
entry points and pass device pointers of torch tensors and torch's current
HIP stream.  There is no CPU fallback; importing fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocfd.so")

OCFD_OK = 0
OCFD_SCHEME_WENO7, OCFD_SCHEME_HYBRID = 0, 1
OCFD_LOWDISS_UD7, OCFD_LOWDISS_C8 = 0, 1
OCFD_PREC_FP64, OCFD_PREC_MIXED = 0, 1
OCFD_SENSOR_PLAIN, OCFD_SENSOR_LEARNED = 0, 1
OCFD_INPUTS_JUMP, OCFD_INPUTS_CURV = 0, 1
OCFD_BC_NONE, OCFD_BC_INFLOW, OCFD_BC_EXTRAP, OCFD_BC_WALL, OCFD_BC_NRBC = 0, 1, 2, 3, 4
OCFD_PART_XI, OCFD_PART_ETA, OCFD_PART_ZETA, OCFD_PART_VISC, OCFD_PART_ALL = 1, 2, 4, 8, 15
OCFD_RED_WENO0 = 9
OCFD_RED_COUNT = 12
OCFD_K_COUNT = 6
ERRORS = {-1: "BADARG", -2: "BADSIZE", -3: "HIP", -4: "UNSUPPORTED", -5: "STATE", -6: "NONFINITE", -7: "CFL"}
OCFD_ERR_NONFINITE, OCFD_ERR_CFL = -6, -7


class ocfd_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("period", ctypes.c_double * 3),
        ("h", ctypes.c_double * 3),
        ("gamma", ctypes.c_double), ("Re", ctypes.c_double), ("Ma", ctypes.c_double), ("Pr", ctypes.c_double),
        ("Tref", ctypes.c_double), ("suth", ctypes.c_double), ("Tw", ctypes.c_double),
        ("theta1", ctypes.c_double), ("theta2", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("viscous", ctypes.c_int32), ("scheme", ctypes.c_int32), ("lowdiss", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("sensor", ctypes.c_int32), ("sensor_every", ctypes.c_int32), ("audit_every", ctypes.c_int32),
        ("three_way", ctypes.c_int32),
        ("characteristic", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("flag_window", ctypes.c_int32), ("sensor_inputs", ctypes.c_int32),
        ("cfl_max", ctypes.c_double),
    ]


class OcfdError(RuntimeError):
    """A failed entry point; .code is its OCFD_ERR_* value."""

    def __init__(self, msg: str, code: int = 0):
        super().__init__(msg)
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library.  torch is imported first so that the library
    binds to the HIP runtime torch already loaded."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OcfdError(f"{LIB_PATH} is missing: build it with `python -m paper_2209_15333_amd.build` "
                            "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(ocfd_params)
        L.ocfd_params_default.argtypes = [pp]
        L.ocfd_workspace_bytes.argtypes = [pp]
        L.ocfd_workspace_bytes.restype = ctypes.c_size_t
        L.ocfd_create.argtypes = [pp, vp, ctypes.POINTER(vp)]
        L.ocfd_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        for name in ("ocfd_set_grid", "ocfd_set_metrics", "ocfd_get_metrics", "ocfd_set_state", "ocfd_get_state",
                     "ocfd_set_flags", "ocfd_set_inflow"):
            getattr(L, name).argtypes = [vp, vp]
        L.ocfd_get_step_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
        L.ocfd_set_step_state.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.ocfd_advance.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
        L.ocfd_substeps_done.argtypes = [vp]
        L.ocfd_substeps_done.restype = ctypes.c_int64
        L.ocfd_dudt.argtypes = [vp, vp, vp, ctypes.c_int32]
        L.ocfd_reduce.argtypes = [vp, ctypes.c_double, dp]
        L.ocfd_reduce_static.argtypes = [pp, vp, vp, ctypes.c_double, vp, vp]
        L.ocfd_profile.argtypes = [vp, ctypes.c_int32]
        L.ocfd_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.ocfd_kernel_name.argtypes = [ctypes.c_int32]
        L.ocfd_kernel_name.restype = ctypes.c_char_p
        L.ocfd_last_error.argtypes = [vp]
        L.ocfd_last_error.restype = ctypes.c_char_p
        L.ocfd_destroy.argtypes = [vp]
        L.ocfd_destroy.restype = None
        fp = ctypes.POINTER(ctypes.c_float)
        L.ocfd_sensor_nparams.argtypes = []
        L.ocfd_sensor_nparams.restype = ctypes.c_int32
        L.ocfd_sensor_set_params.argtypes = [vp, fp]
        L.ocfd_sensor_get_params.argtypes = [vp, fp]
        L.ocfd_sensor_set_threshold.argtypes = [vp, ctypes.c_double]
        L.ocfd_sensor_get_thresholds.argtypes = [vp, dp]
        L.ocfd_sensor_set_thresholds.argtypes = [vp, dp]
        L.ocfd_sensor_flags.argtypes = [vp, vp, ctypes.c_int32, vp]
        L.ocfd_sensor_sample_bytes.argtypes = [ctypes.c_int64]
        L.ocfd_sensor_sample_bytes.restype = ctypes.c_size_t
        L.ocfd_sensor_bind_samples.argtypes = [vp, vp, ctypes.c_size_t]
        L.ocfd_sensor_collect.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_int64)]
        L.ocfd_sensor_train.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                                        ctypes.c_double, dp]
        L.ocfd_sensor_calibrate.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.ocfd_sensor_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int64, fp]
        L.ocfd_sensor_audit.argtypes = [vp, dp]
        _lib = L
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise OcfdError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _check(handle, rc: int, what: str):
    if rc != OCFD_OK:
        msg = lib().ocfd_last_error(handle).decode() if handle else ""
        raise OcfdError(f"{what}: {ERRORS.get(rc, rc)} {msg}", rc)


# ----------------------------------------------------------------- C entry points

def ocfd_params_default() -> ocfd_params:
    p = ocfd_params()
    _check(None, lib().ocfd_params_default(ctypes.byref(p)), "ocfd_params_default")
    return p


def ocfd_workspace_bytes(p: ocfd_params) -> int:
    return int(lib().ocfd_workspace_bytes(ctypes.byref(p)))


def ocfd_create(p: ocfd_params, stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = (stream or torch.cuda.current_stream()).cuda_stream
    _check(None, lib().ocfd_create(ctypes.byref(p), ctypes.c_void_p(st), ctypes.byref(h)), "ocfd_create")
    return h


def ocfd_bind_workspace(h, ws: torch.Tensor):
    _check(h, lib().ocfd_bind_workspace(h, _ptr(ws), ws.numel() * ws.element_size()), "ocfd_bind_workspace")


def ocfd_set_grid(h, xyz: torch.Tensor):
    _check(h, lib().ocfd_set_grid(h, _ptr(xyz)), "ocfd_set_grid")


def ocfd_set_inflow(h, inflow: torch.Tensor):
    _check(h, lib().ocfd_set_inflow(h, _ptr(inflow)), "ocfd_set_inflow")


def ocfd_set_metrics(h, met: torch.Tensor):
    _check(h, lib().ocfd_set_metrics(h, _ptr(met)), "ocfd_set_metrics")


def ocfd_get_metrics(h, met: torch.Tensor):
    _check(h, lib().ocfd_get_metrics(h, _ptr(met)), "ocfd_get_metrics")


def ocfd_set_state(h, U: torch.Tensor):
    _check(h, lib().ocfd_set_state(h, _ptr(U)), "ocfd_set_state")


def ocfd_get_state(h, U: torch.Tensor):
    _check(h, lib().ocfd_get_state(h, _ptr(U)), "ocfd_get_state")


def ocfd_get_step_state(h, Un: torch.Tensor) -> int:
    st = ctypes.c_int32()
    _check(h, lib().ocfd_get_step_state(h, _ptr(Un), ctypes.byref(st)), "ocfd_get_step_state")
    return st.value


def ocfd_set_step_state(h, U: torch.Tensor, Un: torch.Tensor, stage: int):
    _check(h, lib().ocfd_set_step_state(h, _ptr(U), _ptr(Un), stage), "ocfd_set_step_state")


def ocfd_advance(h, n: int, dt: float):
    _check(h, lib().ocfd_advance(h, n, dt), "ocfd_advance")


def ocfd_substeps_done(h) -> int:
    return int(lib().ocfd_substeps_done(h))


def ocfd_dudt(h, U: torch.Tensor, out: torch.Tensor, parts: int = OCFD_PART_ALL):
    _check(h, lib().ocfd_dudt(h, _ptr(U), _ptr(out), parts), "ocfd_dudt")


def ocfd_reduce(h, dt: float = 0.0):
    out = (ctypes.c_double * OCFD_RED_COUNT)()
    _check(h, lib().ocfd_reduce(h, dt, out), "ocfd_reduce")
    return list(out)


def ocfd_reduce_static(p: ocfd_params, U: torch.Tensor, met: torch.Tensor, dt: float, out: torch.Tensor,
                       stream: Optional[torch.cuda.Stream] = None):
    """Enqueue the reduction of U into the device tensor out (OCFD_RED_COUNT
    float64); no allocation, no synchronisation."""
    if out.dtype != torch.float64 or out.numel() < OCFD_RED_COUNT:
        raise OcfdError(f"out must hold {OCFD_RED_COUNT} float64 values")
    st = (stream or torch.cuda.current_stream()).cuda_stream
    _check(None, lib().ocfd_reduce_static(ctypes.byref(p), _ptr(U), _ptr(met), dt, _ptr(out), ctypes.c_void_p(st)),
           "ocfd_reduce_static")


def ocfd_set_flags(h, flags: Optional[torch.Tensor]):
    _check(h, lib().ocfd_set_flags(h, _ptr(flags)), "ocfd_set_flags")


def ocfd_profile(h, enable: bool):
    _check(h, lib().ocfd_profile(h, int(enable)), "ocfd_profile")


def ocfd_profile_read(h):
    ms = (ctypes.c_double * OCFD_K_COUNT)()
    cnt = (ctypes.c_int64 * OCFD_K_COUNT)()
    _check(h, lib().ocfd_profile_read(h, ms, cnt), "ocfd_profile_read")
    return {lib().ocfd_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(OCFD_K_COUNT)}


def ocfd_destroy(h):
    lib().ocfd_destroy(h)


def ocfd_sensor_nparams() -> int:
    return int(lib().ocfd_sensor_nparams())


def _f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def ocfd_sensor_set_params(h, params):
    a, p = _f32(params)
    if a.size != ocfd_sensor_nparams():
        raise OcfdError(f"expected {ocfd_sensor_nparams()} parameters, got {a.size}")
    _check(h, lib().ocfd_sensor_set_params(h, p), "ocfd_sensor_set_params")


def ocfd_sensor_get_params(h):
    import numpy as np
    a, p = _f32(np.zeros(ocfd_sensor_nparams()))
    _check(h, lib().ocfd_sensor_get_params(h, p), "ocfd_sensor_get_params")
    return a


def ocfd_sensor_set_threshold(h, tau: float):
    _check(h, lib().ocfd_sensor_set_threshold(h, tau), "ocfd_sensor_set_threshold")


def ocfd_sensor_set_thresholds(h, tau):
    arr = (ctypes.c_double * 3)(*[float(t) for t in tau])
    _check(h, lib().ocfd_sensor_set_thresholds(h, arr), "ocfd_sensor_set_thresholds")


def ocfd_sensor_get_thresholds(h):
    out = (ctypes.c_double * 3)()
    _check(h, lib().ocfd_sensor_get_thresholds(h, out), "ocfd_sensor_get_thresholds")
    return list(out)


def ocfd_sensor_flags(h, U: torch.Tensor, which: int, flags: torch.Tensor):
    if flags.dtype != torch.uint8:
        raise OcfdError("flags must be uint8")
    _check(h, lib().ocfd_sensor_flags(h, _ptr(U), which, _ptr(flags)), "ocfd_sensor_flags")


def ocfd_sensor_sample_bytes(capacity: int) -> int:
    return int(lib().ocfd_sensor_sample_bytes(capacity))


def ocfd_sensor_bind_samples(h, buf: torch.Tensor):
    _check(h, lib().ocfd_sensor_bind_samples(h, _ptr(buf), buf.numel() * buf.element_size()),
           "ocfd_sensor_bind_samples")


def ocfd_sensor_collect(h, seed: int, keep_weno: float, keep_low: float) -> int:
    tot = ctypes.c_int64()
    _check(h, lib().ocfd_sensor_collect(h, seed, keep_weno, keep_low, ctypes.byref(tot)), "ocfd_sensor_collect")
    return tot.value


def ocfd_sensor_train(h, epochs: int, batch: int, lr: float, seed: int, holdout: float):
    out = (ctypes.c_double * 4)()
    _check(h, lib().ocfd_sensor_train(h, epochs, batch, lr, seed, holdout, out), "ocfd_sensor_train")
    return list(out)


def ocfd_sensor_calibrate(h, holdout: float, margin: float, miss: float = 0.0):
    out = (ctypes.c_double * 4)()
    _check(h, lib().ocfd_sensor_calibrate(h, holdout, margin, miss, out), "ocfd_sensor_calibrate")
    return list(out)


def ocfd_sensor_grad(h, X: torch.Tensor, y: torch.Tensor, w: torch.Tensor):
    """X: [n, 32] int16 tensor holding bf16 bit patterns; y uint8 [n]; w float32 [n]."""
    import numpy as np
    n = X.shape[0]
    g, p = _f32(np.zeros(ocfd_sensor_nparams() + 1))
    _check(h, lib().ocfd_sensor_grad(h, _ptr(X), _ptr(y), _ptr(w), n, p), "ocfd_sensor_grad")
    return g[:-1], float(g[-1])


def ocfd_sensor_audit(h):
    out = (ctypes.c_double * 6)()
    _check(h, lib().ocfd_sensor_audit(h, out), "ocfd_sensor_audit")
    return list(out)


# ----------------------------------------------------------------- convenience

def params_from(case, **overrides) -> ocfd_params:
    """ocfd_params from any object carrying the run attributes (sizes, period,
    h, gamma, Re, Ma, Pr, Tref, suth, theta1, theta2, eps, viscous, scheme,
    lowdiss, periodic; optionally bc, Tw, precision, sensor)."""
    p = ocfd_params_default()
    p.nx, p.ny, p.nz = case.nx, case.ny, case.nz
    for d in range(3):
        p.periodic[d] = int(case.periodic[d])
        p.period[d] = float(case.period[d])
        p.h[d] = float(case.h[d])
    for f in range(6):
        p.bc[f] = int(getattr(case, "bc", (0,) * 6)[f])
    p.gamma, p.Re, p.Ma, p.Pr = case.gamma, case.Re, case.Ma, case.Pr
    p.Tref, p.suth = case.Tref, case.suth
    p.Tw = float(getattr(case, "Tw", 1.0) or 1.0)
    p.theta1, p.theta2, p.weno_eps = case.theta1, case.theta2, case.eps
    p.viscous = int(case.viscous)
    p.scheme = OCFD_SCHEME_HYBRID if case.scheme == "hybrid" else OCFD_SCHEME_WENO7
    p.lowdiss = OCFD_LOWDISS_C8 if case.lowdiss == "c8" else OCFD_LOWDISS_UD7
    p.precision = OCFD_PREC_MIXED if getattr(case, "precision", "fp64") == "mixed" else OCFD_PREC_FP64
    p.sensor = OCFD_SENSOR_LEARNED if getattr(case, "sensor", "plain") == "learned" else OCFD_SENSOR_PLAIN
    p.sensor_every = int(getattr(case, "sensor_every", 1))
    p.audit_every = int(getattr(case, "audit_every", 0))
    p.three_way = int(bool(getattr(case, "three_way", False)))
    p.characteristic = int(bool(getattr(case, "characteristic", False)))
    p.flag_window = int(getattr(case, "flag_window", 0))
    p.sensor_inputs = OCFD_INPUTS_CURV if getattr(case, "sensor_inputs", "jump") == "curv" else OCFD_INPUTS_JUMP
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class Solver:
    """A solver handle with its workspace held in a torch tensor."""

    def __init__(self, params: ocfd_params, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        self.p = params
        self.N = params.nx * params.ny * params.nz
        self.shape = (params.nz, params.ny, params.nx)
        self.device = torch.device(device)
        nbytes = ocfd_workspace_bytes(params)
        if nbytes == 0:
            raise OcfdError("invalid parameters")
        self.h = ocfd_create(params, stream)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ocfd_bind_workspace(self.h, self.ws)

    def close(self):
        if getattr(self, "h", None):
            ocfd_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, nfields: int) -> torch.Tensor:
        return torch.empty((nfields,) + self.shape, dtype=torch.float64, device=self.device)

    def set_grid(self, xyz: torch.Tensor):
        ocfd_set_grid(self.h, xyz)

    def metrics(self) -> torch.Tensor:
        m = self.field(10)
        ocfd_get_metrics(self.h, m)
        return m

    def set_state(self, U: torch.Tensor):
        ocfd_set_state(self.h, U)

    def set_inflow(self, inflow: torch.Tensor):
        ocfd_set_inflow(self.h, inflow)

    def state(self) -> torch.Tensor:
        U = self.field(5)
        ocfd_get_state(self.h, U)
        return U

    def advance(self, n: int, dt: float):
        ocfd_advance(self.h, n, dt)

    def dudt(self, U: torch.Tensor, parts: int = OCFD_PART_ALL) -> torch.Tensor:
        out = self.field(5)
        ocfd_dudt(self.h, U, out, parts)
        return out

    def reduce(self, dt: float = 0.0):
        return ocfd_reduce(self.h, dt)
