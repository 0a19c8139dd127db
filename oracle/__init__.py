"""Plain FP64 CPU oracle of the OpenCFD-SCU right-hand side (arXiv:2209.15333, Sec. 2).

TEST INFRASTRUCTURE.  This package is the independent checker of the GPU
library: only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it.  It shares no code with the GPU path (its C source, header
and parameter struct are its own) and the GPU path never imports it.

The arithmetic lives in ocfd_oracle.c (loops in double precision, built
without contraction); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocfd_oracle.so")

FLAG_LOW, FLAG_WENO7, FLAG_WENO5 = 0, 1, 2
PART_XI, PART_ETA, PART_ZETA, PART_VISC, PART_ALL = 1, 2, 4, 8, 15


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("period", ctypes.c_double * 3),
        ("h", ctypes.c_double * 3),
        ("gamma", ctypes.c_double), ("Re", ctypes.c_double), ("Ma", ctypes.c_double), ("Pr", ctypes.c_double),
        ("Tref", ctypes.c_double), ("suth", ctypes.c_double), ("Tw", ctypes.c_double),
        ("theta1", ctypes.c_double), ("theta2", ctypes.c_double), ("eps", ctypes.c_double),
        ("viscous", ctypes.c_int32), ("scheme", ctypes.c_int32), ("lowdiss", ctypes.c_int32),
        ("three_way", ctypes.c_int32), ("characteristic", ctypes.c_int32), ("flag_window", ctypes.c_int32),
        ("nthreads", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load the oracle library, compiling it first if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_sw_split.argtypes = [pp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, dp, dp, dp]
        L.or_weno7.argtypes = [dp, ctypes.c_double]
        L.or_weno7.restype = ctypes.c_double
        L.or_weno5.argtypes = [dp, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.or_weno5.restype = ctypes.c_double
        L.or_ud7.argtypes = [dp]
        L.or_ud7.restype = ctypes.c_double
        L.or_c8.argtypes = [dp]
        L.or_c8.restype = ctypes.c_double
        L.or_char_matrices.argtypes = [pp, dp, dp, dp, dp]
        L.or_metrics.argtypes = [pp, dp, dp]
        L.or_sensor.argtypes = [pp, dp, dp, u8p]
        L.or_dudt.argtypes = [pp, dp, dp, u8p, ctypes.c_int32, dp]
        L.or_dudt_points.argtypes = [pp, dp, dp, u8p, ctypes.c_int32, ctypes.c_int64, i64p, dp]
        L.or_advance.argtypes = [pp, dp, dp, dp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                 ctypes.c_double, dp]
        L.or_reduce.argtypes = [pp, dp, dp, ctypes.c_double, dp]
        L.or_apply_bc.argtypes = [pp, dp, dp]
        L.or_nrbc_normal.argtypes = [pp, dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, dp]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8p(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_uint8)()
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def params_from_case(case, nthreads: int = 0) -> Params:
    """Oracle parameters for a workloads.Case."""
    P = Params()
    P.nx, P.ny, P.nz = case.nx, case.ny, case.nz
    for d in range(3):
        P.periodic[d] = int(case.periodic[d])
        P.period[d] = float(case.period[d])
        P.h[d] = float(case.h[d])
    for f in range(6):
        P.bc[f] = int(case.bc[f])
    P.gamma, P.Re, P.Ma, P.Pr = case.gamma, case.Re, case.Ma, case.Pr
    P.Tref, P.suth, P.Tw = case.Tref, case.suth, case.Tw
    P.theta1, P.theta2, P.eps = case.theta1, case.theta2, case.eps
    P.viscous = int(case.viscous)
    P.scheme = 1 if case.scheme == "hybrid" else 0
    P.lowdiss = 1 if case.lowdiss == "c8" else 0
    P.three_way = int(bool(case.three_way))
    P.characteristic = int(bool(getattr(case, "characteristic", False)))
    P.flag_window = int(getattr(case, "flag_window", 0))
    P.nthreads = int(nthreads)
    return P


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def sw_split(P: Params, rho, u, v, w, p, alpha):
    fp = np.zeros(5)
    fm = np.zeros(5)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    lib().or_sw_split(ctypes.byref(P), rho, u, v, w, p, _dp(a), _dp(fp), _dp(fm))
    return fp, fm


def char_matrices(P: Params, U, n):
    """(S, S^-1) of eq 34-35 at the conserved state U for the unit normal n (5x5 each)."""
    Uc = np.ascontiguousarray(U, dtype=np.float64)
    nc = np.ascontiguousarray(n, dtype=np.float64)
    S = np.zeros(25)
    Si = np.zeros(25)
    lib().or_char_matrices(ctypes.byref(P), _dp(Uc), _dp(nc), _dp(S), _dp(Si))
    return S.reshape(5, 5), Si.reshape(5, 5)


def weno7(f, eps=1e-6) -> float:
    a = np.ascontiguousarray(f, dtype=np.float64)
    return lib().or_weno7(_dp(a), eps)


def weno5(f, eps=1e-6, valid=(1, 1, 1)) -> float:
    a = np.ascontiguousarray(f, dtype=np.float64)
    v = (ctypes.c_int * 3)(*valid)
    return lib().or_weno5(_dp(a), eps, v)


def ud7(f) -> float:
    return lib().or_ud7(_dp(np.ascontiguousarray(f, dtype=np.float64)))


def c8(f) -> float:
    return lib().or_c8(_dp(np.ascontiguousarray(f, dtype=np.float64)))


def metrics(P: Params, xyz: np.ndarray) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    met = np.zeros((10,) + xyz.shape[1:])
    _check(lib().or_metrics(ctypes.byref(P), _dp(xyz), _dp(met)), "metrics")
    return met


def sensor(P: Params, U: np.ndarray):
    U = np.ascontiguousarray(U, dtype=np.float64)
    theta = np.zeros(U.shape[1:])
    flags = np.zeros((3,) + U.shape[1:], dtype=np.uint8)
    _check(lib().or_sensor(ctypes.byref(P), _dp(U), _dp(theta), _u8p(flags)), "sensor")
    return theta, flags


def dudt(P: Params, met: np.ndarray, U: np.ndarray, flags: Optional[np.ndarray] = None,
         parts: int = PART_ALL) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros_like(U)
    _check(lib().or_dudt(ctypes.byref(P), _dp(met), _dp(U), _u8p(flags), parts, _dp(out)), "dudt")
    return out


def dudt_points(P: Params, met: np.ndarray, U: np.ndarray, nodes: np.ndarray,
                flags: Optional[np.ndarray] = None, parts: int = PART_ALL) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((len(nodes), 5))
    _check(lib().or_dudt_points(ctypes.byref(P), _dp(met), _dp(U), _u8p(flags), parts, len(nodes),
                                nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out)), "dudt_points")
    return out


def advance(P: Params, met: np.ndarray, U: np.ndarray, n: int, dt: float, Un: Optional[np.ndarray] = None,
            stage: int = 0, inflow: Optional[np.ndarray] = None):
    """n substeps from (U, Un, stage); returns (U, Un, stage) as new arrays."""
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    Un = np.array(U if Un is None else Un, dtype=np.float64, order="C", copy=True)
    st = ctypes.c_int32(stage)
    _check(lib().or_advance(ctypes.byref(P), _dp(met), _dp(U), _dp(Un), ctypes.byref(st), n, dt,
                            _dp(inflow)), "advance")
    return U, Un, st.value


def reduce(P: Params, met: np.ndarray, U: np.ndarray, dt: float = 0.0) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros(9)
    _check(lib().or_reduce(ctypes.byref(P), _dp(met), _dp(U), dt, _dp(out)), "reduce")
    return out


def apply_bc(P: Params, U: np.ndarray, inflow: Optional[np.ndarray] = None) -> np.ndarray:
    """The state U with the faces of bounded directions set (a new array)."""
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    _check(lib().or_apply_bc(ctypes.byref(P), _dp(U), _dp(inflow)), "apply_bc")
    return U


def nrbc_normal(P: Params, met: np.ndarray, U: np.ndarray, node, d: int, side: int) -> np.ndarray:
    """Normal-direction part of dU/dt at node (i, j, k) of the nonreflecting
    face (d, side)."""
    out = np.zeros(5)
    i, j, k = node
    _check(lib().or_nrbc_normal(ctypes.byref(P), _dp(np.ascontiguousarray(met)), _dp(np.ascontiguousarray(U)),
                                i, j, k, d, side, _dp(out)), "nrbc_normal")
    return out
