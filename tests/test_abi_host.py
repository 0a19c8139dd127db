"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function its header declares, and rejects bad arguments before any
device work."""
import ctypes
import os

import pytest

from helpers import ROOT, header_functions

LIB = os.path.join(ROOT, "paper_2209_15333_amd", "libocfd.so")


@pytest.fixture(scope="module")
def ocfd():
    if not os.path.exists(LIB):
        pytest.fail("libocfd.so has not been built (run __graft_entry__.build())")
    import paper_2209_15333_amd as pk
    return pk


def test_exports_every_declared_symbol(ocfd):
    names = header_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_header_and_binding_agree(ocfd):
    """The Python binding exposes every C entry point under the same name."""
    missing = [n for n in header_functions() if n not in ("ocfd_kernel_name", "ocfd_last_error")
               and not hasattr(ocfd, n)]
    assert not missing, missing


def test_params_struct_layout(ocfd):
    # 3 + 3 + 6 int32, 3 + 3 + 10 double, 12 int32, 1 double
    assert ctypes.sizeof(ocfd.ocfd_params) == 232
    assert ocfd.ocfd_params.characteristic.offset == 208
    assert ocfd.ocfd_params.check_every.offset == 212 and ocfd.ocfd_params.flag_window.offset == 216
    assert ocfd.ocfd_params.sensor_inputs.offset == 220
    assert ocfd.ocfd_params.cfl_max.offset == 224
    assert ocfd.ocfd_params.bc.offset == 24 and ocfd.ocfd_params.period.offset == 48
    assert ocfd.ocfd_params.Tw.offset == 48 + 8 * 12 and ocfd.ocfd_params.viscous.offset == 48 + 8 * 16


def _params(ocfd, **kw):
    p = ocfd.ocfd_params_default()
    p.nx, p.ny, p.nz = 16, 8, 4
    for d in range(3):
        p.h[d] = 0.1
        p.period[d] = 1.6
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_rejects_bad_parameters(ocfd):
    L = ocfd.lib()
    h = ctypes.c_void_p()
    for bad in (dict(nx=0), dict(gamma=1.0), dict(viscous=4), dict(scheme=7), dict(weno_eps=0.0), dict(Ma=-1.0),
                dict(characteristic=2), dict(sensor_inputs=2), dict(check_every=-1), dict(flag_window=2),
                dict(cfl_max=-1.0), dict(cfl_max=float("inf"))):
        p = _params(ocfd, **bad)
        assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == -1, bad
        assert L.ocfd_workspace_bytes(ctypes.byref(p)) == 0
    # bounded directions: at least 8 nodes, known face kinds, one inflow face,
    # a positive wall temperature
    for bad in (dict(ny=4), dict(bc=3, Tw=0.0), dict(bc=7), dict(bc=1, bc2=1)):
        p = _params(ocfd)
        p.periodic[1] = 0
        if "ny" in bad:
            p.ny = bad["ny"]
        if "bc" in bad:
            p.bc[2] = bad["bc"]
        if "bc2" in bad:
            p.bc[3] = bad["bc2"]
        if "Tw" in bad:
            p.Tw = bad["Tw"]
        assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == -1, bad
    p = _params(ocfd)
    p.periodic[1] = 0
    p.bc[2], p.bc[3] = 3, 2
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    assert L.ocfd_set_inflow(h, ctypes.c_void_p(4096)) == -5     # no workspace yet
    L.ocfd_destroy(h)
    p.sensor = 1
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    L.ocfd_destroy(h)
    # the network decides two ways: the three-way hybrid needs the plain sensor
    p.scheme, p.three_way = 1, 1
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == -4
    p.sensor = 0
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    L.ocfd_destroy(h)


def test_substep_count_without_device_work(ocfd):
    L = ocfd.lib()
    assert L.ocfd_substeps_done(None) == -1
    p = _params(ocfd, check_every=10, cfl_max=0.9, flag_window=1)
    h = ctypes.c_void_p()
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    try:
        assert L.ocfd_substeps_done(h) == 0
    finally:
        L.ocfd_destroy(h)


def test_workspace_and_order_errors(ocfd):
    L = ocfd.lib()
    p = _params(ocfd)
    h = ctypes.c_void_p()
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    try:
        need = L.ocfd_workspace_bytes(ctypes.byref(p))
        assert need >= 47 * 8 * 16 * 8 * 4
        assert L.ocfd_advance(h, 1, 1e-3) == -5                  # no workspace yet
        assert L.ocfd_bind_workspace(h, ctypes.c_void_p(4096 + 8), need) == -1   # misaligned
        assert L.ocfd_bind_workspace(h, ctypes.c_void_p(4096), need - 1) == -2   # too small
        assert b"needed" in L.ocfd_last_error(h)
        assert L.ocfd_bind_workspace(h, None, need) == -1
    finally:
        L.ocfd_destroy(h)


def test_sensor_host_checks(ocfd):
    from oracle import mlp
    L = ocfd.lib()
    assert L.ocfd_sensor_nparams() == mlp.NPARAM == 10497
    assert L.ocfd_sensor_sample_bytes(0) == 0
    assert L.ocfd_sensor_sample_bytes(1000) == 1000 * 77
    p = _params(ocfd)
    h = ctypes.c_void_p()
    assert L.ocfd_create(ctypes.byref(p), None, ctypes.byref(h)) == 0
    try:
        assert L.ocfd_sensor_set_threshold(h, ctypes.c_double(1.5)) == -1
        assert L.ocfd_sensor_set_threshold(h, ctypes.c_double(0.25)) == 0
        t3 = (ctypes.c_double * 3)()
        assert L.ocfd_sensor_get_thresholds(h, t3) == 0 and list(t3) == [0.25] * 3
        assert L.ocfd_sensor_set_thresholds(h, (ctypes.c_double * 3)(0.1, 0.2, 1.5)) == -1
        assert L.ocfd_sensor_set_thresholds(h, (ctypes.c_double * 3)(0.1, 0.2, 0.3)) == 0
        assert L.ocfd_sensor_get_thresholds(h, t3) == 0 and list(t3) == [0.1, 0.2, 0.3]
        assert L.ocfd_sensor_bind_samples(h, ctypes.c_void_p(4096), 16 * 77 - 1) == -2
        assert L.ocfd_sensor_bind_samples(h, ctypes.c_void_p(4097), 10 ** 6) == -1
        out = (ctypes.c_double * 6)()
        assert L.ocfd_sensor_audit(h, out) == 0 and list(out) == [0.0] * 6
    finally:
        L.ocfd_destroy(h)
    bad = _params(ocfd)
    bad.sensor = 5
    assert L.ocfd_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
