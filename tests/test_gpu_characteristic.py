"""Parity of the HIP library's reconstruction in characteristic variables
(Sec. 2.2.2, eq 31-40) with the CPU oracle: dU/dt of WENO7 on a distorted
periodic grid, the three-way hybrid on the oracle's flags, the bounded ramp and
box (masked WENO5 closures in characteristic variables), Runge-Kutta steps
through the Lax tube's shock, and the FP32 form.  Same bars as the
component-wise tests."""
import dataclasses

import numpy as np
import pytest

import workloads
from helpers import rel_errors, ulp_perturbed, assert_within_roundoff

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-12
TOL_DUDT_L2 = 1e-11
TOL_DUDT_INF = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def pk(torch_cuda):
    import paper_2209_15333_amd as pk
    pk.lib()
    return pk


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _solver(pk, torch, case):
    s = pk.Solver(pk.params_from(case))
    s.set_grid(_dev(torch, case.xyz))
    s.set_state(_dev(torch, case.U0))
    if case.inflow is not None:
        s.set_inflow(_dev(torch, case.inflow))
    return s


def _orc(orc, case):
    P = orc.params_from_case(case)
    return P, orc.metrics(P, case.xyz)


def _char(case):
    return dataclasses.replace(case, characteristic=True)


@pytest.mark.parametrize("shape", [(36, 20, 24), (17, 33, 9)])
def test_char_dudt_parity(pk, torch_cuda, orc, shape):
    """WENO7 in characteristic variables everywhere, distorted periodic grid,
    2% noise (every interface has its own normal and state)."""
    case = _char(workloads.taylor_green(shape=shape, distorted=True, Ma=0.5))
    rng = np.random.default_rng(31)
    case.U0 = case.U0 * (1.0 + 0.02 * rng.standard_normal(case.U0.shape))
    print("case", case.name, shape, flush=True)
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    ref = orc.dudt(P, met, case.U0)
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    l2, linf = rel_errors(got, ref)
    print(f"char dudt {shape}: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_DUDT_L2) and np.all(linf <= TOL_DUDT_INF)
    # and it is not the component-wise result
    comp = orc.dudt(orc.params_from_case(dataclasses.replace(case, characteristic=False)), met, case.U0)
    assert rel_errors(comp, ref)[0].max() > 1e-8


def test_char_three_way_forced_flags(pk, torch_cuda, orc):
    """Three-way hybrid on the oracle's flags: WENO7 and WENO5 interfaces in
    characteristic variables, low-dissipation ones component-wise on the GPU
    (the oracle projects those too: an exact identity)."""
    case = _char(workloads.taylor_green(shape=(40, 24, 20), distorted=True))
    case.scheme, case.lowdiss, case.three_way = "hybrid", "c8", True
    rng = np.random.default_rng(5)
    k, j, i = np.meshgrid(*[np.arange(n) - n / 2 for n in (case.nz, case.ny, case.nx)], indexing="ij")
    ball = np.exp(-(i * i + j * j + k * k) / (2.0 * 4.0 ** 2))
    case.U0 = case.U0 * (1.0 + 0.08 * ball * rng.standard_normal(case.U0.shape))
    P, met = _orc(orc, case)
    _, flags = orc.sensor(P, case.U0)
    frac = [(flags == v).mean() for v in (0, 1, 2)]
    print("flag fractions", frac, flush=True)
    assert min(frac) > 0.01
    s = _solver(pk, torch_cuda, case)
    fl = _dev(torch_cuda, flags)   # the library keeps this pointer: hold the tensor while it is set
    pk.ocfd_set_flags(s.h, fl)
    ref = orc.dudt(P, met, case.U0, flags=flags)
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0), flags=flags)
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    pk.ocfd_set_flags(s.h, None)
    del fl
    assert_within_roundoff(got, ref, ref_pert, what="char three-way forced flags")


@pytest.mark.parametrize("name", ["ramp", "box"])
def test_char_bounded(pk, torch_cuda, orc, name):
    """Bounded directions: the masked WENO5 closures in characteristic
    variables; dU/dt and two Runge-Kutta steps with the faces set after every
    stage."""
    case = workloads.compression_ramp(shape=(40, 24, 8)) if name == "ramp" else workloads.bounded_box(shape=(36, 20, 18))
    case = _char(case)
    print("case", case.name, flush=True)
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    ref = orc.dudt(P, met, case.U0)
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0))
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    assert_within_roundoff(got, ref, ref_pert, what=f"char {case.name} dudt")
    s.advance(6, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 6, case.dt, inflow=case.inflow)
    l2, _ = rel_errors(got, ref)
    print(f"char {case.name} 6 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= TOL_L2)


def test_char_lax_tube_advance(pk, torch_cuda, orc):
    """Lax tube, 200 nodes: 60 substeps through the shock in characteristic
    variables against the oracle."""
    case = _char(workloads.lax(200))
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    s.advance(60, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 60, case.dt)
    l2, linf = rel_errors(got, ref)
    print(f"char lax 60 substeps: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_L2)


def test_char_mixed_precision_drift(pk, torch_cuda, orc):
    """FP32 projection and reconstruction: the Lax tube after 60 substeps
    within 1e-5 of the FP64 oracle."""
    case = _char(workloads.lax(200))
    case.precision = "mixed"
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    s.advance(60, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 60, case.dt)
    l2, _ = rel_errors(got, ref)
    print(f"char lax mixed 60 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= 1e-5)
