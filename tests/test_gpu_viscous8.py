"""Parity of the HIP library's eighth-order central viscous terms (Sec. 2.3)
with the CPU oracle: the viscous part and the whole right-hand side on a
distorted periodic grid (WENO7 sweeps, which read the neighbouring viscous
fluxes from memory, and the hybrid, which stages them in LDS), the bounded
ramp and box (the closure ladder), and Runge-Kutta steps."""
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


@pytest.mark.parametrize("scheme", ["weno7", "hybrid"])
@pytest.mark.parametrize("parts", [8, 15])
def test_viscous8_dudt_parity(pk, torch_cuda, orc, scheme, parts):
    case = dataclasses.replace(workloads.taylor_green(shape=(36, 20, 24), distorted=True), viscous=8, scheme=scheme)
    rng = np.random.default_rng(41)
    case.U0 = case.U0 * (1.0 + 0.02 * rng.standard_normal(case.U0.shape))
    print("case", case.name, scheme, parts, flush=True)
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    ref = orc.dudt(P, met, case.U0, parts=parts)
    got = s.dudt(_dev(torch_cuda, case.U0), parts).cpu().numpy()
    l2, linf = rel_errors(got, ref)
    print(f"viscous8 dudt {scheme} parts {parts}: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_DUDT_L2) and np.all(linf <= TOL_DUDT_INF)
    # and it is not the sixth-order result
    ref6 = orc.dudt(orc.params_from_case(dataclasses.replace(case, viscous=6)), met, case.U0, parts=parts)
    assert rel_errors(ref6, ref)[0][1:4].max() > 1e-9


@pytest.mark.parametrize("name", ["ramp", "box"])
def test_viscous8_bounded(pk, torch_cuda, orc, name):
    case = workloads.compression_ramp(shape=(40, 24, 8)) if name == "ramp" else workloads.bounded_box(shape=(36, 20, 18))
    case = dataclasses.replace(case, viscous=8)
    print("case", case.name, flush=True)
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    ref = orc.dudt(P, met, case.U0)
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0))
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    assert_within_roundoff(got, ref, ref_pert, what=f"viscous8 {case.name} dudt")
    s.advance(6, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 6, case.dt, inflow=case.inflow)
    l2, _ = rel_errors(got, ref)
    print(f"viscous8 {case.name} 6 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= TOL_L2)


def test_viscous8_mixed_drift(pk, torch_cuda, orc):
    """FP32 reconstruction (viscous fluxes staged in LDS) with eighth-order
    viscous terms: 30 substeps of the Taylor-Green vortex within 1e-5 of the
    FP64 oracle."""
    case = dataclasses.replace(workloads.taylor_green(shape=(32, 24, 20), distorted=True), viscous=8,
                               precision="mixed")
    s = _solver(pk, torch_cuda, case)
    P, met = _orc(orc, case)
    s.advance(30, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 30, case.dt)
    l2, _ = rel_errors(got, ref)
    print(f"viscous8 mixed 30 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= 1e-5)
