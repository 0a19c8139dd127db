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


def test_char_learned_sensor_hybrid(pk, torch_cuda, orc):
    """The learned sensor's flags driving the characteristic reconstruction:
    developed isotropic turbulence, hybrid C8 with WENO7 where the network's
    probability reaches the threshold.  The threshold sits in the widest gap of
    the oracle's probabilities; the GPU's flags (bf16 operands, FP32 sums) may
    still differ at an interface whose probability is at the threshold, and the
    nodes next to such an interface are left out of the dU/dt comparison."""
    from oracle import mlp
    case = workloads.isotropic_turbulence(24, seed=22093)
    case.scheme, case.lowdiss = "hybrid", "c8"
    P0 = orc.params_from_case(case)
    met = orc.metrics(P0, case.xyz)
    case.U0, _, _ = orc.advance(P0, met, case.U0, 30, case.dt)
    case = _char(case)
    case.sensor = "learned"
    theta = mlp.init_params(5)
    theta[mlp.NPARAM - 33:mlp.NPARAM - 1] *= 300.0
    theta32 = theta.astype(np.float32).astype(np.float64)
    F = mlp.node_features(case.gamma, case.h, met, case.U0).astype(np.float32).astype(np.float64)
    nodes = np.arange(case.N)
    p = np.stack([mlp.forward(theta32, mlp.interface_inputs(F, d, nodes), round_bf16=True)[0] for d in range(3)])
    mid = np.sort(p[(p > 0.1) & (p < 0.9)])
    g = int(np.argmax(np.diff(mid)))
    tau = 0.5 * (mid[g] + mid[g + 1])
    flags = (p >= tau).astype(np.uint8).reshape((3,) + case.U0.shape[1:])
    frac = flags.reshape(3, -1).mean(axis=1)
    print(f"tau {tau:.6f} in a gap of {mid[g + 1] - mid[g]:.2e}; WENO fractions {frac}", flush=True)
    assert np.all(frac > 0.01) and np.all(frac < 0.99)

    s = _solver(pk, torch_cuda, case)
    pk.ocfd_sensor_set_params(s.h, theta)
    pk.ocfd_sensor_set_threshold(s.h, tau)
    fl = torch_cuda.zeros((3,) + case.U0.shape[1:], dtype=torch_cuda.uint8, device="cuda")
    pk.ocfd_sensor_flags(s.h, _dev(torch_cuda, case.U0), pk.OCFD_SENSOR_LEARNED, fl)
    bad = fl.cpu().numpy() != flags
    print("flag disagreements", bad.sum(), flush=True)
    assert bad.sum() <= 1e-4 * case.N + 2
    assert np.all(np.abs(p.reshape(bad.shape)[bad] - tau) < 1e-3)
    # nodes whose stencil reads a disagreeing interface (either side, each direction)
    near = np.zeros(case.U0.shape[1:], bool)
    for d in range(3):
        ax = 2 - d
        for sh in (-1, 0, 1):
            near |= np.roll(bad[d], sh, axis=ax)
    keep = ~near.reshape(-1)

    P = orc.params_from_case(case)
    ref = orc.dudt(P, met, case.U0, flags=flags)
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0), flags=flags)
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    sel = lambda a: a.reshape(5, -1)[:, keep]
    assert_within_roundoff(sel(got), sel(ref), sel(ref_pert), what="char learned hybrid")
    # and the projection mattered where WENO7 was chosen
    comp = orc.dudt(orc.params_from_case(dataclasses.replace(case, characteristic=False)), met, case.U0,
                    flags=flags)
    assert rel_errors(comp, ref)[0].max() > 1e-8
