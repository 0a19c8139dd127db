"""Characteristic nonreflecting faces on the GPU against the oracle: a plane
acoustic pulse in a subsonic stream (the whole field's dU/dt, and the state
after substeps), and the pulse leaving through the face with the reflection
the oracle's pins bound (Sec. 6.1 of the paper names nonreflecting
conditions at the ramp's exit and upper boundary; reading: Thompson's
characteristic condition with the local one-dimensional relations of
Poinsot & Lele, incoming amplitudes zero)."""
import numpy as np
import pytest

import workloads
from helpers import rel_errors, ulp_perturbed, assert_within_roundoff

pytestmark = pytest.mark.gpu


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
    return s


# width 8: the periodic transverse lines take the general path; width 4: the
# short-line wrap; the pulse sits near the upper face so both faces see waves
@pytest.mark.parametrize("width,direction", [(8, 1), (4, -1)])
def test_nrbc_dudt_and_advance_parity(pk, torch_cuda, orc, width, direction):
    case = workloads.acoustic_pulse(n=70, width=width, amplitude=0.02, sigma=0.08,
                                    x0=0.85 if direction > 0 else 0.15, direction=direction)
    print("case", case.name, width, direction, flush=True)
    s = _solver(pk, torch_cuda, case)
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    ref = orc.dudt(P, met, case.U0)
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0))
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy()
    face = got[:, :, :, -1] if direction > 0 else got[:, :, :, 0]
    assert np.abs(face).max() > 1e-3 * np.abs(got).max()     # the face is advanced
    assert_within_roundoff(got, ref, ref_pert, what=f"pulse width {width}")
    s.advance(30, case.dt)
    U = s.state().cpu().numpy()
    Uref, _, _ = orc.advance(P, met, case.U0, 30, case.dt)
    l2, linf = rel_errors(U, Uref)
    print(f"30 substeps: rel L2 {l2}, Linf {linf}", flush=True)
    assert np.all(l2 <= 1e-12) and np.all(linf <= 1e-11)


def test_nrbc_pulse_leaves_without_reflection(pk, torch_cuda):
    """The small pulse of the oracle's pin, run on the GPU until it is five
    widths beyond the face: the pressure left behind is below 5e-4 of it."""
    amp = 1e-5
    case = workloads.acoustic_pulse(n=201, width=8, amplitude=amp)
    s = _solver(pk, torch_cuda, case)
    t_end = (0.5 + 5 * 0.05) / 1.3
    steps = int(np.ceil(t_end / case.dt))
    s.advance(3 * steps, case.dt)
    U = s.state().cpu().numpy()
    rho = U[0]
    u = U[1] / rho
    p = (case.gamma - 1.0) * (U[4] - 0.5 * rho * u * u)
    p0 = 1.0 / case.gamma
    r = np.abs(p - p0).max() / (amp * p0)
    print(f"reflected pressure / pulse {r:.2e}", flush=True)
    assert r < 5e-4
