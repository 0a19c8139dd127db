"""Pins of the oracle's characteristic nonreflecting faces (the paper imposes
nonreflecting conditions at the exit and the upper boundary of the ramp,
Sec. 6.1, without formulas; the reading is Thompson's characteristic
boundary condition with the local one-dimensional relations of Poinsot &
Lele, incoming wave amplitudes set to zero).

* A plane acoustic pulse leaving the grid through such a face leaves almost
  nothing behind: the reflected pressure is below 5e-4 of the pulse and falls
  with grid refinement (the one-sided differences are second order), while
  the zeroth-order extrapolation face reflects several percent.
* A supersonic exit takes every wave from inside: the normal part equals the
  primitive-variable Euler equations with the one-sided derivatives; a
  supersonic entrance takes none (zero normal part).
* A uniform stream on a distorted grid stays steady at the faces (to rounding).
"""
import numpy as np
import pytest

import workloads

AMP = 1e-5   # small enough that the pulse's own nonlinearity (~AMP) stays below the measured reflections


def _reflection(orc, n, bc, direction=1, u0=0.3):
    c = workloads.acoustic_pulse(n=n, width=1, bc=bc, amplitude=AMP, u0=u0, direction=direction)
    P = orc.params_from_case(c, nthreads=1)
    met = orc.metrics(P, c.xyz)
    speed = 1.0 + u0 if direction > 0 else 1.0 - u0
    t_end = (0.5 + 5 * 0.05) / speed          # the pulse is five widths beyond the face
    steps = int(np.ceil(t_end / c.dt))
    U, _, _ = orc.advance(P, met, c.U0, 3 * steps, c.dt)
    rho = U[0]
    u = U[1] / rho
    p = (c.gamma - 1.0) * (U[4] - 0.5 * rho * u * u)
    p0 = 1.0 / c.gamma
    return np.abs(p - p0).max() / (AMP * p0)


@pytest.mark.parametrize("direction", [1, -1])
def test_acoustic_pulse_leaves_without_reflection(orc, direction):
    r_nrbc = _reflection(orc, 201, 4, direction)
    r_extrap = _reflection(orc, 201, 2, direction)
    print(f"direction {direction}: reflected pressure / pulse: nonreflecting {r_nrbc:.2e}, "
          f"extrapolation {r_extrap:.2e}")
    assert r_nrbc < 5e-4
    assert r_extrap > 0.03


def test_reflection_falls_with_refinement(orc):
    r101 = _reflection(orc, 101, 4)
    r201 = _reflection(orc, 201, 4)
    print(f"reflection n=101 {r101:.2e}, n=201 {r201:.2e}")
    assert r201 < r101 / 3.0


def _one_sided(q0, q1, q2, h, side):
    d = (-3.0 * q0 + 4.0 * q1 - q2) / (2.0 * h)
    return -d if side else d


@pytest.mark.parametrize("side", [0, 1])
def test_supersonic_faces(orc, side):
    """u0 = 1.5 > c: at the exit (upper face) every wave leaves, so the
    normal part is the primitive Euler equations along x; at the entrance
    (lower face) every wave enters and the normal part is zero."""
    c = workloads.acoustic_pulse(n=41, bc=4, amplitude=0.05, u0=1.5, x0=0.5 if side == 0 else 0.98, sigma=0.08)
    P = orc.params_from_case(c, nthreads=1)
    met = orc.metrics(P, c.xyz)
    i = c.nx - 1 if side else 0
    got = orc.nrbc_normal(P, met, c.U0, (i, 1, 2), 0, side)
    if side == 0:
        # the uniform grid's metric derivatives are rounding noise
        assert np.abs(got).max() <= 1e-12 * np.abs(c.U0).max() / c.h[0]
        return
    g = c.gamma
    U = c.U0[:, 2, 1, :]
    rho = U[0]
    u = U[1] / rho
    p = (g - 1.0) * (U[4] - 0.5 * rho * u * u)
    h = c.h[0]
    dr = _one_sided(rho[i], rho[i - 1], rho[i - 2], h, 1)
    du = _one_sided(u[i], u[i - 1], u[i - 2], h, 1)
    dp = _one_sided(p[i], p[i - 1], p[i - 2], h, 1)
    r, v, pr = rho[i], u[i], p[i]
    rho_t = -(v * dr + r * du)
    u_t = -(v * du + dp / r)
    p_t = -(v * dp + g * pr * du)
    ref = np.array([rho_t, v * rho_t + r * u_t, 0.0, 0.0, p_t / (g - 1.0) + 0.5 * v * v * rho_t + r * v * u_t])
    assert np.abs(got[0]) > 0.1
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_uniform_stream_steady_at_faces(orc):
    """Uniform flow on a distorted grid bounded in xi with nonreflecting faces:
    every wave amplitude vanishes, and the metric-derivative part balances the
    transverse fluxes' metric derivatives, so the faces' dU/dt is of the order
    of the interior's free-stream residual (without that part it is about a
    hundred times larger)."""
    c = workloads.uniform_flow(n=(24, 12, 10), viscous=0)
    c.periodic = (0, 1, 1)
    c.bc = (4, 4, 0, 0, 0, 0)
    P = orc.params_from_case(c, nthreads=1)
    met = orc.metrics(P, c.xyz)
    L = orc.dudt(P, met, c.U0)
    face = max(np.abs(L[:, :, :, 0]).max(), np.abs(L[:, :, :, -1]).max())
    inner = np.abs(L[:, :, :, 4:-4]).max()
    print("face |dU/dt|", face, "interior", inner)
    assert face <= 10.0 * inner
