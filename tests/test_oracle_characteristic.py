"""Pins of the oracle's reconstruction in characteristic variables (Sec. 2.2.2,
eq 31-40): the eigenvector matrices against the flux Jacobian (an
independent complex-step derivative of the Euler flux), the frame of eq 39-40
worked by hand, the exact identity for linear stencils, and what the option is
for, fewer spurious oscillations, against exact Riemann solutions."""
import dataclasses

import numpy as np
import pytest

import workloads
from oracle import exact

G = 1.4


def _state(rng):
    rho = rng.uniform(0.3, 3.0)
    vel = rng.normal(size=3) * 1.5
    p = rng.uniform(0.2, 4.0)
    U = np.array([rho, *(rho * vel), p / (G - 1.0) + 0.5 * rho * vel @ vel])
    return U, rho, vel, p


def _normals(rng, k):
    out = [np.array(v, float) for v in ((1, 0, 0), (0, 1, 0), (0, 0, 1), (0, -1, 0), (0.6, 0.0, -0.8),
                                        (0.0, 0.6, 0.8), (0.0, 0.8, 0.6), (1, 1, 1), (-1, 2, -2))]
    out += list(rng.normal(size=(k, 3)))
    return [n / np.linalg.norm(n) for n in out]


def _euler_flux(U, n):
    """Inviscid flux of the conserved variables U through the unit normal n
    (mass, momentum, total energy; eq 1-8 with the metrics replaced by n)."""
    rho = U[0]
    vel = U[1:4] / rho
    p = (G - 1.0) * (U[4] - 0.5 * rho * (vel @ vel))
    un = vel @ n
    return np.array([rho * un, *(U[1:4] * un + p * n), (U[4] + p) * un])


def _jacobian(U, n):
    """dF/dU by the complex step: exact to rounding."""
    A = np.zeros((5, 5))
    hs = 1e-30
    for i in range(5):
        Uc = U.astype(complex)
        Uc[i] += 1j * hs
        A[:, i] = _euler_flux(Uc, n.astype(complex)).imag / hs
    return A


def _params(orc):
    case = workloads.sod(8, width=2)
    return orc.params_from_case(case)


def test_char_matrices_are_inverse(orc):
    P = _params(orc)
    rng = np.random.default_rng(3101)
    for n in _normals(rng, 20):
        U, *_ = _state(rng)
        S, Si = orc.char_matrices(P, U, n)
        assert np.abs(S @ Si - np.eye(5)).max() < 1e-13
        assert np.abs(Si @ S - np.eye(5)).max() < 1e-13


def test_char_matrices_diagonalise_the_flux_jacobian(orc):
    """Rows of S are left eigenvectors in the order of eq 33: u_n (three
    times), u_n - c, u_n + c."""
    P = _params(orc)
    rng = np.random.default_rng(3102)
    for n in _normals(rng, 20):
        U, rho, vel, p = _state(rng)
        S, Si = orc.char_matrices(P, U, n)
        c = np.sqrt(G * p / rho)
        un = vel @ n
        D = S @ _jacobian(U, n) @ Si
        lam = np.array([un, un, un, un - c, un + c])
        scale = np.abs(vel).max() + c
        assert np.abs(D - np.diag(lam)).max() < 1e-12 * scale


def test_char_frame_eq39(orc):
    """Rows 2 and 3 of S hold l and m: orthonormal, m = n x l, and the branch
    of eq 39 worked by hand for the axis normals."""
    P = _params(orc)
    rng = np.random.default_rng(3103)
    U, *_ = _state(rng)
    hand = {(0, 0, 1): ((-1, 0, 0), (0, -1, 0)),    # |n3| > |n2|: (-n3, 0, n1)
            (1, 0, 0): ((0, 1, 0), (0, 0, 1)),      # |n3| <= |n2|: (-n2, n1, 0)/|(n1, n2)|
            (0, 1, 0): ((-1, 0, 0), (0, 0, 1))}
    for n, (l_ex, m_ex) in hand.items():
        S, _ = orc.char_matrices(P, U, np.array(n, float))
        assert np.array_equal(S[1, 1:4], np.array(l_ex, float))
        assert np.array_equal(S[2, 1:4], np.array(m_ex, float))
    for n in _normals(rng, 20):
        S, _ = orc.char_matrices(P, U, n)
        l, m = S[1, 1:4], S[2, 1:4]
        F = np.stack([l, m, n])
        assert np.abs(F @ F.T - np.eye(3)).max() < 1e-14
        assert np.abs(np.cross(n, l) - m).max() < 1e-15


def _smooth_case(lowdiss):
    case = workloads.taylor_green(12, distorted=True, Ma=0.5)
    return dataclasses.replace(case, scheme="hybrid", lowdiss=lowdiss)


@pytest.mark.parametrize("lowdiss", ["ud7", "c8"])
def test_char_is_exact_for_linear_stencils(orc, lowdiss):
    """S^-1 L(S f) = L(f) for a linear stencil L and a fixed S: with every
    interface on the low-dissipation stencil the characteristic and the
    component-wise right-hand sides agree to rounding (distorted grid, so the
    interface normals vary)."""
    case = _smooth_case(lowdiss)
    flags = np.zeros((3, case.nz, case.ny, case.nx), np.uint8)
    P0 = orc.params_from_case(case)
    P1 = orc.params_from_case(dataclasses.replace(case, characteristic=True))
    met = orc.metrics(P0, case.xyz)
    a = orc.dudt(P0, met, case.U0, flags)
    b = orc.dudt(P1, met, case.U0, flags)
    for q in range(5):
        assert np.abs(a[q] - b[q]).max() <= 1e-11 * np.abs(a).max()
    # WENO7 everywhere: the projection changes the nonlinear weights
    flags[:] = 1
    a = orc.dudt(P0, met, case.U0, flags)
    b = orc.dudt(P1, met, case.U0, flags)
    assert np.abs(a - b).max() > 1e-9 * np.abs(a).max()


def _run(orc, case, char):
    case = dataclasses.replace(case, characteristic=char)
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    U, _, _ = orc.advance(P, met, case.U0, case.nsteps, case.dt)
    return case, U


def test_char_removes_the_lax_overshoot(orc):
    """Lax tube, 200 nodes, t = 0.13: the component-wise WENO7 density
    overshoots the exact post-shock plateau (1.3041) by several percent; the
    characteristic one stays within 1% of it and is closer to the exact
    solution in L1."""
    case = workloads.lax(200)
    t = case.nsteps // 3 * case.dt
    x = case.xyz[0][0, 0]
    win = x >= 1.0
    rho_ex, _, _ = exact.riemann_sample((0.445, 0.698, 3.528), (0.5, 0.0, 0.571), (x[win] - 1.5) / t)
    plateau = rho_ex.max()
    assert plateau == pytest.approx(1.30408, abs=1e-4)
    res = {}
    for char in (False, True):
        _, U = _run(orc, case, char)
        rho = U[0][0, 0][win]
        res[char] = (rho.max() - plateau, np.mean(np.abs(rho - rho_ex)))
    assert res[False][0] > 0.03
    assert res[True][0] < 0.01
    assert res[True][1] < res[False][1]


def test_char_sod_total_variation(orc):
    """Sod two-tube box, 200 nodes, t = 0.2: the exact density is monotone in
    each tube (total variation 4 x 0.875 / 2 = 1.75 over the box); the
    characteristic reconstruction's excess variation is under 3%, below the
    component-wise one's."""
    case = workloads.sod(200, width=2)
    tv = {}
    for char in (False, True):
        _, U = _run(orc, case, char)
        rho = U[0][0, 0]
        tv[char] = np.abs(np.diff(np.append(rho, rho[0]))).sum()
    assert tv[True] < 1.03 * 1.75
    assert tv[True] < tv[False]
