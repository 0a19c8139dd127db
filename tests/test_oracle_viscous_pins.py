"""Pins of the oracle's viscous terms beyond the unit-temperature cases: the
Sutherland viscosity law (eq 15) against a published table of air viscosity,
and the stress-work part u_j tau_ij of the energy flux (eq 12) against a
closed form worked by hand from eq 9-13; and of the Adam update of the
learned sensor's training against closed forms of its definition."""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _shear_case(d, T, Tref=288.15, n=64, a=1, b=2):
    """u = d sin(a x + b y), v = w = 0, rho = 1 and uniform temperature T
    (p = rho T / (gamma Ma^2)), on the distorted periodic grid."""
    case = workloads.taylor_green(n, distorted=True)
    x, y, z = case.xyz
    one = np.ones_like(x)
    p = one * T / (case.gamma * case.Ma ** 2)
    case.U0 = workloads.conserved(case.gamma, one, d * np.sin(a * x + b * y), 0 * x, 0 * x, p)
    case.Re = 50.0
    case.Tref = Tref
    return case


def _viscous_rhs(orc, case):
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    return orc.dudt(P, met, case.U0, parts=orc.PART_VISC)


# For u = d sin(s), s = a x + b y, and uniform mu (uniform T), eq 13 gives
#   tau_xx = (4a/3) K d cos s, tau_xy = b K d cos s, tau_yy = tau_zz = -(2a/3) K d cos s,
# K = mu / Re, and eq 9-12 give the viscous parts of dU/dt:
#   d(rho u)/dt = -(4a^2/3 + b^2) K d sin s,   d(rho v)/dt = -(a b / 3) K d sin s,
#   dE/dt = d(u tau_xx)/dx + d(u tau_xy)/dy = (4a^2/3 + b^2) K d^2 cos 2s.
# With a = 1, b = 2 the energy row 16/3 differs from what a stress work
# u_i sum_j tau_ij (10/3) or a missing one (0) would give.
def _expected(case, d, K, a=1, b=2):
    x, y, _ = case.xyz
    s = a * x + b * y
    c = 4.0 * a * a / 3.0 + b * b
    return -c * K * d * np.sin(s), -(a * b / 3.0) * K * d * np.sin(s), c * K * d * d * np.cos(2.0 * s)


@pytest.mark.parametrize("T", [1.0, 2.84])
def test_stress_work_energy_row(orc, T):
    d = 0.2
    case = _shear_case(d, T)
    L = _viscous_rhs(orc, case)
    # K from the x-momentum row (at T = 1, mu = 1 whatever the Sutherland constant)
    eu, _, _ = _expected(case, d, 1.0)
    K = float(np.sum(L[1] * eu) / np.sum(eu * eu))
    if T == 1.0:
        assert abs(K - 1.0 / case.Re) < 1e-5 / case.Re
    exp_u, exp_v, exp_E = _expected(case, d, K)
    sc = (16.0 / 3.0) * K * d          # amplitude of the momentum rows; the energy row's is sc * d
    assert np.abs(L[1] - exp_u).max() < 1e-4 * sc
    assert np.abs(L[2] - exp_v).max() < 1e-4 * sc
    assert np.abs(L[3]).max() < 1e-4 * sc
    assert np.abs(L[4] - exp_E).max() < 1e-4 * sc * d, np.abs(L[4] - exp_E).max() / (sc * d)
    assert np.abs(L[0]).max() == 0.0


def test_sutherland_against_air_table(orc):
    """mu(T)/mu(Tref) of the oracle (nondimensional T = T_K / Tref, eq 15 with
    S = 110.4 K / Tref) against the tabulated air viscosity, Tref = 300 K:
    within Sutherland's stated 2% inside its range, 3% at 100 K."""
    tab = json.load(open(os.path.join(GOLDEN, "air_viscosity.json")))
    T_K = tab["T_kelvin"]
    mu = dict(zip(T_K, tab["mu_1e7_Ns_per_m2"]))
    d = 1e-3
    lo, hi = tab["sutherland_stated_range_kelvin"]
    for TK in T_K:
        case = _shear_case(d, TK / 300.0, Tref=300.0)
        L = _viscous_rhs(orc, case)
        eu, _, _ = _expected(case, d, 1.0)
        K = float(np.sum(L[1] * eu) / np.sum(eu * eu))
        ratio = K * case.Re
        want = mu[TK] / mu[300.0]
        tol = tab["sutherland_stated_accuracy"] if lo <= TK <= hi else 0.03
        assert abs(ratio / want - 1.0) <= tol, (TK, ratio, want)


def test_sutherland_at_the_ramp_temperatures(orc):
    """The ramp's wall (307 K) over its free stream (108.1 K): the oracle's
    mu(2.84) with Tref 108.1 K against the table interpolated in log-log
    (power law between neighbouring entries), within 3%."""
    tab = json.load(open(os.path.join(GOLDEN, "air_viscosity.json")))
    T = np.array(tab["T_kelvin"])
    m = np.array(tab["mu_1e7_Ns_per_m2"])

    def interp(tk):
        i = int(np.searchsorted(T, tk)) - 1
        e = math.log(m[i + 1] / m[i]) / math.log(T[i + 1] / T[i])
        return m[i] * (tk / T[i]) ** e
    d = 1e-3
    case = _shear_case(d, 307.0 / 108.1, Tref=108.1)
    L = _viscous_rhs(orc, case)
    eu, _, _ = _expected(case, d, 1.0)
    ratio = float(np.sum(L[1] * eu) / np.sum(eu * eu)) * case.Re
    want = interp(307.0) / interp(108.1)
    assert abs(ratio / want - 1.0) <= 0.03, (ratio, want)


# ---------------------------------------------------------------- Adam

def test_adam_first_step_is_signed_learning_rate():
    """After one step from zero moments both bias corrections are exact:
    mhat = g, vhat = g^2, so theta moves by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    g = rng.normal(size=100) * 10.0 ** rng.uniform(-3, 3, 100)
    th, m, v = mlp.adam_step(np.zeros(100), np.zeros(100), np.zeros(100), g, 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-15)


def test_adam_alternating_gradient_closed_form():
    """Gradients g then -g: m2 = -(1 - b1)^2 g ... so mhat2 = -(1 - b1)/(1 + b1) g,
    and v2 = (1 - b2)(1 + b2) g^2 ... so vhat2 = g^2: the second step is
    +lr (1 - b1)/(1 + b1) sign(g) (for |g| >> eps)."""
    g = np.array([2.0, -0.5, 1e3])
    lr = 0.1
    th, m, v = mlp.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr)
    th2, m2, v2 = mlp.adam_step(th, m, v, -g, 2, lr)
    step2 = th2 - th
    assert np.allclose(step2, lr * (0.1 / 1.9) * np.sign(g), rtol=1e-9)
    assert np.allclose(m2 / (1 - 0.81), -(0.1 / 1.9) * g, rtol=1e-12)
    assert np.allclose(v2 / (1 - 0.999 ** 2), g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_at_the_learning_rate():
    """With a constant gradient every bias-corrected moment is exact at every
    step, so each of t steps moves -lr g / (|g| + eps)."""
    g = np.array([3.0, -1e-2])
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 11):
        th, m, v = mlp.adam_step(th, m, v, g, t, 0.05)
    assert np.allclose(th, -10 * 0.05 * g / (np.abs(g) + 1e-8), rtol=1e-12)
