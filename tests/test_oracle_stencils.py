"""Pins of the oracle's interface reconstructions and Steger-Warming split.

Each check compares the oracle with something fixed independently of it:
the WENO coefficients derived here symbolically from their definition, the
coefficients the paper prints (eq 41), polynomial exactness, and the flux
Jacobian of eq 6 split by a numerical eigen-decomposition.
"""
import functools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@functools.lru_cache(maxsize=None)
def _weno_from_definition(k):
    """Candidate values at x = 1/2 and smoothness indicators of the k-point
    candidates, derived from the definition: the degree k-1 polynomial whose
    cell averages over cells of unit width match the data; the indicator is
    sum_{l=1}^{k-1} integral over the central cell of (d^l p / dx^l)^2."""
    sp = pytest.importorskip("sympy")
    x = sp.symbols("x")
    fs = sp.symbols(f"f0:{2 * k - 1}")
    out = []
    for r in range(k):
        cells = list(range(-k + 1 + r, r + 1))
        cs = sp.symbols(f"c0:{k}")
        p = sum(cs[a] * x ** a for a in range(k))
        half = sp.Rational(1, 2)
        eqs = [sp.integrate(p, (x, c - half, c + half)) - fs[c + k - 1] for c in cells]
        P = p.subs(sp.solve(eqs, cs))
        q = sp.lambdify(fs, P.subs(x, half))
        beta = sp.lambdify(fs, sum(sp.integrate(sp.diff(P, x, l) ** 2, (x, -half, half)) for l in range(1, k)))
        out.append((q, beta))
    return out


@functools.lru_cache(maxsize=None)
def _linear_weights(k):
    """Linear weights that make the convex combination of the k candidates
    equal the (2k-1)-point upwind value: solved from the candidate values."""
    cands = _weno_from_definition(k)
    n = 2 * k - 1
    M = np.zeros((n, k))
    for r, (q, _) in enumerate(cands):
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            M[i, r] = q(*e)
    # The combination must reproduce the upwind polynomial value of degree 2k-2:
    # the cell-average reconstruction of all n cells evaluated at x = 1/2.
    sp = pytest.importorskip("sympy")
    x = sp.symbols("x")
    fs = sp.symbols(f"f0:{n}")
    cs = sp.symbols(f"c0:{n}")
    p = sum(cs[a] * x ** a for a in range(n))
    half = sp.Rational(1, 2)
    eqs = [sp.integrate(p, (x, c - half, c + half)) - fs[c + k - 1] for c in range(-k + 1, k)]
    P = p.subs(sp.solve(eqs, cs))
    target = np.array([float(P.subs(x, half).coeff(f)) for f in fs])
    d, *_ = np.linalg.lstsq(M, target, rcond=None)
    assert np.allclose(M @ d, target, atol=1e-14)
    return d


def _weno_reference(f, k, eps):
    cands = _weno_from_definition(k)
    d = _linear_weights(k)
    q = np.array([c[0](*f) for c in cands])
    b = np.array([c[1](*f) for c in cands])
    a = d / (eps + b) ** 2
    return float(np.sum(a / a.sum() * q))


def test_weno7_matches_definition(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        f = rng.normal(size=7) * rng.choice([1e-3, 1.0, 30.0])
        ref = _weno_reference(f, 4, 1e-6)
        assert orc.weno7(f, 1e-6) == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_weno5_matches_definition(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        f = rng.normal(size=5) * rng.choice([1e-3, 1.0, 30.0])
        ref = _weno_reference(f, 3, 1e-6)
        assert orc.weno5(f, 1e-6) == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_weno_linear_weights_are_the_textbook_ones():
    assert np.allclose(_linear_weights(4), np.array([1, 12, 18, 4]) / 35.0, atol=1e-14)
    assert np.allclose(_linear_weights(3), np.array([1, 6, 3]) / 10.0, atol=1e-14)


def test_weno7_linear_limit_is_eq41(orc):
    """With a huge epsilon the nonlinear weights become the linear ones, and the
    seventh-order WENO value must then equal the printed upwind scheme eq 41."""
    g = json.load(open(os.path.join(GOLDEN, "eq41_ud7.json")))
    coef = np.array(g["numerators"]) / g["denominator"]
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = rng.normal(size=7)
        assert orc.weno7(f, 1e30) == pytest.approx(float(coef @ f), rel=1e-13, abs=1e-15)
        assert orc.ud7(f) == pytest.approx(float(coef @ f), rel=1e-14, abs=1e-15)


def _poly_samples(deg, rng, n=16):
    c = rng.normal(size=deg + 1)
    j = np.arange(-8, n)
    return c, j, np.polyval(c, j.astype(float))


@pytest.mark.parametrize("deg", range(0, 8))
def test_ud7_difference_is_exact_derivative(orc, deg):
    """(f_{j+1/2} - f_{j-1/2}) of eq 41 is a seventh-order derivative: exact for
    polynomials of degree <= 7 sampled at the nodes."""
    rng = np.random.default_rng(10 + deg)
    c, j, f = _poly_samples(deg, rng)
    i0 = 8  # node j = 0
    right = orc.ud7(f[i0 - 3:i0 + 4])
    left = orc.ud7(f[i0 - 4:i0 + 3])
    exact = np.polyval(np.polyder(c), 0.0) if deg > 0 else 0.0
    assert right - left == pytest.approx(exact, abs=1e-11 * max(1.0, np.abs(c).max()))


@pytest.mark.parametrize("deg", range(0, 9))
def test_c8_difference_is_eighth_order_central(orc, deg):
    rng = np.random.default_rng(30 + deg)
    c, j, f = _poly_samples(deg, rng)
    i0 = 8
    right = orc.c8(f[i0 - 3:i0 + 5])
    left = orc.c8(f[i0 - 4:i0 + 4])
    exact = np.polyval(np.polyder(c), 0.0) if deg > 0 else 0.0
    assert right - left == pytest.approx(exact, abs=1e-10 * max(1.0, np.abs(c).max()))


def test_ud7_minus_c8_is_seventh_difference(orc):
    """UD7 differs from C8 by the eighth-point difference / 280 (upwind dissipation)."""
    rng = np.random.default_rng(4)
    binom = np.array([-1, 7, -21, 35, -35, 21, -7, 1], dtype=float)
    for _ in range(20):
        g = rng.normal(size=8)
        assert orc.ud7(g[:7]) - orc.c8(g) == pytest.approx(float(binom @ g) / 280.0, abs=1e-14)


def test_weno5_masking_reduces_to_substencils(orc):
    rng = np.random.default_rng(5)
    f = rng.normal(size=5)
    q = [(2 * f[0] - 7 * f[1] + 11 * f[2]) / 6, (-f[1] + 5 * f[2] + 2 * f[3]) / 6, (2 * f[2] + 5 * f[3] - f[4]) / 6]
    for r in range(3):
        valid = [0, 0, 0]
        valid[r] = 1
        assert orc.weno5(f, 1e-6, valid) == pytest.approx(q[r], rel=1e-15, abs=1e-15)


def _flux_eq6(gamma, U, alpha):
    """Inviscid flux of eq 6 (with xi_t = 0) for conserved U and alpha = metric row / J."""
    rho, mu, mv, mw, E = U
    u, v, w = mu / rho, mv / rho, mw / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    V = alpha[0] * u + alpha[1] * v + alpha[2] * w
    return np.array([rho * V, mu * V + alpha[0] * p, mv * V + alpha[1] * p, mw * V + alpha[2] * p, (E + p) * V])


def _random_state(rng, gamma=1.4):
    rho = rng.uniform(0.2, 3.0)
    vel = rng.normal(size=3) * rng.choice([0.1, 1.0, 4.0])
    p = rng.uniform(0.1, 5.0)
    alpha = rng.normal(size=3) * rng.uniform(0.1, 3.0)
    return rho, vel, p, alpha


def test_sw_split_sums_to_flux(orc):
    """f+ + f- = F of eq 6 for any state and metric (eq 30)."""
    P = orc.Params()
    P.gamma = 1.4
    rng = np.random.default_rng(6)
    for _ in range(2000):
        rho, vel, p, alpha = _random_state(rng)
        fp, fm = orc.sw_split(P, rho, *vel, p, alpha)
        U = np.array([rho, rho * vel[0], rho * vel[1], rho * vel[2], p / 0.4 + 0.5 * rho * vel @ vel])
        F = _flux_eq6(1.4, U, alpha)
        scale = np.abs(F).max() + np.abs(fp).max()
        assert np.abs(fp + fm - F).max() <= 1e-14 * scale


def test_sw_split_is_positive_part_of_jacobian(orc):
    """Steger-Warming: f+ = A+ U with A+ = R max(Lambda, 0) R^-1 of the flux
    Jacobian A = dF/dU (eq 6 is homogeneous of degree one, so F = A U).  The
    Jacobian is taken by complex-step differentiation of eq 6 and split by a
    numerical eigen-decomposition, independently of eq 23."""
    P = orc.Params()
    P.gamma = 1.4
    rng = np.random.default_rng(7)
    for _ in range(200):
        rho, vel, p, alpha = _random_state(rng)
        U = np.array([rho, rho * vel[0], rho * vel[1], rho * vel[2], p / 0.4 + 0.5 * rho * vel @ vel])
        A = np.zeros((5, 5))
        for j in range(5):
            dU = np.zeros(5, dtype=complex)
            dU[j] = 1e-30j
            A[:, j] = np.imag(_flux_eq6(1.4, U.astype(complex) + dU, alpha.astype(complex))) / 1e-30
        lam, R = np.linalg.eig(A)
        lam = lam.real
        Rinv = np.linalg.inv(R)
        Ap = (R @ np.diag(np.maximum(lam, 0.0)) @ Rinv).real
        Am = (R @ np.diag(np.minimum(lam, 0.0)) @ Rinv).real
        fp, fm = orc.sw_split(P, rho, *vel, p, alpha)
        scale = np.abs(_flux_eq6(1.4, U, alpha)).max() + np.abs(Ap @ U).max()
        assert np.abs(fp - Ap @ U).max() <= 1e-9 * scale
        assert np.abs(fm - Am @ U).max() <= 1e-9 * scale


def test_sw_split_supersonic(orc):
    P = orc.Params()
    P.gamma = 1.4
    alpha = np.array([0.6, 0.8, 0.0])  # sigma = 1
    rho, p = 1.0, 1.0 / 1.4              # c = 1
    fp, fm = orc.sw_split(P, rho, 3.0, 0.1, -0.2, p, alpha)
    assert np.all(fm == 0.0)
    fp, fm = orc.sw_split(P, rho, -3.0, 0.1, -0.2, p, alpha)
    assert np.all(fp == 0.0)
