"""Whole-field pins of the oracle: metrics against the analytic mapping,
geometric conservation, free-stream preservation, discrete conservation,
closed-form viscous operators, the sensor formula, convergence to exact
solutions (isentropic vortex, Sod) and restart/translation invariants."""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(orc, case):
    P = orc.params_from_case(case)
    return P, orc.metrics(P, case.xyz)


# ---------------------------------------------------------------- metrics

def test_metrics_match_analytic_mapping(orc):
    """Discrete conservative metrics vs eq 3 evaluated with the exact
    derivatives of the analytic distorted mapping."""
    n = 32
    case = workloads.taylor_green(n, distorted=True)
    P, met = _setup(orc, case)
    L = case.period
    A = 0.1 * case.h[0]
    ph = workloads.distortion_phases(22092)
    X = np.stack(np.meshgrid(*[np.arange(n) * (L[d] / n) for d in (2, 1, 0)], indexing="ij")[::-1])
    s = [2 * math.pi * X[d] / L[d] for d in range(3)]
    g = np.zeros((3, 3) + X.shape[1:])  # g[c][d] = d x_c / d xi_d
    for c in range(3):
        for d in range(3):
            term = A * (2 * math.pi / L[d]) * np.cos(s[d] + ph[3 * c + d])
            for e in range(3):
                if e != d:
                    term = term * np.sin(s[e] + ph[3 * c + e])
            g[c, d] = (1.0 if c == d else 0.0) + term
    # eq 3 (times 1/J): row r, column c = cofactor of the Jacobian matrix
    cof = np.zeros_like(g)
    for r in range(3):
        for c in range(3):
            r1, r2 = (r + 1) % 3, (r + 2) % 3
            c1, c2 = (c + 1) % 3, (c + 2) % 3
            cof[r, c] = g[c1, r1] * g[c2, r2] - g[c1, r2] * g[c2, r1]
    det = np.linalg.det(np.moveaxis(g, (0, 1), (-2, -1)))
    for r in range(3):
        for c in range(3):
            assert np.abs(met[3 * r + c] - cof[r, c]).max() < 1e-9, (r, c)
    assert np.abs(met[9] - det).max() < 1e-9


def _d8(f, axis, h):
    a = [4 / 5, -1 / 5, 4 / 105, -1 / 280]
    return sum(a[m - 1] * (np.roll(f, -m, axis) - np.roll(f, m, axis)) for m in range(1, 5)) / h


def test_geometric_conservation_law(orc):
    """sum_d D8_d(metric row d / J) = 0 to roundoff on a distorted periodic grid."""
    case = workloads.isentropic_vortex(shape=(24, 20, 16), distorted=True, dt=1e-3)
    P, met = _setup(orc, case)
    axis = {0: 2, 1: 1, 2: 0}  # array axis of direction d
    for c in range(3):
        gcl = sum(_d8(met[3 * d + c], axis[d], case.h[d]) for d in range(3))
        scale = max(np.abs(met[3 * d + c]).max() / case.h[d] for d in range(3))
        assert np.abs(gcl).max() <= 1e-13 * scale


# ------------------------------------------------------------ free stream

def test_free_stream_preservation(orc):
    """Uniform flow on a distorted grid: the viscous residual is exactly zero,
    the central (C8) path is at roundoff, the upwind paths converge to zero
    at high order."""
    res = {}
    for n in (16, 32):
        case = workloads.uniform_flow((n, n, n))
        P, met = _setup(orc, case)
        Lv = orc.dudt(P, met, case.U0, parts=orc.PART_VISC)
        assert np.all(Lv == 0.0)
        scale = np.abs(case.U0).max() * 3.0 / case.h[0]
        jinv = met[9]
        case.scheme = "hybrid"
        flags = np.zeros((3, n, n, n), np.uint8)
        for low in ("c8", "ud7"):
            case.lowdiss = low
            Pl = orc.params_from_case(case)
            r = np.abs(orc.dudt(Pl, met, case.U0, flags=flags) * jinv).max()
            res[(low, n)] = r / scale
        case.scheme = "weno7"
        res[("weno7", n)] = np.abs(orc.dudt(orc.params_from_case(case), met, case.U0) * jinv).max() / scale
    assert res[("c8", 16)] < 1e-13 and res[("c8", 32)] < 1e-13
    assert res[("ud7", 16)] / res[("ud7", 32)] > 2 ** 7
    assert res[("weno7", 16)] / res[("weno7", 32)] > 2 ** 7
    assert res[("weno7", 32)] < 1e-7


# ---------------------------------------------------------- conservation

@pytest.mark.parametrize("which", ["tgv", "vortex", "hybrid"])
def test_discrete_conservation(orc, which):
    if which == "tgv":
        case = workloads.taylor_green(shape=(16, 12, 20), distorted=True, dt=2e-3)
    elif which == "vortex":
        case = workloads.isentropic_vortex(shape=(20, 16, 12), distorted=True, dt=0.02)
    else:
        case = workloads.taylor_green(shape=(16, 16, 16), distorted=True, dt=2e-3)
        case.scheme = "hybrid"
        case.theta1 = 1e-4
    P, met = _setup(orc, case)
    r0 = orc.reduce(P, met, case.U0)
    U, _, _ = orc.advance(P, met, case.U0, 12, case.dt)
    r1 = orc.reduce(P, met, U)
    tot = np.array([np.abs(case.U0[m] * met[9]).sum() for m in range(5)])
    tot[1:4] = tot[1:4].sum()   # momentum: scale by the whole momentum vector
    assert np.all(np.abs(r1[:5] - r0[:5]) <= 1e-13 * tot)


# -------------------------------------------------------- viscous closed forms

def _viscous_case(fields, n=32):
    """State from analytic primitive fields evaluated on a distorted grid."""
    case = workloads.taylor_green(n, distorted=True)
    x, y, z = case.xyz
    rho, u, v, w, p = fields(x, y, z, case)
    case.U0 = workloads.conserved(case.gamma, rho, u, v, w, p)
    case.Re = 50.0
    return case


def test_viscous_shear_and_bulk(orc):
    d = 1e-3

    def f(x, y, z, c):
        one = np.ones_like(x)
        return one, d * np.sin(x + y), np.zeros_like(x), np.zeros_like(x), one / (c.gamma * c.Ma ** 2)
    case = _viscous_case(f)
    P, met = _setup(orc, case)
    L = orc.dudt(P, met, case.U0, parts=orc.PART_VISC)
    x, y, z = case.xyz
    nu = 1.0 / case.Re   # mu(T = 1) = 1
    # d(rho u)/dt = d tau_xx/dx + d tau_xy/dy = -(4/3 + 1) nu d sin(x+y)
    # d(rho v)/dt = d tau_xy/dx + d tau_yy/dy = -(1 - 2/3) nu d sin(x+y)
    exp_u = -(7.0 / 3.0) * nu * d * np.sin(x + y)
    exp_v = -(1.0 / 3.0) * nu * d * np.sin(x + y)
    sc = nu * d
    assert np.abs(L[0]).max() == 0.0
    assert np.abs(L[1] - exp_u).max() < 1e-4 * sc
    assert np.abs(L[2] - exp_v).max() < 1e-4 * sc
    assert np.abs(L[3]).max() < 1e-4 * sc


def test_viscous_heat_conduction(orc):
    d = 1e-5

    def f(x, y, z, c):
        p = np.full_like(x, 1.0 / (c.gamma * c.Ma ** 2))
        T = 1.0 + d * np.sin(z)
        return c.gamma * c.Ma ** 2 * p / T, np.zeros_like(x), np.zeros_like(x), np.zeros_like(x), p
    case = _viscous_case(f)
    P, met = _setup(orc, case)
    L = orc.dudt(P, met, case.U0, parts=orc.PART_VISC)
    kc = 1.0 / ((case.gamma - 1.0) * case.Ma ** 2 * case.Pr * case.Re)
    exp_E = -kc * d * np.sin(case.xyz[2])
    assert np.abs(L[4] - exp_E).max() < 1e-4 * kc * d
    assert np.abs(L[1:4]).max() < 1e-9 * kc * d


def test_taylor_green_dissipation_rate(orc):
    """KE(0) = 1/8 and the viscous part of dKE/dt at t = 0 equals -3/(4 Re)."""
    rates = {}
    for visc in (6, 0):
        case = workloads.taylor_green(32)
        case.viscous = visc
        P, met = _setup(orc, case)
        U = case.U0
        L = orc.dudt(P, met, U)
        rho, m = U[0], U[1:4]
        if visc:
            assert (0.5 * (m ** 2).sum(0) / rho).mean() == pytest.approx(0.125, rel=1e-14)
        rates[visc] = ((m * L[1:4]).sum(0) / rho - 0.5 * (m ** 2).sum(0) / rho ** 2 * L[0]).mean()
    assert rates[6] - rates[0] == pytest.approx(-3.0 / (4.0 * 1600.0), rel=1e-2)
    assert abs(rates[0]) < 0.1 * 3.0 / (4.0 * 1600.0)


# ---------------------------------------------------------------- sensor

def test_sensor_closed_forms(orc):
    g = json.load(open(os.path.join(GOLDEN, "eq43_thresholds.json")))
    case = workloads.taylor_green(16)
    case.scheme = "hybrid"
    case.theta1, case.theta2 = g["theta1"], g["theta2"]
    nx = 16
    r = 3.0
    shp = case.U0.shape[1:]
    p = np.ones(shp)
    p[:, :, 8:] = r       # step between nodes 7 and 8 along x
    one = np.ones(shp)
    zero = np.zeros(shp)
    U = workloads.conserved(1.4, one, zero, zero, zero, p)
    P = orc.params_from_case(case)
    theta, flags = orc.sensor(P, U)
    # nodes 7 and 8 (and the wrapped step between 15 and 0)
    assert theta[3, 4, 7] == pytest.approx((r - 1) / (r + 3), rel=1e-15)
    assert theta[3, 4, 8] == pytest.approx((r - 1) / (1 + 3 * r), rel=1e-15)
    assert np.all(theta[:, :, [2, 3, 4, 5, 10, 11, 12, 13]] == 0.0)
    # an x interface j+1/2 is WENO iff a node of j-3..j+4 has theta > theta1
    hot = theta[3, 4] > case.theta1
    for j in range(nx):
        win = [(j + m) % nx for m in range(-3, 5)]
        assert flags[0, 3, 4, j] == (1 if hot[win].any() else 0)
    # theta is a node quantity shared by all directions: along y and z every
    # interface of a hot x column is WENO, every other one low-dissipation
    for d in (1, 2):
        assert np.array_equal(flags[d], np.broadcast_to(hot.astype(np.uint8), flags[d].shape))
    # uniform pressure: theta = 0 everywhere
    theta0, _ = orc.sensor(P, case.U0 * 0 + workloads.conserved(1.4, one, zero, zero, zero, one))
    assert np.all(theta0 == 0.0)


# --------------------------------------------------------- exact solutions

def _vortex_error(orc, N, eps, dist=True):
    dt = 0.01 * (64 / N) ** (7 / 3)
    steps = int(round(0.5 / dt))
    dt = 0.5 / steps
    case = workloads.isentropic_vortex(shape=(N, N, 1), distorted=dist, dt=dt)
    case.eps = eps
    P, met = _setup(orc, case)
    U, _, _ = orc.advance(P, met, case.U0, 3 * steps, dt)
    rho_ex, _, _, _ = exact.isentropic_vortex(case.xyz[0], case.xyz[1], 0.5)
    return float(np.sqrt(np.mean((U[0] - rho_ex) ** 2)))


@pytest.mark.slow
def test_isentropic_vortex_convergence(orc):
    """Exact translated vortex (Euler) on a distorted grid: the linear scheme
    (eq 41, reached by WENO7 with a huge epsilon) converges at close to 7th
    order and WENO7 at high order with small error."""
    lin = [_vortex_error(orc, N, 1e30) for N in (64, 128)]
    assert math.log2(lin[0] / lin[1]) > 6.0
    nonlin = [_vortex_error(orc, N, 1e-6) for N in (64, 128)]
    assert math.log2(nonlin[0] / nonlin[1]) > 4.5
    assert nonlin[1] < 2e-6


def test_sod_star_state_matches_textbook():
    g = json.load(open(os.path.join(GOLDEN, "sod_star_toro.json")))
    p, u = exact.riemann_star((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    rho_l, _, _ = exact.riemann_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([u - 1e-9]))
    rho_r, _, _ = exact.riemann_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([u + 1e-9]))
    assert p == pytest.approx(g["p_star"], abs=1e-5)
    assert u == pytest.approx(g["u_star"], abs=1e-5)
    assert rho_l[0] == pytest.approx(g["rho_star_left"], abs=1e-5)
    assert rho_r[0] == pytest.approx(g["rho_star_right"], abs=1e-5)


def _sod_run(orc, n, axis, width=1):
    case = workloads.sod(n, axis=axis, width=width)
    P, met = _setup(orc, case)
    U, _, _ = orc.advance(P, met, case.U0, case.nsteps, case.dt)
    return case, U


@pytest.mark.slow
def test_sod_converges_to_exact_solution(orc):
    errs = []
    for n in (100, 200, 400):
        case, U = _sod_run(orc, n, 0)
        x = case.xyz[0][0, 0]
        rho_ex, _, _ = exact.sod_two_tube(x, 0.2)
        rho = U[0][0, 0]
        errs.append(np.mean(np.abs(rho - rho_ex)) * 2.0)
        if n == 400:
            h = 2.0 / n
            # shock and contact of the right tube within two cells
            right = x > 1.5
            xs, rs = x[right], rho[right]

            def crossing(level):
                i = np.where((rs[:-1] - level) * (rs[1:] - level) <= 0)[0]
                return xs[i]
            p_s, u_s = exact.riemann_star((1, 0, 1), (0.125, 0, 0.1))
            shock = 1.5 + 0.2 * 1.75216
            contact = 1.5 + 0.2 * u_s
            assert np.min(np.abs(crossing(0.5 * (0.26557 + 0.125)) - shock)) < 2 * h
            assert np.min(np.abs(crossing(0.5 * (0.42632 + 0.26557)) - contact)) < 2 * h
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.01


def test_sod_orientation_invariance(orc):
    """The same tube along x, y and z gives bitwise the same profile."""
    prof = []
    for axis in range(3):
        case = workloads.sod(60, axis=axis, width=2)
        case.nsteps = 30
        P, met = _setup(orc, case)
        U, _, _ = orc.advance(P, met, case.U0, case.nsteps, case.dt)
        a = {0: 3, 1: 2, 2: 1}[axis]
        prof.append((np.moveaxis(U[0], a - 1 + 0, -1).reshape(-1, 60),
                     np.moveaxis(U[1 + axis], a - 1, -1).reshape(-1, 60)))
    for axis in (1, 2):
        assert np.array_equal(prof[0][0], prof[axis][0])
        assert np.array_equal(prof[0][1], prof[axis][1])


# ------------------------------------------------------------ invariants

def test_restart_is_bitwise(orc):
    case = workloads.taylor_green(shape=(12, 16, 8), distorted=True, dt=2e-3)
    P, met = _setup(orc, case)
    Ua, _, sa = orc.advance(P, met, case.U0, 5, case.dt)
    U1, Un1, s1 = orc.advance(P, met, case.U0, 2, case.dt)
    Ub, _, sb = orc.advance(P, met, U1, 3, case.dt, Un=Un1, stage=s1)
    assert sa == sb == 2
    assert np.array_equal(Ua, Ub)


@pytest.mark.parametrize("axis,shift", [(3, 3), (2, -5), (1, 7)])
def test_translation_invariance(orc, axis, shift):
    """Rolling every periodic input (state and metrics) by whole nodes rolls
    dU/dt bitwise: the same arithmetic runs at every node, so any slip in
    the index wrap-around shows up."""
    case = workloads.taylor_green(shape=(16, 12, 20), distorted=True)
    rng = np.random.default_rng(0)
    case.U0 = case.U0 + 0.01 * rng.normal(size=case.U0.shape) * np.array([1, 1, 1, 1, 50.0])[:, None, None, None]
    case.scheme = "hybrid"
    P, met = _setup(orc, case)
    L0 = orc.dudt(P, met, case.U0)
    roll = lambda a: np.ascontiguousarray(np.roll(a, shift, axis=axis))
    L1 = orc.dudt(P, roll(met), roll(case.U0))
    assert np.array_equal(roll(L0), L1)


def test_reduction_cfl_uniform_state(orc):
    case = workloads.uniform_flow((8, 8, 8), amplitude_frac=0.0, vel=(0.5, 0.3, 0.2), Ma=0.5)
    P, met = _setup(orc, case)
    r = orc.reduce(P, met, case.U0, 1e-2)
    c = 1.0 / 0.5
    h = case.h[0]
    assert r[5] == pytest.approx(1e-2 * (0.5 + 0.3 + 0.2 + 3 * c) / h, rel=1e-12)
    assert r[0] == pytest.approx(case.N, rel=1e-12)   # 1/J = 1 when h is the node spacing
    assert r[8] == 0.0
