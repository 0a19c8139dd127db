"""Pins of the oracle's central viscous terms of sixth and eighth order (Sec.
2.3): the observed order of the two-pass operator against its closed form,
the boundary ladder (second-order one-sided at the end node, then second-,
fourth- and sixth-order central at the next three nodes, then the interior
order) located by where a cubic profile becomes exact, and the Taylor-Green
dissipation rate."""
import dataclasses

import numpy as np
import pytest

import workloads


def _shear_error(orc, n, order):
    """Max error of d(rho u)/dt for u = d sin(x + y) (closed form
    -(7/3) nu d sin(x + y)) relative to nu d, on the uniform periodic grid."""
    case = workloads.taylor_green(n)
    x, y, z = case.xyz
    d = 1e-3
    one = np.ones_like(x)
    case = dataclasses.replace(case, viscous=order, Re=50.0,
                               U0=workloads.conserved(case.gamma, one, d * np.sin(x + y), 0 * x, 0 * x,
                                                      one / (case.gamma * case.Ma ** 2)))
    P = orc.params_from_case(case)
    L = orc.dudt(P, orc.metrics(P, case.xyz), case.U0, parts=orc.PART_VISC)
    nu = 1.0 / case.Re
    return np.abs(L[1] + (7.0 / 3.0) * nu * d * np.sin(x + y)).max() / (nu * d)


@pytest.mark.parametrize("order", [6, 8])
def test_viscous_convergence_order(orc, order):
    e = [_shear_error(orc, n, order) for n in (16, 24, 32)]
    rates = [np.log(e[0] / e[1]) / np.log(24 / 16), np.log(e[1] / e[2]) / np.log(32 / 24)]
    print(order, e, rates)
    assert all(abs(r - order) < 0.3 for r in rates)


@pytest.mark.parametrize("order,first_exact", [(6, 5), (8, 6)])
def test_viscous_boundary_ladder(orc, order, first_exact):
    """u = a y^3 along a bounded eta line (uniform grid, so the metrics are
    exact): du/dy is exact only where the first pass uses fourth order or
    more (two nodes in); the second pass of node i (half width min(order/2,
    distance to the end)) is exact iff every node it reads is, i.e. from the
    5th node in at sixth order and the 6th at eighth order."""
    case = workloads.taylor_green(shape=(8, 24, 8), distorted=False)
    case = dataclasses.replace(case, periodic=(1, 0, 1), bc=(0, 0, 2, 2, 0, 0), viscous=order, Re=50.0)
    x, y, z = case.xyz
    a = 1e-3
    one = np.ones_like(x)
    case.U0 = workloads.conserved(case.gamma, one, a * y ** 3, 0 * x, 0 * x, one / (case.gamma * case.Ma ** 2))
    P = orc.params_from_case(case)
    L = orc.dudt(P, orc.metrics(P, case.xyz), case.U0, parts=orc.PART_VISC)
    nu = 1.0 / case.Re
    err = (np.abs(L[1] - nu * 6.0 * a * y) / (nu * 6.0 * a * y.max()))[0, :, 0]
    n = case.ny
    dist = np.minimum(np.arange(n), n - 1 - np.arange(n))
    inner = (dist >= first_exact)
    assert err[inner].max() < 1e-13
    ramp = (dist >= 1) & (dist < first_exact)
    assert err[ramp].min() > 1e-8
    assert err[dist == first_exact - 1].min() > 1e-8


def test_taylor_green_dissipation_rate_eighth_order(orc):
    """Viscous part of dKE/dt at t = 0 equals -3/(4 Re) with the eighth-order terms."""
    rates = {}
    for visc in (8, 0):
        case = workloads.taylor_green(32)
        case.viscous = visc
        P = orc.params_from_case(case)
        U = case.U0
        L = orc.dudt(P, orc.metrics(P, case.xyz), U)
        rho, m = U[0], U[1:4]
        rates[visc] = ((m * L[1:4]).sum(0) / rho - 0.5 * (m ** 2).sum(0) / rho ** 2 * L[0]).mean()
    assert rates[8] - rates[0] == pytest.approx(-3.0 / (4.0 * 1600.0), rel=1e-2)
