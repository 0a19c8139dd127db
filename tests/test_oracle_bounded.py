"""Pins of the oracle on grids with bounded (non-periodic) directions: the
one-sided and reduced-order closures of the derivative operators (Sec. 2.3),
the masked fifth-order WENO at interfaces whose stencil leaves the domain
(Sec. 2.2.4), and the boundary kinds of the compression-ramp case.

Each check compares the oracle with something fixed independently of it:
exact derivatives of polynomial mappings, the periodic oracle at nodes whose
stencils never reach a boundary, mirror symmetry, convergence to the exact
right-hand side of a smooth flow, and the definitions of the face kinds."""
import numpy as np
import pytest

import workloads


def _case(nx, ny, nz, periodic, xyz, U0, bc=(0,) * 6, viscous=0, scheme="weno7", Tw=1.0, period=(0, 0, 0),
          h=(1.0, 1.0, 1.0), Re=100.0, Ma=0.5):
    return workloads.Case(name="bounded", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=U0, period=period, h=h, dt=1e-3,
                          nsteps=1, periodic=periodic, bc=bc, gamma=1.4, Re=Re, Ma=Ma, Pr=0.72, Tw=Tw,
                          viscous=viscous, scheme=scheme)


def test_metrics_exact_for_separable_quadratic_mapping(orc):
    """x = x(xi), y = y(eta) quadratic, z = zeta: every closure (one-sided at
    the ends, then 2nd to 8th order) differentiates quadratics exactly, and the
    conservative metrics reduce to xi_x/J = y_eta z_zeta, eta_y/J = x_xi z_zeta,
    zeta_z/J = x_xi y_eta, 1/J = x_xi y_eta z_zeta."""
    nx, ny, nz = 13, 11, 6
    h = (0.1, 0.2, 0.3)
    xi, eta, zeta = (np.arange(n) * hh for n, hh in zip((nx, ny, nz), h))
    K, J, I = np.meshgrid(zeta, eta, xi, indexing="ij")
    x = I + 0.3 * I * I
    y = 2.0 * J - 0.25 * J * J
    z = K
    xyz = np.stack([x, y, z])
    case = _case(nx, ny, nz, (0, 0, 1), xyz, np.zeros((5, nz, ny, nx)), period=(0, 0, nz * h[2]), h=h)
    P = orc.params_from_case(case)
    met = orc.metrics(P, xyz)
    xx, yy, zz = 1.0 + 0.6 * I, 2.0 - 0.5 * J, np.ones_like(K)
    ref = np.zeros_like(met)
    ref[0] = yy * zz
    ref[4] = xx * zz
    ref[8] = xx * yy
    ref[9] = xx * yy * zz
    assert np.abs(met - ref).max() < 1e-12


def test_metrics_one_sided_closure_order(orc):
    """On a cubic mapping the end node's one-sided derivative is second order:
    its error falls by ~4 per halving of the spacing."""
    errs = []
    for n in (17, 33, 65):
        hh = 1.0 / (n - 1)
        xi = np.arange(n) * hh
        K, J, I = np.meshgrid(np.arange(8) * hh, np.arange(8) * hh, xi, indexing="ij")
        xyz = np.stack([I + 0.5 * I ** 3, J, K])
        case = _case(n, 8, 8, (0, 1, 1), xyz, np.zeros((5, 8, 8, n)), period=(0, 8 * hh, 8 * hh), h=(hh, hh, hh))
        met = orc.metrics(orc.params_from_case(case), xyz)
        errs.append(abs(met[9][0, 0, 0] - (1.0 + 1.5 * xi[0] ** 2) * 1.0))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def _periodic_field(nx, ny, nz, seed):
    """A smooth periodic state on a uniform Cartesian grid."""
    rng = np.random.default_rng(seed)
    K, J, I = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in (nz, ny, nx)], indexing="ij")
    ph = rng.uniform(0, 2 * np.pi, 6)
    rho = 1.0 + 0.1 * np.sin(I + ph[0]) * np.cos(J + ph[1])
    u = 0.3 + 0.2 * np.sin(J + ph[2])
    v = 0.1 * np.cos(I + ph[3]) * np.sin(K + ph[4])
    w = 0.05 * np.sin(I + J + ph[5])
    p = 1.0 / (1.4 * 0.5 ** 2) * (1.0 + 0.05 * np.cos(I - K))
    return workloads.conserved(1.4, rho, u, v, w, p)


@pytest.mark.parametrize("scheme", ["weno7", "hybrid"])
def test_interior_nodes_match_periodic_oracle(orc, scheme):
    """Along a bounded direction, a node whose inviscid stencils (j-4 .. j+4)
    and viscous stencils (j-6 .. j+6) stay inside the domain is computed by the
    same arithmetic as on the periodic grid: bitwise equal."""
    nx, ny, nz = 24, 20, 6
    U = _periodic_field(nx, ny, nz, 1)
    h = (2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz)
    K, J, I = np.meshgrid(*[np.arange(n) * hh for n, hh in zip((nz, ny, nx), h[::-1])], indexing="ij")
    xyz = np.stack([I, J, K])
    per = _case(nx, ny, nz, (1, 1, 1), xyz, U, viscous=6, scheme=scheme, period=(2 * np.pi,) * 3, h=h)
    bnd = _case(nx, ny, nz, (0, 0, 1), xyz, U, viscous=6, scheme=scheme, period=(0, 0, 2 * np.pi), h=h)
    Pp, Pb = orc.params_from_case(per), orc.params_from_case(bnd)
    met = orc.metrics(Pp, xyz)
    flags = None
    if scheme == "hybrid":
        _, flags = orc.sensor(Pp, U)
    a = orc.dudt(Pp, met, U, flags)
    b = orc.dudt(Pb, met, U, flags)
    inner = (slice(None), slice(None), slice(6, ny - 6), slice(6, nx - 6))
    assert np.array_equal(a[inner], b[inner])
    # nodes near the ends differ (closures), and the end faces are zero
    assert not np.array_equal(a[:, :, 1:4, 6:-6], b[:, :, 1:4, 6:-6])
    assert np.all(b[:, :, :, 0] == 0) and np.all(b[:, :, :, -1] == 0)
    assert np.all(b[:, :, 0, :] == 0) and np.all(b[:, :, -1, :] == 0)


def test_mirror_symmetry(orc):
    """A state mirrored about the middle of a bounded direction (u odd, the
    rest even) has a mirrored right-hand side: the closures at the two ends
    are mirror images of each other."""
    n, ny = 20, 8
    hh = 0.1
    x = (np.arange(n) - (n - 1) / 2) * hh
    K, J, X = np.meshgrid(np.arange(4) * hh, np.arange(ny) * hh, x, indexing="ij")
    xyz = np.stack([X, J, K])
    rng = np.random.default_rng(5)
    a = rng.uniform(0.5, 1.5, 3)
    rho = 1.0 + 0.2 * np.exp(-a[0] * X ** 2) * (1 + 0.1 * np.sin(2 * np.pi * J / (ny * hh)))
    u = 0.4 * np.sin(a[1] * X)
    v = 0.1 * np.cos(X) * np.cos(2 * np.pi * J / (ny * hh))
    w = 0.0 * X
    p = 2.0 + 0.3 * np.cos(a[2] * X)
    U = workloads.conserved(1.4, rho, u, v, w, p)
    for viscous in (0, 6):
        case = _case(n, ny, 4, (0, 1, 1), xyz, U, viscous=viscous, period=(0, ny * hh, 4 * hh), h=(hh,) * 3)
        P = orc.params_from_case(case)
        met = orc.metrics(P, xyz)
        d = orc.dudt(P, met, U)
        m = d[:, :, :, ::-1].copy()
        m[1] *= -1.0
        scale = np.abs(d).max(axis=(1, 2, 3), keepdims=True) + 1e-300
        assert np.abs(d - m).max() / scale.max() < 1e-12, viscous
        assert np.all(np.abs(d - m) <= 1e-11 * scale)


def test_closures_converge_to_exact_rhs(orc):
    """Density wave carried by uniform u and p along a bounded xi: the exact
    right-hand side is -rho'(x) (u, u^2, 0, 0, u^3/2).  With the masked WENO5
    at the three interfaces nearest each end, the max error over all nodes
    that are not on a face falls at least at second order."""
    errs = []
    for n in (32, 64, 128):
        hh = 2.0 / (n - 1)
        x = -1.0 + np.arange(n) * hh
        K, J, X = np.meshgrid(np.arange(1) * hh, np.arange(1) * hh, x, indexing="ij")
        xyz = np.stack([X, J, K])
        rho = 1.0 + 0.2 * np.sin(np.pi * X + 0.3)
        drho = 0.2 * np.pi * np.cos(np.pi * X + 0.3)
        u0, p0 = 0.5, 1.0
        U = workloads.conserved(1.4, rho, u0 + 0 * X, 0 * X, 0 * X, p0 + 0 * X)
        case = _case(n, 1, 1, (0, 1, 1), xyz, U, period=(0, hh, hh), h=(hh, hh, hh))
        P = orc.params_from_case(case)
        d = orc.dudt(P, orc.metrics(P, xyz), U)
        ref = -drho * np.array([u0, u0 ** 2, 0.0, 0.0, 0.5 * u0 ** 3])[:, None, None, None]
        errs.append(np.abs(d - ref)[:, :, :, 1:-1].max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_boundary_kinds(orc):
    """Faces after the boundary step: inflow = the given state (face indexed
    by the other two node indices, lower direction fastest), extrapolation =
    primitives of the first interior node, wall = no slip, T = Tw, pressure of
    the first interior node; corners take the last face applied (eta+ after
    xi+); interior nodes untouched."""
    nx, ny, nz = 10, 9, 4
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.8, 1.2, (nz, ny, nx))
    u, v, w = (rng.uniform(-0.3, 0.3, (nz, ny, nx)) for _ in range(3))
    p = rng.uniform(0.9, 1.1, (nz, ny, nx))
    U = workloads.conserved(1.4, rho, u, v, w, p)
    inflow = rng.uniform(0.5, 2.0, (5, nz, ny))
    Tw, Ma, g = 2.5, 0.5, 1.4
    case = _case(nx, ny, nz, (0, 0, 1), np.zeros((3, nz, ny, nx)), U, bc=(1, 2, 3, 2, 0, 0), Tw=Tw, Ma=Ma)
    P = orc.params_from_case(case)
    out = orc.apply_bc(P, U, inflow)
    assert np.array_equal(out[:, :, 1:-1, 1:-1], U[:, :, 1:-1, 1:-1])
    # inflow face i = 0 (rows j = 1 .. ny-2: the wall and the top overwrite the corners)
    assert np.array_equal(out[:, :, 1:-1, 0], inflow[:, :, 1:-1])

    def prim(V):
        r = V[0]
        uu, vv, ww = V[1] / r, V[2] / r, V[3] / r
        return r, uu, vv, ww, (g - 1) * (V[4] - 0.5 * r * (uu * uu + vv * vv + ww * ww))
    # outlet i = nx-1 from the state at i = nx-2
    a, b = prim(out[:, :, 1:-1, -1]), prim(U[:, :, 1:-1, -2])
    for qa, qb in zip(a, b):
        assert np.allclose(qa, qb, rtol=1e-14, atol=1e-15)
    # wall j = 0 from the updated row j = 1 (including the inflow and outlet columns)
    r, uu, vv, ww, pw = prim(out[:, :, 0, :])
    assert np.all(out[1:4, :, 0, :] == 0.0)
    _, _, _, _, p1 = prim(out[:, :, 1, :])
    assert np.allclose(pw, p1, rtol=1e-14)
    assert np.allclose(g * Ma * Ma * pw / r, Tw, rtol=1e-14)
    # top j = ny-1 from row ny-2
    a, b = prim(out[:, :, -1, :]), prim(out[:, :, -2, :])
    for qa, qb in zip(a, b):
        assert np.allclose(qa, qb, rtol=1e-14, atol=1e-15)


def test_ramp_short_run_stays_physical(orc):
    """A reduced compression ramp runs 30 substeps with positive pressure and
    density, zero wall velocity and the inflow face held."""
    case = workloads.compression_ramp(shape=(48, 24, 4))
    P = orc.params_from_case(case, nthreads=8)
    met = orc.metrics(P, case.xyz)
    U, _, _ = orc.advance(P, met, case.U0, 30, case.dt, inflow=case.inflow)
    red = orc.reduce(P, met, U, case.dt)
    assert red[8] == 0 and red[6] > 0 and red[7] > 0
    assert red[5] < 0.6
    assert np.all(U[1:4, :, 0, :] == 0.0)
    assert np.array_equal(U[:, :, 1:-1, 0], case.inflow[:, :, 1:-1])
