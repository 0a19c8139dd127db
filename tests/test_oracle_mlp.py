"""Pins of the learned-sensor oracle: the FP64 backward pass against central
finite differences of the loss, the bfloat16 rounding against its definition,
and the node features against closed forms."""
import numpy as np
import pytest

import workloads
from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1)
    theta[-34:-1] *= 10.0       # a non-trivial output layer
    X = rng.normal(size=(64, 32))
    y = (rng.random(64) < 0.3).astype(float)
    w = rng.uniform(0.5, 2.0, 64)
    L, g = mlp.loss_and_grad(theta, X, y, w)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, 200, replace=False)
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, y, w)[0] - mlp.loss_and_grad(tm, X, y, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), i


def test_bf16_rounding_definition():
    # values exactly halfway between two bfloat16 numbers round to the even one
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    assert mlp.bf16(one + ulp / 2) == 1.0
    assert mlp.bf16(one + 3 * ulp / 2) == 1.0 + 2 * ulp
    x = np.random.default_rng(1).normal(size=1000).astype(np.float32)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-45)   # half an ulp of 7 stored bits
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_features_closed_forms(orc):
    """Uniform flow: zero divergence, vorticity and jumps.  A shear u = a sin y:
    |curl| from the second-order difference of sin.  A density step along x:
    the normalised first differences on both sides of it (and at the periodic
    seam).  A pressure linear in x: the plain sensor (eq 42, computed by the
    C oracle) is silent, the pressure jump is not: the feature is not the
    label."""
    case = workloads.uniform_flow((12, 10, 8), amplitude_frac=0.0)
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    F = mlp.node_features(case.gamma, case.h, met, case.U0)
    assert F.shape[0] == 4 and np.abs(F).max() < 1e-12
    x, y, z = case.xyz
    a = 0.3
    rho = np.ones_like(x)
    p = np.full_like(x, 1.0 / (1.4 * 0.25))
    U = workloads.conserved(1.4, rho, a * np.sin(y), 0 * x, 0 * x, p)
    F = mlp.node_features(1.4, case.h, met, U)
    hy = case.h[1]
    curl = a * np.cos(y) * np.sin(hy) / hy
    c = np.sqrt(1.4 * p / rho)
    assert np.abs(F[0]).max() < 1e-14
    assert np.allclose(F[1], np.cbrt(met[9]) * np.abs(curl) / c, rtol=1e-12, atol=1e-15)
    r = 3.0
    rho = np.where(np.arange(12)[None, None, :] >= 6, r, 1.0) * np.ones_like(x)
    U = workloads.conserved(1.4, rho, 0 * x, 0 * x, 0 * x, p)
    F = mlp.node_features(1.4, case.h, met, U, theta1=0.02)
    for node in (5, 6, 11, 0):
        assert F[3][0, 0, node] == pytest.approx((r - 1) / (r + 1) / 0.02, rel=1e-14), node
    assert F[3][0, 0, 3] == 0.0 and F[3][0, 0, 8] == 0.0 and np.all(F[2] == 0.0)
    # linear pressure p = p0 (1 + e x) in the interior of x (away from the seam)
    e = 0.01
    pl = p * (1.0 + e * x)
    U = workloads.conserved(1.4, np.ones_like(x), 0 * x, 0 * x, 0 * x, pl)
    theta, _ = orc.sensor(P, U)
    F = mlp.node_features(1.4, case.h, met, U, theta1=0.02)
    hx = case.h[0]
    xi = x[:, :, 1:-1]
    assert np.allclose(F[2][:, :, 1:-1], e * hx / (1.0 + e * xi) / 0.02, rtol=1e-10)
    assert np.abs(theta[:, :, 1:-1]).max() < 1e-13 and F[2][:, :, 1:-1].min() > 0.01
    # the "curv" inputs: the pressure feature times theta1 is the plain
    # sensor's node value, on a noisy state
    rng = np.random.default_rng(4)
    U = case.U0 * (1.0 + 0.05 * rng.standard_normal(case.U0.shape))
    theta, _ = orc.sensor(P, U)
    F = mlp.node_features(1.4, case.h, met, U, theta1=case.theta1, inputs="curv")
    assert np.allclose(F[2] * case.theta1, theta, rtol=1e-13, atol=1e-16)


def test_features_on_bounded_lines(orc):
    """Along a bounded direction the end nodes take a one-sided difference over
    one spacing (exact for linear fields) and add no jump term: u = a x,
    v = b x give div = a and |curl| = |b| at every node, ends included; a
    density quadratic in y has a known normalised first difference inside
    and none at the eta ends."""
    nx, ny, nz = 12, 9, 4
    hh = (0.2, 0.3, 0.25)
    K, J, I = np.meshgrid(*[np.arange(n) * s for n, s in zip((nz, ny, nx), hh[::-1])], indexing="ij")
    xyz = np.stack([I, J, K])
    case = workloads.Case(name="b", nx=nx, ny=ny, nz=nz, xyz=xyz, U0=np.zeros((5, nz, ny, nx)),
                          period=(0, 0, nz * hh[2]), h=hh, dt=1e-3, nsteps=1, periodic=(0, 0, 1))
    P = orc.params_from_case(case)
    met = orc.metrics(P, xyz)
    a, b = 0.2, -0.15
    rho = 1.0 + 0.1 * J * J
    p = np.full_like(I, 2.0)
    U = workloads.conserved(1.4, rho, a * I, b * I, 0 * I, p)
    F = mlp.node_features(1.4, hh, met, U, periodic=(0, 0, 1), theta1=0.02)
    c = np.sqrt(1.4 * p / rho)
    delta = np.cbrt(met[9])
    assert np.allclose(F[0], delta * a / c, rtol=1e-12)
    assert np.allclose(F[1], delta * abs(b) / c, rtol=1e-12)
    y = J[:, 1:-1, :]
    # rho(y + h) - rho(y - h) = 0.4 y h;  rho(y + h) + rho(y - h) = 2 + 0.2 (y^2 + h^2)
    inner = 0.4 * y * hh[1] / (2.0 + 0.2 * (y * y + hh[1] ** 2)) / 0.02
    assert np.allclose(F[3][:, 1:-1, :], inner, rtol=1e-10)
    assert np.all(F[3][:, 0, :] == 0.0) and np.all(F[3][:, -1, :] == 0.0)
    assert np.abs(F[2]).max() < 1e-12   # uniform pressure, recovered from E with rounding
    rng = np.random.default_rng(6)
    U = U * (1.0 + 0.05 * rng.standard_normal(U.shape))
    theta, _ = orc.sensor(P, U)
    F = mlp.node_features(1.4, hh, met, U, periodic=(0, 0, 1), theta1=case.theta1, inputs="curv")
    assert np.allclose(F[2] * case.theta1, theta, rtol=1e-13, atol=1e-16)
    assert mlp.window_inside(nx, np.arange(nx), False).tolist() == [False] * 3 + [True] * (nx - 7) + [False] * 4
