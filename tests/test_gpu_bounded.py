"""Parity of the HIP library with the CPU oracle on grids with bounded
directions: a reduced compression ramp (bounded xi and eta, periodic zeta;
inflow, outflow, wall and top faces) and a box bounded in all three
directions.  Same bars as the periodic parity tests: states after substeps
within 1e-12 (relative L2 per field), dU/dt within a multiple of the
oracle's own one-ulp sensitivity; the face kinds exactly."""
import numpy as np
import pytest

import workloads
from helpers import rel_errors, ulp_perturbed, assert_within_roundoff

pytestmark = pytest.mark.gpu

TOL_L2 = 1e-12


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


CASES = {
    "ramp": lambda: workloads.compression_ramp(shape=(40, 24, 8)),
    "box": lambda: workloads.bounded_box(shape=(36, 20, 18)),
}


def face_masks(case):
    """[nz, ny, nx] masks: nodes on a bounded face whose kind sets them after a
    stage (every kind but the nonreflecting one, 4), and nodes that lie on
    nonreflecting faces only."""
    shp = (case.nz, case.ny, case.nx)
    k, j, i = np.meshgrid(*[np.arange(n) for n in shp], indexing="ij")
    pos = (i, j, k)
    n = (case.nx, case.ny, case.nz)
    on_set = np.zeros(shp, bool)
    on_nrbc = np.zeros(shp, bool)
    for d in range(3):
        if case.periodic[d]:
            continue
        for side, at in ((0, pos[d] == 0), (1, pos[d] == n[d] - 1)):
            if case.bc[2 * d + side] == 4:
                on_nrbc |= at
            else:
                on_set |= at
    return on_set, on_nrbc & ~on_set


def _solver(pk, torch, case):
    s = pk.Solver(pk.params_from(case))
    s.set_grid(_dev(torch, case.xyz))
    s.set_state(_dev(torch, case.U0))
    if case.inflow is not None:
        s.set_inflow(_dev(torch, case.inflow))
    return s


@pytest.mark.parametrize("name", list(CASES))
def test_bounded_metrics_parity(pk, torch_cuda, orc, name):
    case = CASES[name]()
    print("case", case.name, flush=True)
    s = _solver(pk, torch_cuda, case)
    met = orc.metrics(orc.params_from_case(case), case.xyz)
    got = s.metrics().cpu().numpy()
    assert np.abs(got - met).max() <= 1e-13 * np.abs(met).max()


PARTS = {"xi": 1, "eta": 2, "zeta": 4, "visc": 8, "all": 15}


@pytest.mark.parametrize("part", list(PARTS))
@pytest.mark.parametrize("name", list(CASES))
def test_bounded_dudt_parity(pk, torch_cuda, orc, name, part):
    case = CASES[name]()
    print("case", case.name, part, flush=True)
    s = _solver(pk, torch_cuda, case)
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    ref = orc.dudt(P, met, case.U0, parts=PARTS[part])
    ref_pert = orc.dudt(P, met, ulp_perturbed(case.U0), parts=PARTS[part])
    got = s.dudt(_dev(torch_cuda, case.U0), PARTS[part]).cpu().numpy()
    # nodes on faces whose kind sets them after the stage: exactly zero; nodes
    # of nonreflecting faces only: advanced (nonzero) and compared below
    set_mask, nrbc_mask = face_masks(case)
    assert np.all(got[:, set_mask] == 0.0)
    if nrbc_mask.any() and part in ("xi", "all"):
        assert np.all(np.abs(got[:, nrbc_mask]).max(axis=0) > 0.0)
    assert_within_roundoff(got, ref, ref_pert, what=f"{case.name} {part}")


@pytest.mark.parametrize("name", list(CASES))
def test_bounded_advance_parity(pk, torch_cuda, orc, name):
    """Two full Runge-Kutta steps with the faces set after every stage."""
    case = CASES[name]()
    print("case", case.name, flush=True)
    s = _solver(pk, torch_cuda, case)
    s.advance(6, case.dt)
    got = s.state().cpu().numpy()
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    ref, _, _ = orc.advance(P, met, case.U0, 6, case.dt, inflow=case.inflow)
    l2, linf = rel_errors(got, ref)
    print(f"{case.name}: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_L2)
    # wall (eta-): no slip exactly; inflow face (xi-, away from the edges that
    # later faces overwrite) held
    assert np.all(got[1:4, :, 0, :] == 0.0)
    ks = slice(None) if case.periodic[2] else slice(1, -1)
    assert np.array_equal(got[:, ks, 1:-1, 0], case.inflow[:, ks, 1:-1])


@pytest.mark.parametrize("lowdiss", ["c8", "ud7"])
def test_bounded_hybrid_parity(pk, torch_cuda, orc, lowdiss):
    """Hybrid scheme with its own pressure sensor (windows clipped at the ends)."""
    case = CASES["ramp"]()
    case.scheme, case.lowdiss = "hybrid", lowdiss
    # pressure noise in a ball around the grid centre, so the sensor marks part
    # of the domain (the initial pressure is uniform)
    rng = np.random.default_rng(17)
    k, j, i = np.meshgrid(*[np.arange(n) - n / 2 for n in (case.nz, case.ny, case.nx)], indexing="ij")
    ball = np.exp(-(i * i + j * j) / (2.0 * 5.0 ** 2))
    U0 = case.U0.copy()
    U0[4] *= 1.0 + 0.05 * ball * rng.standard_normal(ball.shape)
    case.U0 = U0
    s = _solver(pk, torch_cuda, case)
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    theta, flags = orc.sensor(P, case.U0)
    fl = torch_cuda.zeros((3,) + case.U0.shape[1:], dtype=torch_cuda.uint8, device="cuda")
    pk.ocfd_sensor_flags(s.h, _dev(torch_cuda, case.U0), pk.OCFD_SENSOR_PLAIN, fl)
    low = (flags == 0).mean()
    print(f"ramp hybrid {lowdiss}: low-dissipation fraction {low:.3f}", flush=True)
    assert 0.05 < low < 0.95
    assert np.array_equal(fl.cpu().numpy(), flags)
    # WENO fractions of the evaluation: nonzero flags or bounded-end closures,
    # over the interfaces that exist (none at the last node of a bounded line)
    s.dudt(_dev(torch_cuda, case.U0))
    got = np.array(s.reduce(case.dt))[9:12]
    ref = []
    for d, ax in enumerate((3, 2, 1)):
        n = case.U0.shape[ax]
        pos = np.arange(n).reshape([-1 if a == ax - 1 else 1 for a in range(3)])
        weno = flags[d] != 0
        if not case.periodic[d]:
            exists = np.broadcast_to(pos < n - 1, weno.shape)
            weno = weno | np.broadcast_to((pos < 3) | (pos > n - 5), weno.shape)
        else:
            exists = np.ones_like(weno)
        ref.append((weno & exists).sum() / exists.sum())
    print(f"ramp hybrid {lowdiss}: WENO fractions {got} (oracle flags {ref})", flush=True)
    assert np.allclose(got, ref, rtol=1e-15, atol=0)
    s.advance(3, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, met, case.U0, 3, case.dt, inflow=case.inflow)
    l2, _ = rel_errors(got, ref)
    print(f"ramp hybrid {lowdiss}: rel L2 {l2}", flush=True)
    assert np.all(l2 <= TOL_L2)


# box-narrow: bounded in every direction with fewer xi nodes than one chunk
# of 16 and ragged eta and zeta lines (the aligned xi blocks and the bounded
# 24-slot eta and zeta sweeps at their edges)
@pytest.mark.parametrize("which", ["ramp", "box-narrow"])
def test_bounded_mixed_precision_drift(pk, torch_cuda, orc, which):
    """FP32 split and reconstruction on bounded grids: 30 substeps stay
    within 1e-5 of the FP64 oracle."""
    case = CASES["ramp"]() if which == "ramp" else workloads.bounded_box(shape=(12, 20, 18))
    case.precision = "mixed"
    s = _solver(pk, torch_cuda, case)
    s.advance(30, case.dt)
    got = s.state().cpu().numpy()
    P = orc.params_from_case(case)
    ref, _, _ = orc.advance(P, orc.metrics(P, case.xyz), case.U0, 30, case.dt, inflow=case.inflow)
    l2, _ = rel_errors(got, ref)
    print(f"{which} mixed 30 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= 1e-5)
    if which == "ramp":
        assert np.all(got[1:4, :, 0, :] == 0.0)


@pytest.mark.parametrize("lowdiss", ["c8", "ud7"])
def test_bounded_mixed_hybrid_drift(pk, torch_cuda, orc, lowdiss):
    """FP32 split and reconstruction in the hybrid scheme on the ramp (the
    bounded xi sweep takes its one-list path; its own pressure sensor marks a
    ball of noise as WENO): 30 substeps stay within 1e-5 of the FP64 oracle."""
    case = CASES["ramp"]()
    case.scheme, case.lowdiss, case.precision = "hybrid", lowdiss, "mixed"
    rng = np.random.default_rng(29)
    k, j, i = np.meshgrid(*[np.arange(n) - n / 2 for n in (case.nz, case.ny, case.nx)], indexing="ij")
    ball = np.exp(-(i * i + j * j) / (2.0 * 5.0 ** 2))
    U0 = case.U0.copy()
    U0[4] *= 1.0 + 0.05 * ball * rng.standard_normal(ball.shape)
    case.U0 = U0
    P = orc.params_from_case(case)
    _, flags = orc.sensor(P, case.U0)
    weno = (flags[0] != 0).mean()
    print(f"ramp mixed hybrid {lowdiss}: xi WENO fraction of the first substep {weno:.3f}", flush=True)
    assert 0.05 < weno < 0.95
    s = _solver(pk, torch_cuda, case)
    s.advance(30, case.dt)
    got = s.state().cpu().numpy()
    ref, _, _ = orc.advance(P, orc.metrics(P, case.xyz), case.U0, 30, case.dt, inflow=case.inflow)
    l2, _ = rel_errors(got, ref)
    print(f"ramp mixed hybrid {lowdiss} 30 substeps: rel L2 {l2}", flush=True)
    assert np.all(l2 <= 1e-5)


def test_bounded_call_order_errors(pk, torch_cuda):
    case = CASES["ramp"]()
    s = pk.Solver(pk.params_from(case))
    s.set_grid(_dev(torch_cuda, case.xyz))
    s.set_state(_dev(torch_cuda, case.U0))
    with pytest.raises(pk.OcfdError, match="STATE"):
        s.advance(1, case.dt)                       # inflow face without its state
    per = workloads.taylor_green(shape=(16, 16, 8))
    t = pk.Solver(pk.params_from(per))
    with pytest.raises(pk.OcfdError, match="UNSUPPORTED"):
        t.set_inflow(_dev(torch_cuda, np.zeros((5, 8, 16))))


def _ramp_noise_ball(case, rng, z_sigma):
    """Seeded pressure noise in a ball around the ramp corner (mid-span): the
    initial pressure is uniform, so without it the sensor marks no interior
    interface.  Returns the ball's weight per node; case.U0 and the inflow
    face are replaced."""
    x = case.xyz[0][case.nz // 2]
    y = case.xyz[1][case.nz // 2]
    zi = np.arange(case.nz)[:, None, None] - case.nz // 2
    ball = np.exp(-(x * x + (y - 1.0) ** 2)[None] / (2.0 * 1.5 ** 2) - zi * zi / (2.0 * z_sigma ** 2))
    U0 = case.U0.copy()
    U0[4] *= 1.0 + 0.05 * ball * rng.standard_normal(ball.shape)
    case.U0 = U0
    case.inflow = np.ascontiguousarray(U0[:, :, :, 0])
    return ball


def _ramp_sample(case, rng, n_any, n_near):
    """Sampled node indices: n_any anywhere and n_near of them within six
    nodes of the inflow, outflow, wall or top faces."""
    nx, ny, nz = case.nx, case.ny, case.nz
    edge = np.r_[0:6, nx - 6:nx]
    wall = np.r_[0:6, ny - 6:ny]
    near = []
    for _ in range(n_near):
        i = rng.choice(edge) if rng.random() < 0.5 else rng.integers(nx)
        j = rng.choice(wall) if rng.random() < 0.5 or i not in edge else rng.integers(ny)
        near.append(i + nx * (j + ny * rng.integers(nz)))
    return np.r_[rng.choice(case.N, n_any, replace=False), near].astype(np.int64)


RAMP_FORMS = {"weno7": {}, "weno7_char": dict(characteristic=True),
              "hybrid3_char": dict(characteristic=True, scheme="hybrid", lowdiss="ud7", three_way=True)}


@pytest.mark.parametrize("form", list(RAMP_FORMS))
def test_ramp_full_size_sampled(pk, torch_cuda, orc, form):
    """The compression ramp at the benchmark's size (1024 x 160 x 128) in its
    launch configuration, for each FP64 form the benchmark times there: WENO7,
    WENO7 in characteristic variables, and the three-way hybrid in
    characteristic variables (the GPU's own sensor; seeded pressure noise
    around the corner so that all three stencils occur).  dU/dt at sampled
    nodes, a third of them within six nodes of the inflow, outflow, wall and
    top faces, against the oracle evaluated node by node; the hybrid's oracle
    uses its own sensor over the whole field."""
    import dataclasses
    case = dataclasses.replace(workloads.compression_ramp(), **RAMP_FORMS[form])
    hyb = case.scheme == "hybrid"
    rng = np.random.default_rng(7)
    if hyb:
        ball = _ramp_noise_ball(case, np.random.default_rng(23), 20.0)
    print("case", case.name, form, flush=True)
    s = _solver(pk, torch_cuda, case)
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy().reshape(5, -1)
    s.close()
    del s
    torch_cuda.cuda.empty_cache()
    nodes = _ramp_sample(case, rng, 80, 40)
    flags = None
    P = orc.params_from_case(case, nthreads=0)
    met = orc.metrics(P, case.xyz)
    if hyb:
        nodes = np.r_[nodes, rng.choice(np.flatnonzero(ball.reshape(-1) > 0.3), 60, replace=False)]
        theta, flags = orc.sensor(P, case.U0)
        # flags could differ only where theta lies at a threshold
        assert np.abs(theta - case.theta1).min() > 1e-12 and np.abs(theta - case.theta2).min() > 1e-12
        del theta
        inner = flags[:, 8:-8, 8:-8, 8:-8]
        frac = [(inner == v).mean() for v in (0, 1, 2)]
        print("interior flag fractions (low, WENO7, WENO5)", frac, flush=True)
        assert min(frac) > 1e-3
    nodes = np.unique(nodes)
    ref = orc.dudt_points(P, met, case.U0, nodes, flags=flags).T
    ref_pert = orc.dudt_points(P, met, ulp_perturbed(case.U0), nodes, flags=flags).T
    assert_within_roundoff(got[:, nodes], ref, ref_pert,
                           what=f"{case.name} {form} sampled dU/dt ({len(nodes)} nodes)")


def test_ramp_at_scale_hybrid_sampled(pk, torch_cuda, orc):
    """The ramp at its largest size (2048 x 256 x 256, 134 M points) with the
    plain FP64 hybrid (UD7 / WENO7, the GPU's own sensor) in the launch
    configuration the benchmark times: dU/dt at sampled nodes, some within
    six nodes of the faces, against the oracle node by node (its own sensor
    over the whole field).  Flags could differ only where theta lies within
    1e-12 of theta1 in a sampled node's windows; there are none here."""
    import dataclasses
    case = dataclasses.replace(workloads.compression_ramp(shape=(2048, 256, 256)), scheme="hybrid", lowdiss="ud7")
    ball = _ramp_noise_ball(case, np.random.default_rng(19), 40.0)
    print("case", case.name, "hybrid", flush=True)
    s = _solver(pk, torch_cuda, case)
    got = s.dudt(_dev(torch_cuda, case.U0)).cpu().numpy().reshape(5, -1)
    weno = np.array(s.reduce(case.dt))[9:12]
    s.close()
    del s
    torch_cuda.cuda.empty_cache()
    print("GPU WENO fractions", weno, flush=True)
    rng = np.random.default_rng(8)
    nodes = _ramp_sample(case, rng, 60, 30)
    # and nodes inside the ball, where WENO7 and low-dissipation interfaces mix
    nodes = np.unique(np.r_[nodes, rng.choice(np.flatnonzero(ball.reshape(-1) > 0.3), 60, replace=False)])
    P = orc.params_from_case(case, nthreads=0)
    met = orc.metrics(P, case.xyz)
    theta, flags = orc.sensor(P, case.U0)
    assert np.abs(theta - case.theta1).min() > 1e-12
    ref_frac = []
    for d, ax in enumerate((3, 2, 1)):
        n = case.U0.shape[ax]
        pos = np.arange(n).reshape([-1 if a == ax - 1 else 1 for a in range(3)])
        w = flags[d] != 0
        if not case.periodic[d]:
            exists = np.broadcast_to(pos < n - 1, w.shape)
            w = w | np.broadcast_to((pos < 3) | (pos > n - 5), w.shape)
        else:
            exists = np.ones_like(w)
        ref_frac.append((w & exists).sum() / exists.sum())
    print("oracle WENO fractions", ref_frac, flush=True)
    assert np.allclose(weno, ref_frac, rtol=1e-15, atol=0)
    assert min(ref_frac) > 0.005   # interior WENO7 interfaces in every direction
    del theta
    ref = orc.dudt_points(P, met, case.U0, nodes, flags=flags).T
    ref_pert = orc.dudt_points(P, met, ulp_perturbed(case.U0), nodes, flags=flags).T
    assert_within_roundoff(got[:, nodes], ref, ref_pert, what=f"{case.name} hybrid sampled dU/dt ({len(nodes)} nodes)")
