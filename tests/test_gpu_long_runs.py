"""The 256^3 distorted-grid runs at their stated lengths against the oracle's
runs of the same inputs (stored by tests/golden/make_c2_long_runs.py, which
calls only the oracle and the seeded generators): the isentropic vortex 198
substeps (66 whole Runge-Kutta steps, so the exact translated solution of
the Euler equations applies; Sec. 2.4, eq 45) and the Taylor-Green vortex
200 substeps, in the launch configuration the benchmark times.

Whole-field comparison without moving 670 MB per field off the GPU machine's
oracle: four seeded random projections of every field (for a difference d
the projection r.d has the spread of the L2 norm of d), the per-field L2
norms, the conserved totals, and the state at 1024 sampled nodes.  The bar
is the FP64 path's: 1e-12 relative (the projections' spread allowed 5x), or
30x the oracle's own sensitivity to a one-ulp change of the initial state
over the same run where that is larger (stored beside the run).
The vortex's error against its exact translated solution is reported beside
the oracle's own.
"""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "c2_long_runs.json")


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


@pytest.fixture(scope="module")
def gold():
    if not os.path.exists(GOLD):
        pytest.skip("tests/golden/c2_long_runs.json not generated")
    with open(GOLD) as f:
        return json.load(f)


def _norms(torch, U):
    f = U.reshape(5, -1)
    mom = float(torch.linalg.vector_norm(f[1:4]))
    return [float(torch.linalg.vector_norm(f[0])), mom, mom, mom, float(torch.linalg.vector_norm(f[4]))]


def _run(pk, torch, case, substeps):
    s = pk.Solver(pk.params_from(case))
    s.set_grid(torch.from_numpy(case.xyz).cuda())
    s.set_state(torch.from_numpy(case.U0).cuda())
    s.advance(substeps, case.dt)
    U = s.state()
    red = s.reduce(case.dt)
    s.close()
    return U, red


@pytest.mark.parametrize("which", ["vortex", "taylor_green"])
def test_c2_run_at_stated_length(pk, torch_cuda, gold, which):
    torch = torch_cuda
    g = gold[which]
    case = workloads.isentropic_vortex(256, distorted=True) if which == "vortex" else \
        workloads.taylor_green(256, distorted=True)
    assert [case.nx, case.ny, case.nz] == g["shape"] and case.dt == g["dt"]
    print(f"{which}: {g['substeps']} substeps on the GPU", flush=True)
    U, red = _run(pk, torch, case, g["substeps"])
    norms = _norms(torch, U)
    # conserved totals and L2 norms
    # 1/J is about 1 on these grids (computational spacing = nominal physical
    # spacing); the momentum components share the momentum vector's scale (w = 0)
    for m in range(5):
        scale = np.abs(case.U0[1:4]).sum() if 1 <= m <= 3 else np.abs(case.U0[m]).sum()
        assert abs(red[m] - g["sum_over_J"][m]) <= 1e-12 * scale, m
        assert abs(norms[m] - g["l2_norms"][m]) <= 1e-12 * g["l2_norms"][m], m
    # random projections: whole-field difference, against the 1e-12 bar (the
    # projections' spread allowed 5x) or, where rounding grows over the run,
    # 30x the oracle's own one-ulp sensitivity over the same run
    w = workloads.projection_weights(case.N)
    Uf = U.reshape(5, -1)
    ulp = g.get("projections_ulp_perturbed")
    # the oracle's own sensitivity: its run from the state perturbed by one
    # ulp, as the largest relative projection difference over fields
    sens_max = max(abs(ulp[k][m] - g["projections"][k][m]) / g["l2_norms"][m]
                   for k in range(len(w)) for m in range(5)) if ulp else 0.0
    worst = 0.0
    for k, r in enumerate(w):
        rt = torch.from_numpy(r).cuda()
        for m in range(5):
            got = float(torch.dot(rt, Uf[m]))
            err = abs(got - g["projections"][k][m]) / g["l2_norms"][m]
            sens = abs(ulp[k][m] - g["projections"][k][m]) / g["l2_norms"][m] if ulp else 0.0
            worst = max(worst, err)
            assert err <= max(5e-12, 30.0 * sens), (k, m, err, sens)
        del rt
    # sampled nodes
    nodes = torch.from_numpy(np.array(g["sample_nodes"], dtype=np.int64)).cuda()
    got = Uf[:, nodes].T.cpu().numpy()
    ref = np.array(g["sample_values"])
    scale = np.abs(ref).max(axis=0)
    scale[1:4] = np.abs(ref[:, 1:4]).max()          # the momentum vector's scale (w = 0 in these flows)
    samp = (np.abs(got - ref) / scale).max()
    print(f"{which}: worst projection difference / norm {worst:.2e}, sampled nodes {samp:.2e}, "
          f"oracle one-ulp sensitivity {sens_max:.2e}", flush=True)
    # sampled nodes against the same bar: 1e-11, or 30x the oracle's own
    # sensitivity where rounding grows over the run (the Taylor-Green run:
    # a one-ulp change of the initial state moves the oracle's projections
    # by up to 1.6e-11 of the norm after 200 substeps)
    assert samp <= max(1e-11, 30.0 * sens_max)
    if which == "vortex":
        from oracle import exact
        t = g["exact_time"]          # (substeps / 3) dt: a substep is one Runge-Kutta stage
        rho, u, v, p = exact.isentropic_vortex(case.xyz[0], case.xyz[1], t)
        gm = case.gamma
        ex = np.stack([rho, rho * u, rho * v, np.zeros_like(rho), p / (gm - 1.0) + 0.5 * rho * (u * u + v * v)])
        Uc = U.cpu().numpy()
        d = (Uc - ex).reshape(5, -1)
        exn = ex.reshape(5, -1)
        mom = np.sqrt((exn[1:4] ** 2).sum())
        nr = [np.sqrt((exn[0] ** 2).sum()), mom, mom, mom, np.sqrt((exn[4] ** 2).sum())]
        err = [float(np.sqrt((d[m] ** 2).sum()) / nr[m]) for m in range(5)]
        print(f"vortex at t = {t}: rel L2 error vs the exact translated solution, GPU {err}, "
              f"oracle {g['rel_l2_error_vs_exact']}", flush=True)
        for m in (0, 1, 2, 4):
            assert abs(err[m] - g["rel_l2_error_vs_exact"][m]) <= 1e-6 * g["rel_l2_error_vs_exact"][m] + 1e-12
