"""Writes c2_long_runs.json: the oracle's 256^3 runs of the configuration
"isentropic vortex + Taylor-Green on distorted periodic grids" at their stated
lengths (vortex 198 substeps, i.e. 66 whole Runge-Kutta steps, so the exact
translated solution applies; Taylor-Green 200 substeps).

Only the oracle and the seeded input generators are called.  Stored per run:
the per-field sums of U/J (conservation), the per-field L2 norms, four random
projections of every field (workloads.projection_weights: a whole-field
comparison, since r.(a - b) has the spread of |a - b|), the state at 1024
sampled nodes (workloads.sample_nodes), and for the vortex the per-field L2
error of the oracle against the exact translated solution.

Also stored: the projections of the oracle's run from the state moved by
about one unit in the last place, whose difference from the projections above
is the oracle's own rounding sensitivity over the run.

Run:  python tests/golden/make_c2_long_runs.py [threads] [vortex|taylor_green|vortex_ulp|taylor_green_ulp]
(about two hours on 8 cores; with a part named, only that part is redone and
the rest is kept from the existing file)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))     # tests/ (helpers.ulp_perturbed)

import numpy as np

import oracle
from oracle import exact
import workloads


def projections(U, weights):
    """[k][m] = sum over nodes of r_k * U_m, accumulated in extended precision."""
    out = []
    for r in weights:
        rl = r.astype(np.longdouble)
        out.append([float(np.sum(rl * U[m].reshape(-1).astype(np.longdouble))) for m in range(5)])
    return out


def norms(U):
    """Per-field L2 norms; the three momentum fields share the momentum vector's."""
    f = U.reshape(5, -1)
    mom = float(np.sqrt(np.sum(f[1:4] ** 2)))
    return [float(np.sqrt(np.sum(f[0] ** 2))), mom, mom, mom, float(np.sqrt(np.sum(f[4] ** 2)))]


def run(case, substeps, threads, exact_fn=None):
    P = oracle.params_from_case(case, nthreads=threads)
    met = oracle.metrics(P, case.xyz)
    t0 = time.perf_counter()
    U, _, stage = oracle.advance(P, met, case.U0, substeps, case.dt)
    el = time.perf_counter() - t0
    print(f"{case.name}: {substeps} substeps in {el:.0f} s", flush=True)
    red = oracle.reduce(P, met, U)
    red0 = oracle.reduce(P, met, case.U0)
    N = case.N
    w = workloads.projection_weights(N)
    nodes = workloads.sample_nodes(N)
    out = {"workload": case.name, "shape": [case.nx, case.ny, case.nz], "dt": case.dt, "substeps": substeps,
           "stage_after": stage, "sum_over_J_initial": [float(v) for v in red0[:5]],
           "sum_over_J": [float(v) for v in red[:5]], "l2_norms": norms(U),
           "projections": projections(U, w), "sample_nodes": nodes.tolist(),
           "sample_values": U.reshape(5, -1)[:, nodes].T.tolist(), "oracle_seconds": round(el, 1)}
    if exact_fn is not None:
        # one substep is one Runge-Kutta stage: time advances by dt per whole step of three
        assert substeps % 3 == 0
        t = (substeps // 3) * case.dt
        ref = exact_fn(case, t)
        d = (U - ref).reshape(5, -1)
        nr = norms(ref)
        out["exact_time"] = t
        out["rel_l2_error_vs_exact"] = [float(np.sqrt(np.sum(d[m] ** 2)) / nr[m]) for m in range(5)]
    return out


def ulp_projections(case, substeps, threads):
    """Projections of the oracle's run from the state moved by about one unit
    in the last place (tests/helpers.ulp_perturbed): their difference from the
    unperturbed run's projections is the oracle's own rounding sensitivity
    over the run."""
    from helpers import ulp_perturbed
    P = oracle.params_from_case(case, nthreads=threads)
    met = oracle.metrics(P, case.xyz)
    t0 = time.perf_counter()
    U, _, _ = oracle.advance(P, met, ulp_perturbed(case.U0), substeps, case.dt)
    print(f"{case.name} (one-ulp perturbed): {substeps} substeps in {time.perf_counter() - t0:.0f} s", flush=True)
    return projections(U, workloads.projection_weights(case.N))


def vortex_exact(case, t):
    rho, u, v, p = exact.isentropic_vortex(case.xyz[0], case.xyz[1], t)
    g = case.gamma
    return np.stack([rho, rho * u, rho * v, np.zeros_like(rho), p / (g - 1.0) + 0.5 * rho * (u * u + v * v)])


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    only = sys.argv[2] if len(sys.argv) > 2 else None     # "vortex" or "taylor_green": redo that run only
    path = os.path.join(HERE, "c2_long_runs.json")
    res = {"generator": "tests/golden/make_c2_long_runs.py (oracle only)"}
    if only and os.path.exists(path):
        with open(path) as f:
            res = json.load(f)
    if only in (None, "vortex"):
        vx = workloads.isentropic_vortex(256, distorted=True)
        res["vortex"] = run(vx, 198, threads, vortex_exact)
        del vx
    if only in (None, "taylor_green"):
        tg = workloads.taylor_green(256, distorted=True)
        res["taylor_green"] = run(tg, 200, threads)
    for name in ("vortex", "taylor_green"):
        if only in (None, name + "_ulp"):
            case = workloads.isentropic_vortex(256, distorted=True) if name == "vortex" else \
                workloads.taylor_green(256, distorted=True)
            res[name]["projections_ulp_perturbed"] = ulp_projections(case, res[name]["substeps"], threads)
            del case
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
