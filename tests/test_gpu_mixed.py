"""Mixed-precision form: Steger-Warming split, smoothness indicators and
reconstruction in FP32, flux difference / viscous terms / RK accumulation /
reductions in FP64.  Bar: per-field relative L2 drift <= 1e-5 against the FP64
oracle after 100 substeps, conserved totals held to FP64 roundoff."""
import numpy as np
import pytest

import workloads
from helpers import rel_errors

pytestmark = pytest.mark.gpu

TOL_DRIFT = 1e-5


@pytest.fixture(scope="module")
def pk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_15333_amd as pk
    pk.lib()
    return pk


def _run(pk, case, n):
    import torch
    s = pk.Solver(pk.params_from(case))
    s.set_grid(torch.from_numpy(case.xyz).cuda())
    s.set_state(torch.from_numpy(case.U0).cuda())
    r0 = np.array(s.reduce(case.dt))
    s.advance(n, case.dt)
    r1 = np.array(s.reduce(case.dt))
    return s.state().cpu().numpy(), r0, r1


# tgv-hybrid-ragged: every line length leaves a partial last chunk of 16
# nodes (36 = 2 x 16 + 4 along xi, whose Runge-Kutta sweep loads whole
# aligned blocks); tgv-narrow: fewer xi nodes than one chunk
@pytest.mark.parametrize("which", ["tgv32", "vortex", "tgv-hybrid", "tgv-hybrid-ragged", "tgv-narrow"])
def test_mixed_drift_vs_fp64_oracle(pk, orc, which):
    if which == "tgv32":
        case = workloads.taylor_green(32)
    elif which == "vortex":
        case = workloads.isentropic_vortex(shape=(48, 40, 8), distorted=True, dt=0.02)
    elif which == "tgv-narrow":
        case = workloads.taylor_green(shape=(12, 24, 20), distorted=True, dt=1e-3)
    else:
        shape = (32, 24, 20) if which == "tgv-hybrid" else (36, 20, 12)
        case = workloads.taylor_green(shape=shape, distorted=True, dt=1e-3)
        case.scheme = "hybrid"
    P = orc.params_from_case(case)
    met = orc.metrics(P, case.xyz)
    ref, _, _ = orc.advance(P, met, case.U0, 100, case.dt)
    case.precision = "mixed"
    got, r0, r1 = _run(pk, case, 100)
    l2, linf = rel_errors(got, ref)
    print(f"{which}: mixed vs FP64 oracle after 100 substeps: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_DRIFT)
    # the mixed form still conserves to FP64 roundoff
    assert abs(r1[0] - r0[0]) <= 1e-13 * abs(r0[0])
    assert abs(r1[4] - r0[4]) <= 1e-13 * abs(r0[4])


@pytest.mark.parametrize("which", ["tgv", "vortex"])
def test_mixed_full_size_drift(pk, which):
    """100 substeps of the 256^3 distorted workloads in the mixed form against
    the FP64 path (parity-checked against the oracle to 1e-12 elsewhere)."""
    case = (workloads.taylor_green(256, distorted=True) if which == "tgv"
            else workloads.isentropic_vortex(256, distorted=True))
    ref, _, _ = _run(pk, case, 100)
    case.precision = "mixed"
    got, r0, r1 = _run(pk, case, 100)
    l2, linf = rel_errors(got, ref)
    print(f"{which}256 mixed vs FP64 after 100 substeps: rel L2 {l2}, rel Linf {linf}", flush=True)
    assert np.all(l2 <= TOL_DRIFT)
    assert abs(r1[0] - r0[0]) <= 1e-13 * abs(r0[0])
    assert abs(r1[4] - r0[4]) <= 1e-13 * abs(r0[4])


@pytest.mark.parametrize("characteristic", [False, True])
def test_mixed_ramp_full_size_drift(pk, characteristic):
    """The compression ramp at the benchmark's size (1024 x 160 x 128, C8
    viscous terms, inflow, outflow and isothermal wall): 100 substeps of the
    FP32 form, component-wise and in characteristic variables, against the
    FP64 path of the same scheme."""
    import dataclasses
    import torch
    case = dataclasses.replace(workloads.compression_ramp(), characteristic=characteristic)

    def run(c):
        s = pk.Solver(pk.params_from(c))
        s.set_grid(torch.from_numpy(c.xyz).cuda())
        s.set_state(torch.from_numpy(c.U0).cuda())
        s.set_inflow(torch.from_numpy(np.ascontiguousarray(c.inflow)).cuda())
        s.advance(100, c.dt)
        out = s.state().cpu().numpy()
        s.close()
        del s
        torch.cuda.empty_cache()
        return out

    ref = run(case)
    got = run(dataclasses.replace(case, precision="mixed"))
    assert np.all(np.isfinite(got))
    l2, linf = rel_errors(got, ref)
    print(f"ramp mixed (characteristic {characteristic}) vs FP64 after 100 substeps: rel L2 {l2}, rel Linf {linf}",
          flush=True)
    assert np.all(l2 <= TOL_DRIFT)
