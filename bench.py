"""Throughput of the FP64 path on one MI355X, in grid-point substeps per second.

Workload: the plain FP64 method on two 256^3 periodic grids distorted by a
sinusoidal mapping (amplitude 0.1 h, seeded phases): the Taylor-Green vortex
(Re 1600, M 0.1, WENO7 + sixth-order viscous terms) and the isentropic
vortex (strength 5, advection (1,1,0), M 0.5, Euler).  One benchmark step is
one Runge-Kutta substep of each of the two runs.  Inputs are synthetic and
already resident in HBM when the timed region starts.

Prints one JSON line.  The dominant kernel's duration comes from HIP events
the library records around every launch on its stream during the timed
region; the CPU baseline is the oracle on a bounded sample (one substep of
each 256^3 run on the host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 flops per grid point of one launch, counted from the formulas of the
# method (add, multiply, divide and square root count one each; an FMA two).
FLOPS_PRIM = 15          # rho, u, v, w, p and c of a node
FLOPS_SW = 92            # Steger-Warming split of a node, both signs
FLOPS_WENO7 = 143        # one seventh-order WENO reconstruction
FLOPS_IFACE = 10 * FLOPS_WENO7 + 5
FLOPS_DIFF = 10          # flux difference of the five components
FLOPS_MODE = {"set": 0, "add": 5, "rk": 30}
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector
HBM_PEAK_GBS = 8000.0

# HBM counters of the dominant kernel in the default configuration (FP64,
# 256^3), per launch averaged over both runs, from the rocprofv3 --pmc runs
# summarised in profiles/fp64_weno7_headline_256cube.md.  A 512 MiB device copy
# reads FETCH_SIZE = 256 MiB and WRITE_SIZE = 512 MiB, so bytes fetched are
# 2 x FETCH_SIZE.  Valid for the kernel as committed with that file; other
# configurations report null.
PMC_TRAFFIC = {"sweep_xi": {"fetch_kib": 1473148, "write_kib": 665600}}


def sweep_flops(mode: str) -> int:
    return FLOPS_PRIM + FLOPS_SW + FLOPS_IFACE + FLOPS_DIFF + FLOPS_MODE[mode]


def make_cases(n: int):
    import workloads
    return [workloads.taylor_green(n, distorted=True), workloads.isentropic_vortex(n, distorted=True)]


def cpu_baseline(cases, threads: int):
    """The oracle, unchanged, on one substep of each run (metrics excluded)."""
    import oracle
    total_pts, total_t = 0, 0.0
    for c in cases:
        P = oracle.params_from_case(c, nthreads=threads)
        met = oracle.metrics(P, c.xyz)
        t0 = time.perf_counter()
        oracle.advance(P, met, c.U0, 1, c.dt)
        total_t += time.perf_counter() - t0
        total_pts += c.N
        del met
    # the same oracle on one core, on a smaller sample of the same kind
    import workloads
    small = workloads.taylor_green(96, distorted=True)
    P = oracle.params_from_case(small, nthreads=1)
    met = oracle.metrics(P, small.xyz)
    t0 = time.perf_counter()
    oracle.advance(P, met, small.U0, 1, small.dt)
    t1 = time.perf_counter() - t0
    return {"value": total_pts / total_t / 1e9, "unit": "Gpt-substeps/s", "cores": threads, "kind": "oracle",
            "sample": f"one substep of each of the {len(cases)} runs at full size ({total_pts} point-substeps), "
                      f"{total_t:.1f} s",
            "single_core": {"value": small.N / t1 / 1e9, "cores": 1,
                            "sample": f"one substep of the distorted Taylor-Green vortex at 96^3 ({small.N} "
                                      f"point-substeps), {t1:.1f} s"}}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rel_l2(torch, a, b):
    """Per-field relative L2 of a against b ([5, ...] device tensors); the
    momentum components share the norm of the momentum vector."""
    out = []
    mom = float(torch.linalg.vector_norm(b[1:4]))
    for m in range(5):
        d = float(torch.linalg.vector_norm(a[m] - b[m]))
        n = mom if 1 <= m <= 3 else float(torch.linalg.vector_norm(b[m]))
        out.append(d / n if n > 0 else d)
    return out


def _timed_run(torch, pk, case, U, substeps, warmup=2, setup=None):
    """A fresh solver for `case` started from state U: `warmup` substeps, then
    the state is set again and `substeps` substeps are timed.  Returns
    (Gpt-substeps/s, final state, solver)."""
    s = pk.Solver(pk.params_from(case))
    s.set_grid(torch.from_numpy(case.xyz).cuda())
    if case.inflow is not None:
        s.set_inflow(torch.from_numpy(case.inflow).cuda())
    if setup:
        setup(s)
    s.set_state(U)
    s.advance(warmup, case.dt)
    s.set_state(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(substeps, case.dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return case.N * substeps / el / 1e9, s.state(), s


def form_hit_learned(torch, pk, n, develop, every, substeps):
    """Decaying isotropic turbulence (hybrid WENO7 / C8): `develop` substeps of
    the plain FP64 hybrid with samples of the plain sensor's flags every
    `every` substeps over its last 40%, GPU training and calibration of the
    perceptron, then
    `substeps` substeps from the developed state with (i) WENO7 everywhere,
    FP64, (ii) the plain FP64 hybrid, (iii) FP32 reconstruction + learned
    sensor (re-evaluated every substep, audited every 50), (iv) the same with
    the network re-evaluated once per Runge-Kutta step.  The time step is
    twice the generator's default (CFL about 0.5).  At 512^3 the plain
    sensor marks its first interfaces near t = 0.5 (1400 substeps) and about
    0.24% of them at t = 0.9 (2500 substeps), where the forms are timed."""
    import dataclasses
    import workloads
    t_all = time.perf_counter()
    case = workloads.isotropic_turbulence(n)
    case.dt *= 2.0        # acoustic CFL ~0.5 (the generator's default is ~0.25)
    _log(f"hit{n}: inputs ready ({time.perf_counter() - t_all:.0f} s)")
    s = pk.Solver(pk.params_from(case))
    s.set_grid(torch.from_numpy(case.xyz).cuda())
    s.set_state(torch.from_numpy(case.U0).cuda())
    cap = 8_000_000
    buf = torch.empty(pk.ocfd_sensor_sample_bytes(cap), dtype=torch.uint8, device="cuda")
    pk.ocfd_sensor_bind_samples(s.h, buf)
    t0 = time.perf_counter()
    total = 0
    first = int(0.6 * develop)     # shocklets form late: sample the last 40% of the development
    for k in range(develop // every):
        s.advance(every, case.dt)
        if (k + 1) * every > first:
            total = pk.ocfd_sensor_collect(s.h, 5000 + k, 0.25, 0.0005)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    _log(f"hit{n}: developed {develop} substeps in {t_dev:.1f} s, {total} samples")
    pk.ocfd_sensor_set_params(s.h, workloads.sensor_initial_weights(11))
    t0 = time.perf_counter()
    stats = pk.ocfd_sensor_train(s.h, 4, 2048, 3e-3, 7, 0.1)
    cal = pk.ocfd_sensor_calibrate(s.h, 0.1, 0.5)
    t_train = time.perf_counter() - t0
    params = pk.ocfd_sensor_get_params(s.h)
    tau = cal[0]
    _log(f"hit{n}: trained in {t_train:.1f} s, loss {stats[0]:.4f} -> {stats[1]:.4f}, tau {tau:.3g}, "
         f"held-out recall {cal[1]}, false-positive rate {cal[2]:.4f}")
    U = s.state()
    del buf
    s.close()
    del s
    torch.cuda.empty_cache()

    def learned(sv):
        pk.ocfd_sensor_set_params(sv.h, params)
        pk.ocfd_sensor_set_threshold(sv.h, tau)

    res = {}
    ref = None
    for name, kw in (("weno7_fp64", dict(scheme="weno7")),
                     ("hybrid_plain_fp64", dict()),
                     ("hybrid_plain_fp32", dict(precision="mixed")),
                     ("hybrid_learned_fp32", dict(precision="mixed", sensor="learned", sensor_every=1,
                                                  audit_every=50)),
                     ("hybrid_learned_fp32_every3", dict(precision="mixed", sensor="learned", sensor_every=3,
                                                         audit_every=51))):
        c = dataclasses.replace(case, **kw)
        rate, Uf, sv = _timed_run(torch, pk, c, U, substeps, setup=learned if c.sensor == "learned" else None)
        entry = {"gpt_substeps_per_s": round(rate, 4)}
        if name == "hybrid_plain_fp64":
            ref = Uf
        elif ref is not None:
            entry["rel_l2_vs_plain_fp64_hybrid"] = [float(f"{e:.3e}") for e in _rel_l2(torch, Uf, ref)]
        if c.sensor == "learned":
            a = pk.ocfd_sensor_audit(sv.h)
            entry["audit"] = {"runs": int(a[0]), "plain_weno_frac": round(a[2] / max(a[1], 1), 5),
                              "learned_weno_frac": round(a[3] / max(a[1], 1), 5),
                              "missed_frac_of_plain_weno": round(a[4] / max(a[2], 1), 6),
                              "mismatch_rate": round(a[5] / max(a[1], 1), 6)}
        res[name] = entry
        _log(f"hit{n}: {name}: {entry}")
        sv.close()
        del sv, Uf
        torch.cuda.empty_cache()
    base = res["weno7_fp64"]["gpt_substeps_per_s"]
    plain = res["hybrid_plain_fp64"]["gpt_substeps_per_s"]
    for k in res:
        res[k]["speedup_vs_weno7_fp64"] = round(res[k]["gpt_substeps_per_s"] / base, 3)
        res[k]["speedup_vs_hybrid_plain_fp64"] = round(res[k]["gpt_substeps_per_s"] / plain, 3)
    return {"workload": f"decaying isotropic turbulence {n}^3 (k0 4, Mt 0.6, Re_lambda 100), C6 viscous, "
                        f"state after {develop} plain FP64 hybrid substeps; {substeps} timed substeps per form",
            "training": {"samples": total, "epochs": 4, "batch": 2048, "loss_first_last": [round(stats[0], 5),
                         round(stats[1], 5)], "tau": tau, "heldout_recall": cal[1],
                         "heldout_false_positive_rate": round(cal[2], 5), "train_s": round(t_train, 2)},
            "forms": res}


def learned_overhead(torch, pk, n, substeps):
    """Cost of the learned sensor on the Taylor-Green n^3 distorted run: FP32
    hybrid with the perceptron evaluated every substep, the output bias set to
    -30 so every interface takes the low-dissipation stencil (the sensor's own
    kernels are then the only difference from the plain hybrid)."""
    import dataclasses
    import workloads
    base = workloads.taylor_green(n, distorted=True)
    c = dataclasses.replace(base, scheme="hybrid", precision="mixed", sensor="learned", sensor_every=1)
    w = workloads.sensor_initial_weights(3)
    w[-1] = -30.0

    def setup(sv):
        pk.ocfd_sensor_set_params(sv.h, w)
        pk.ocfd_sensor_set_threshold(sv.h, 0.5)
    U = torch.from_numpy(base.U0).cuda()
    s = pk.Solver(pk.params_from(c))
    s.set_grid(torch.from_numpy(c.xyz).cuda())
    setup(s)
    s.set_state(U)
    s.advance(2, c.dt)
    torch.cuda.synchronize()
    pk.ocfd_profile(s.h, True)
    t0 = time.perf_counter()
    s.advance(substeps, c.dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = pk.ocfd_profile_read(s.h)
    pk.ocfd_profile(s.h, False)
    s.close()
    return {"workload": f"Taylor-Green {n}^3 distorted, FP32 hybrid, network every substep, all flags low",
            "gpt_substeps_per_s": round(c.N * substeps / el / 1e9, 4),
            "avg_launch_us": {k: round(v[0] / v[1] * 1e3, 1) for k, v in prof.items() if v[1]}}


def form_ramp_mixed(torch, pk, shape, substeps):
    """Compression ramp from the same inflow state, `substeps` substeps each:
    WENO7 FP64 and its FP32 split/reconstruction form, both again in
    characteristic variables, and the three-way hybrid in characteristic
    variables.  FP32 forms carry their relative L2 against the FP64 form of
    the same scheme."""
    import dataclasses
    import workloads
    case = workloads.compression_ramp(shape=shape)
    U = torch.from_numpy(case.U0).cuda()
    forms = (("weno7_fp64", dict(precision="fp64"), None),
             ("weno7_fp32", dict(precision="mixed"), "weno7_fp64"),
             ("weno7_char_fp64", dict(characteristic=True), None),
             ("weno7_char_fp32", dict(characteristic=True, precision="mixed"), "weno7_char_fp64"),
             ("hybrid3_char_fp64", dict(characteristic=True, scheme="hybrid", lowdiss="ud7", three_way=True), None))
    res = {}
    finals = {}
    for name, kw, vs in forms:
        c = dataclasses.replace(case, **kw)
        rate, Uf, sv = _timed_run(torch, pk, c, U, substeps)
        entry = {"gpt_substeps_per_s": round(rate, 4)}
        if vs is None:
            finals[name] = Uf
        else:
            entry[f"rel_l2_vs_{vs}"] = [float(f"{e:.3e}") for e in _rel_l2(torch, Uf, finals[vs])]
        if name != "weno7_fp64":
            entry["speedup_vs_weno7_fp64"] = round(rate / res["weno7_fp64"]["gpt_substeps_per_s"], 3)
        res[name] = entry
        _log(f"ramp: {name}: {entry}")
        sv.close()
        del sv
        torch.cuda.empty_cache()
    nx, ny, nz = shape
    return {"workload": f"Mach 2.9 24-degree compression ramp {nx}x{ny}x{nz}, inflow/outflow/isothermal wall "
                        f"Tw 2.84/periodic span, C8 viscous, Re_delta 5e4; {substeps} substeps from the inflow state",
            "forms": res}


def form_ramp_full(torch, pk, shape, train, substeps, report):
    """The ramp at scale with the full chosen form.  The plain FP64 hybrid
    (UD7 / WENO7, plain sensor) runs `train` substeps from the inflow state
    with the plain sensor's flags sampled every 50 substeps; the perceptron is
    trained and calibrated on the GPU (an unbiased sample of every snapshot,
    32 epochs).  Then, from the same inflow state, the plain FP64 hybrid and
    the FP32 + learned-sensor hybrid (network every substep, and once per
    Runge-Kutta step; audited every `report` substeps, union fallback) run
    `substeps` substeps each in turns of `report`; after every turn the
    per-field relative L2 of each learned form against the plain one and the
    audit rates of the turn are recorded.  Each form's time is the sum of its
    turns."""
    import dataclasses
    import workloads
    t_all = time.perf_counter()
    case = dataclasses.replace(workloads.compression_ramp(shape=shape), scheme="hybrid", lowdiss="ud7")
    nx, ny, nz = shape
    _log(f"ramp{nx}x{ny}x{nz}: inputs ready ({time.perf_counter() - t_all:.0f} s)")
    xyz = torch.from_numpy(case.xyz).cuda()
    inflow = torch.from_numpy(case.inflow).cuda()
    U0 = torch.from_numpy(case.U0).cuda()

    def solver(c):
        sv = pk.Solver(pk.params_from(c))
        sv.set_grid(xyz)
        sv.set_inflow(inflow)
        sv.set_state(U0)
        return sv
    s = solver(case)
    cap = 8_000_000
    buf = torch.empty(pk.ocfd_sensor_sample_bytes(cap), dtype=torch.uint8, device="cuda")
    pk.ocfd_sensor_bind_samples(s.h, buf)
    t0 = time.perf_counter()
    total = 0
    every = 50
    for k in range(train // every):
        s.advance(every, case.dt)
        # the same keep rate for both classes: an unbiased sample of every
        # snapshot, spread over the whole run (about 0.8 M per snapshot)
        total = pk.ocfd_sensor_collect(s.h, 9000 + k, 0.002, 0.002)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    pk.ocfd_sensor_set_params(s.h, workloads.sensor_initial_weights(13))
    t0 = time.perf_counter()
    epochs = 32
    stats = pk.ocfd_sensor_train(s.h, epochs, 2048, 3e-3, 9, 0.1)
    cal = pk.ocfd_sensor_calibrate(s.h, 0.1, 0.5)
    t_train = time.perf_counter() - t0
    params = pk.ocfd_sensor_get_params(s.h)
    tau = cal[0]
    _log(f"ramp{nx}x{ny}x{nz}: {train} plain substeps in {t_dev:.1f} s, {total} samples; trained in {t_train:.1f} s, "
         f"tau {tau:.3g}, held-out recall {cal[1]}, false-positive rate {cal[2]:.4f}")
    del buf
    s.close()
    del s
    torch.cuda.empty_cache()
    plain = solver(case)
    # the network every substep, and once per Runge-Kutta step (its flags
    # then hold for the step's three stages)
    learned = solver(dataclasses.replace(case, precision="mixed", sensor="learned", sensor_every=1,
                                         audit_every=report))
    learned3 = solver(dataclasses.replace(case, precision="mixed", sensor="learned", sensor_every=3,
                                          audit_every=report))
    for sv in (learned, learned3):
        pk.ocfd_sensor_set_params(sv.h, params)
        pk.ocfd_sensor_set_threshold(sv.h, tau)
    elapsed = {"p": 0.0, "l": 0.0, "l3": 0.0}
    turns = []
    prev = [0.0] * 6
    prev3 = [0.0] * 6
    for k in range(substeps // report):
        for sv, which in ((plain, "p"), (learned, "l"), (learned3, "l3")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sv.advance(report, case.dt)
            torch.cuda.synchronize()
            elapsed[which] += time.perf_counter() - t0
        a = pk.ocfd_sensor_audit(learned.h)
        d = [a[i] - prev[i] for i in range(6)]
        prev = a
        a3 = pk.ocfd_sensor_audit(learned3.h)
        d3 = [a3[i] - prev3[i] for i in range(6)]
        prev3 = a3
        red = plain.reduce(case.dt)
        turns.append({"substeps": (k + 1) * report,
                      "rel_l2_learned_fp32_vs_plain_fp64": [float(f"{e:.3e}") for e in
                                                            _rel_l2(torch, learned.state(), plain.state())],
                      "plain_weno_frac": round(d[2] / max(d[1], 1), 5),
                      "learned_weno_frac": round(d[3] / max(d[1], 1), 5),
                      "mismatch_rate": round(d[5] / max(d[1], 1), 6),
                      "missed_frac_of_plain_weno": round(d[4] / max(d[2], 1), 6),
                      "plain_weno_frac_by_direction": [round(v, 5) for v in red[9:12]],
                      "rel_l2_learned_per_step_fp32_vs_plain_fp64": [float(f"{e:.3e}") for e in
                                                                     _rel_l2(torch, learned3.state(), plain.state())],
                      "learned_per_step_weno_frac": round(d3[3] / max(d3[1], 1), 5),
                      "learned_per_step_missed_frac_of_plain_weno": round(d3[4] / max(d3[2], 1), 6)})
        _log(f"ramp{nx}x{ny}x{nz}: {turns[-1]}")
    rate_p = case.N * substeps / elapsed["p"] / 1e9
    rate_l = case.N * substeps / elapsed["l"] / 1e9
    rate_l3 = case.N * substeps / elapsed["l3"] / 1e9
    plain.close()
    learned.close()
    learned3.close()
    del plain, learned, learned3, xyz, inflow, U0
    torch.cuda.empty_cache()
    return {"workload": f"Mach 2.9 24-degree compression ramp {nx}x{ny}x{nz} ({case.N} points), C8 viscous, "
                        f"hybrid UD7 / WENO7 from the inflow state; {substeps} substeps per form",
            "training": {"plain_substeps": train, "samples": total, "epochs": epochs, "batch": 2048,
                         "loss_first_last": [round(stats[0], 5), round(stats[1], 5)], "tau": tau,
                         "heldout_recall": cal[1], "heldout_false_positive_rate": round(cal[2], 5),
                         "train_s": round(t_train, 2)},
            "forms": {"hybrid_plain_fp64": {"gpt_substeps_per_s": round(rate_p, 4)},
                      "hybrid_learned_fp32": {"gpt_substeps_per_s": round(rate_l, 4),
                                              "speedup_vs_hybrid_plain_fp64": round(rate_l / rate_p, 3)},
                      "hybrid_learned_per_step_fp32": {"gpt_substeps_per_s": round(rate_l3, 4),
                                                       "speedup_vs_hybrid_plain_fp64": round(rate_l3 / rate_p, 3)}},
            "every_100_substeps": turns}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="grid points per direction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="fp64: the plain path; mixed: FP32 split/reconstruction, FP64 difference and RK")
    ap.add_argument("--learned-overhead", action="store_true",
                    help="also time the learned sensor's kernels on the 256^3 Taylor-Green run")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the isotropic-turbulence and compression-ramp form comparisons")
    ap.add_argument("--forms", choices=["all", "hit", "ramp", "ramp_full"], default="all",
                    help="which form comparisons to run (unless --no-forms)")
    ap.add_argument("--ramp-full-shape", type=str, default="2048,256,256")
    ap.add_argument("--ramp-full-substeps", type=int, default=1000)
    ap.add_argument("--hit-n", type=int, default=512)
    ap.add_argument("--hit-develop", type=int, default=2500,
                    help="plain FP64 hybrid substeps before the forms are timed (t ~ 0.9 at 512^3)")
    ap.add_argument("--form-substeps", type=int, default=100)
    ap.add_argument("--ramp-shape", type=str, default="1024,160,128")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 512 MiB device-to-device copy first, as the reference dispatch "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver keeps the whole domain on a single device; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_15333_amd as pk

    if args.calibration_copy:
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("[bench] calibration copy: 536870912 bytes read, 536870912 bytes written", file=sys.stderr, flush=True)

    cases = make_cases(args.n)
    for c in cases:
        c.precision = args.precision
    solvers = []
    for c in cases:
        s = pk.Solver(pk.params_from(c))
        s.set_grid(torch.from_numpy(c.xyz).cuda())
        s.set_state(torch.from_numpy(c.U0).cuda())
        solvers.append(s)
    torch.cuda.synchronize()
    print(f"[bench] {len(cases)} runs of {args.n}^3 ready", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        for s, c in zip(solvers, cases):
            s.advance(1, c.dt)
    torch.cuda.synchronize()
    for s in solvers:
        pk.ocfd_profile(s.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for s, c in zip(solvers, cases):
            s.advance(1, c.dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = [pk.ocfd_profile_read(s.h) for s in solvers]
    for s in solvers:
        pk.ocfd_profile(s.h, False)
    elapsed = t1 - t0
    pts = sum(c.N for c in cases) * args.steps
    value = pts / elapsed / 1e9
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # Dominant kernel class over both runs.
    tot = {}
    for p in prof:
        for k, (ms, cnt) in p.items():
            a = tot.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
    for k, (ms, cnt) in sorted(tot.items(), key=lambda kv: -kv[1][0]):
        if cnt:
            print(f"[bench] {k:14s} {ms / cnt * 1e3:9.1f} us/launch  {cnt:6d} launches  {ms:9.2f} ms",
                  file=sys.stderr, flush=True)
    dom = max((k for k in tot if k.startswith("sweep")), key=lambda k: tot[k][0])
    # The xi sweep (last) applies the Runge-Kutta update and eta accumulates;
    # zeta (first) stores the sum, or adds to the viscous divergence.
    flops_launch = {}
    for c, p in zip(cases, prof):
        ms, cnt = p[dom]
        mode = {"sweep_xi": "rk", "sweep_eta": "add", "sweep_zeta": "add" if c.viscous else "set"}[dom]
        flops_launch[c.name] = (sweep_flops(mode) * c.N, ms / cnt)
    total_flops = sum(f * 1 for f, _ in flops_launch.values())
    total_ms = sum(t for _, t in flops_launch.values())
    achieved = total_flops / (total_ms * 1e-3) / 1e12
    # The mixed form does the split and reconstruction (nearly all of a sweep's
    # flops) in FP32, so it is measured against the FP32 vector peak.
    peak = FP32_PEAK_TFLOPS if args.precision == "mixed" else FP64_PEAK_TFLOPS
    traffic = None
    if args.precision == "fp64" and args.n == 256 and dom in PMC_TRAFFIC:
        t = PMC_TRAFFIC[dom]
        traffic = 2 * t["fetch_kib"] * 1024 + t["write_kib"] * 1024
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
            "avg_launch_us": {k: round(v[1] * 1e3, 1) for k, v in flops_launch.items()},
            "flops_per_launch": {k: v[0] for k, v in flops_launch.items()}}

    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()
    overhead = learned_overhead(torch, pk, args.n, args.steps) if args.learned_overhead else None
    forms = None
    if not args.no_forms:
        forms = {}
        if args.forms in ("all", "hit"):
            forms["isotropic_turbulence"] = form_hit_learned(torch, pk, args.hit_n, args.hit_develop, 50,
                                                             args.form_substeps)
        if args.forms in ("all", "ramp"):
            forms["compression_ramp"] = form_ramp_mixed(torch, pk, tuple(int(v) for v in args.ramp_shape.split(",")),
                                                        args.form_substeps)
        if args.forms in ("all", "ramp_full"):
            forms["compression_ramp_at_scale"] = form_ramp_full(
                torch, pk, tuple(int(v) for v in args.ramp_full_shape.split(",")), 500, args.ramp_full_substeps, 100)

    cpu = None
    if not args.no_cpu_baseline:
        print(f"[bench] oracle baseline on {args.cpu_threads} threads", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cases, args.cpu_threads)

    out = {
        "metric": "Gpt-substeps/s: plain FP64 vs FP32+learned-sensor form at stated L2 error",
        "value": round(value, 4),
        "unit": "Gpt-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 split/reconstruction + f64 difference/RK",
        "data": "synthetic",
        "config": {"workload": f"isentropic vortex + Taylor-Green on {args.n}^3 distorted periodic grids, "
                               "SW + WENO7 + C6 viscous (TGV), RK3; one step = one substep of each",
                   "points_per_step": sum(c.N for c in cases), "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    if overhead is not None:
        out["learned_overhead"] = overhead
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
