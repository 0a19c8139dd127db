"""Throughput of the hot path on one MI355X, in grid-point substeps per second.

Headline: the Mach 2.9 compression ramp on a 2048 x 256 x 256 body-fitted grid
(134 M points), the plain FP64 hybrid (UD7 / WENO7 with the pressure sensor
of eq 42-43) against the FP32 split/reconstruction form with the learned
sensor trained in-run from the plain sensor's flags, on the identical seeded
grid and inflow state.  `value` is the FP32 + learned form's throughput; the
plain FP64 rate, the ratio and the learned form's per-field relative L2
against the plain one after the timed substeps sit beside it.  Inputs are
synthetic and resident in HBM when the timed region starts.

The dominant kernel's duration comes from HIP events the library records
around every launch on its stream during the timed region.  The CPU baseline
is the oracle on a bounded slab of the same workload.  Further comparisons
(the 256^3 FP64 WENO7 runs, isotropic turbulence 512^3, the 1024 x 160 x 128
ramp) follow under `forms`.

Prints one JSON line.
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
FLOPS_IFACE_LOW = 5 * 27 + 5   # one linear-stencil interface (UD7 of both signs), five components
FLOPS_DIFF = 10          # flux difference of the five components
FLOPS_MODE = {"set": 0, "add": 5, "rk": 30}
# The paper-style manual count (its Table 6 convention): Steger-Warming split
# of a node, one WENO7 and one linear-stencil reconstruction, the RK update.
FLOPS_COUNT_SW = 140
FLOPS_COUNT_WENO = 200
FLOPS_COUNT_LOW = 15
FLOPS_COUNT_RK = 21
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
# The same for the xi Runge-Kutta hybrid sweeps of the ramp at 2048x256x256,
# FP64 and FP32 split/reconstruction (profiles/ramp_headline_2048x256x256.md;
# its 5.37 GB state copy gives the same factors).
PMC_TRAFFIC_RAMP = {"fp64": {"fetch_kib": 15979708, "write_kib": 5242880},
                    "mixed": {"fetch_kib": 11954710, "write_kib": 5242880}}


def make_cases(n: int):
    import workloads
    return [workloads.taylor_green(n, distorted=True), workloads.isentropic_vortex(n, distorted=True)]


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
    case.sensor_inputs = "curv"
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
    taus = pk.ocfd_sensor_get_thresholds(s.h)
    _log(f"hit{n}: trained in {t_train:.1f} s, loss {stats[0]:.4f} -> {stats[1]:.4f}, tau {tau:.3g}, "
         f"held-out recall {cal[1]}, false-positive rate {cal[2]:.4f}")
    U = s.state()
    del buf
    s.close()
    del s
    torch.cuda.empty_cache()

    def learned(sv):
        pk.ocfd_sensor_set_params(sv.h, params)
        pk.ocfd_sensor_set_thresholds(sv.h, taus)

    res = {}
    ref = None
    for name, kw in (("weno7_fp64", dict(scheme="weno7")),
                     ("hybrid_plain_fp64", dict()),
                     ("hybrid_plain_fp32", dict(precision="mixed")),
                     ("hybrid_learned_fp32", dict(precision="mixed", sensor="learned", sensor_every=1,
                                                  audit_every=50)),
                     ("hybrid_learned_fp32_every3", dict(precision="mixed", sensor="learned", sensor_every=3,
                                                         audit_every=51)),
                     ("hybrid_learned_fp32_every6", dict(precision="mixed", sensor="learned", sensor_every=6,
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
                         round(stats[1], 5)], "tau": tau, "tau_by_direction": taus, "heldout_recall": cal[1],
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


def _prof_avg_us(prof):
    return {k: round(v[0] / v[1] * 1e3, 1) for k, v in prof.items() if v[1]}


def _sweep_roofline(prof, N, weno_frac, mixed, hybrid=True, viscous=True, last_dir=0):
    """Roofline entry of the sweep class with the largest time in `prof`
    (ocfd_profile_read of a timed region).

    Flops per node of a sweep launch by the paper-style manual count (its
    Sec. 5.4, Table 6 convention: an FMA counts two): 140 for the
    Steger-Warming split, 10 reconstructions of 200 (WENO7) or 15 (linear
    stencil) flops, 21 for the Runge-Kutta update in the last sweep;
    weno_frac[d] is the WENO fraction of direction d's interfaces.
    Algorithmic bytes per node (each array once): U 40, the metric row 24,
    the sum of the earlier sweeps 40 (accumulating and last sweeps), in the
    last sweep U^n 40 x 2/3 (stages 2 and 3) and 1/J 8; hybrid sweeps read
    their viscous-flux row 32 and one flag byte; every sweep writes 40.  The
    binding roof is the one the algorithmic work reaches first: FP64 (or FP32)
    vector flops or HBM bytes.  The design-count flop figure (every operation
    as computed) is kept beside it."""
    sweeps = [k for k in prof if k.startswith("sweep") and prof[k][1]]
    dom = max(sweeps, key=lambda k: prof[k][0])
    d = {"sweep_xi": 0, "sweep_eta": 1, "sweep_zeta": 2}[dom]
    phi = float(weno_frac[d])
    rk = d == last_dir
    first = d == 2
    flops = FLOPS_COUNT_SW + 10 * (FLOPS_COUNT_LOW + (FLOPS_COUNT_WENO - FLOPS_COUNT_LOW) * phi) + \
        (FLOPS_COUNT_RK if rk else 0)
    design = FLOPS_PRIM + FLOPS_SW + phi * FLOPS_IFACE + (1.0 - phi) * FLOPS_IFACE_LOW + FLOPS_DIFF + \
        FLOPS_MODE["rk" if rk else "add"]
    vdiv = viscous and not hybrid and not mixed      # the first sweep adds onto the viscous divergence
    nbytes = 40 + 24 + 40                             # U, metric row; output
    nbytes += 40 if (not first or vdiv) else 0        # the sum of the earlier sweeps
    nbytes += (40 * 2 / 3 + 8) if rk else 0           # U^n (stages 2, 3), 1/J
    nbytes += 32 if (viscous and (hybrid or mixed)) else 0   # this direction's viscous-flux row
    nbytes += 1 if hybrid else 0                      # interface flag
    ms, cnt = prof[dom]
    t = ms / cnt * 1e-3
    peak = FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
    t_alu = flops * N / (peak * 1e12)
    t_hbm = nbytes * N / (HBM_PEAK_GBS * 1e9)
    out = {"kernel": dom, "avg_launch_us": round(t * 1e6, 1), "weno_frac": round(phi, 4),
           "flops_per_node": round(flops, 1), "bytes_per_node": round(nbytes, 1),
           "alu_frac": round(t_alu / t, 4), "hbm_frac": round(t_hbm / t, 4),
           "frac_design_count": round(design * N / t / 1e12 / peak, 4),
           "flops_per_node_design_count": round(design, 1), "traffic": None}
    if t_hbm > t_alu:
        out.update({"bound": "hbm", "achieved": round(nbytes * N / t / 1e9, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(t_hbm / t, 4)})
    else:
        out.update({"bound": "alu", "achieved": round(flops * N / t / 1e12, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(t_alu / t, 4)})
    return out


def headline_ramp(torch, pk, shape, train, epochs, steps, warmup, report=100):
    """The ramp at scale: plain FP64 hybrid (UD7 / WENO7, plain sensor) against
    the FP32 + learned-sensor hybrid on the identical seeded grid and inflow
    state.  The plain FP64 hybrid runs `train` substeps from the inflow state
    with an unbiased sample of the plain sensor's flags every 50 substeps; the
    perceptron is trained (`epochs` passes) and calibrated on the GPU.  Then
    each form runs `warmup` substeps from the inflow state and is reset to
    it, and both march `steps` substeps in turns of `report`, each turn timed
    (kernel classes by the library's HIP events on the solver's stream).
    After every turn: the learned form's per-field relative L2 against the
    plain one, both forms' WENO fractions per direction and the learned
    sensor's audit of that turn."""
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
    # two sample sets from the same plain run: node features with the plain
    # sensor's second differences as the pressure / density inputs ("curv",
    # the headline form) and with first differences ("jump")
    s = solver(dataclasses.replace(case, sensor_inputs="curv"))
    sj = solver(dataclasses.replace(case, sensor_inputs="jump"))
    cap = 8_000_000
    bufs = []
    for sv in (s, sj):
        bufs.append(torch.empty(pk.ocfd_sensor_sample_bytes(cap), dtype=torch.uint8, device="cuda"))
        pk.ocfd_sensor_bind_samples(sv.h, bufs[-1])
    t0 = time.perf_counter()
    total = 0
    every = 50
    for k in range(train // every):
        s.advance(every, case.dt)
        # the same keep rate for both classes: an unbiased sample of every
        # snapshot, spread over the whole run
        total = pk.ocfd_sensor_collect(s.h, 9000 + k, 0.002, 0.002)
        sj.set_state(s.state())
        pk.ocfd_sensor_collect(sj.h, 9000 + k, 0.002, 0.002)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    # WENO fraction of the developed state under both readings of the sensor window
    win = {"stencil_j-3..j+4": [round(v, 5) for v in s.reduce(case.dt)[9:12]]}
    alt = pk.Solver(pk.params_from(case, flag_window=1))
    alt.set_grid(xyz)
    fl = torch.empty((3,) + tuple(U0.shape[1:]), dtype=torch.uint8, device="cuda")
    pk.ocfd_sensor_flags(alt.h, s.state(), pk.OCFD_SENSOR_PLAIN, fl)
    win["nodes_j,j+1"] = [round(float(fl[d].float().mean()), 5) for d in range(3)]
    alt.close()
    del alt, fl
    nets = {}
    for key, sv in (("curv", s), ("jump", sj)):
        pk.ocfd_sensor_set_params(sv.h, workloads.sensor_initial_weights(13))
        t0 = time.perf_counter()
        stats = pk.ocfd_sensor_train(sv.h, epochs, 2048, 3e-3, 9, 0.1)
        cal = pk.ocfd_sensor_calibrate(sv.h, 0.1, 0.5)
        t_train = time.perf_counter() - t0
        nets[key] = {"params": pk.ocfd_sensor_get_params(sv.h), "taus": pk.ocfd_sensor_get_thresholds(sv.h),
                     "info": {"samples": total, "epochs": epochs, "batch": 2048,
                              "loss_first_last": [round(stats[0], 5), round(stats[1], 5)],
                              "tau_by_direction": pk.ocfd_sensor_get_thresholds(sv.h), "heldout_recall": cal[1],
                              "heldout_false_positive_rate": round(cal[2], 5), "train_s": round(t_train, 2)}}
        _log(f"ramp{nx}x{ny}x{nz}: {key} inputs: trained in {t_train:.1f} s, taus {nets[key]['taus']}, "
             f"held-out recall {cal[1]}, false-positive rate {cal[2]:.4f}")
    _log(f"ramp{nx}x{ny}x{nz}: {train} plain substeps in {t_dev:.1f} s, {total} samples; WENO fractions {win}")
    del bufs
    s.close()
    sj.close()
    del s, sj
    torch.cuda.empty_cache()
    # the network every second RK step (6 substeps); beside it the same network
    # once per RK step, and first-difference inputs
    learned_case = dataclasses.replace(case, precision="mixed", sensor="learned", sensor_every=6,
                                       audit_every=report, sensor_inputs="curv")
    cases = {"plain_fp64": case, "learned_fp32": learned_case,
             "learned_fp32_every3": dataclasses.replace(learned_case, sensor_every=3),
             "learned_fp32_jump": dataclasses.replace(learned_case, sensor_inputs="jump")}
    learned = [name for name in cases if name != "plain_fp64"]
    solvers = {}
    for name, c in cases.items():
        sv = solver(c)
        if c.sensor == "learned":
            net = nets[c.sensor_inputs]
            pk.ocfd_sensor_set_params(sv.h, net["params"])
            pk.ocfd_sensor_set_thresholds(sv.h, net["taus"])
        sv.advance(warmup, c.dt)
        sv.set_state(U0)
        solvers[name] = sv
    torch.cuda.synchronize()
    # both forms march in turns of `report` substeps; each turn is timed on its
    # own (kernel classes by the library's HIP events), the comparisons
    # between turns are not
    elapsed = {name: 0.0 for name in cases}
    fracs = {name: [] for name in cases}
    turns = []
    prev = {name: pk.ocfd_sensor_audit(solvers[name].h) for name in learned}
    for sv in solvers.values():
        pk.ocfd_profile(sv.h, True)
    done = 0
    while done < steps:
        n = min(report, steps - done)
        for name, sv in solvers.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sv.advance(n, case.dt)
            torch.cuda.synchronize()
            elapsed[name] += time.perf_counter() - t0
        done += n
        red = {name: sv.reduce(case.dt) for name, sv in solvers.items()}
        for name in cases:
            fracs[name].append(red[name][9:12])
        turn = {"substeps": done,
                "plain_weno_frac_by_direction": [round(v, 5) for v in red["plain_fp64"][9:12]]}
        for name in learned:
            a = pk.ocfd_sensor_audit(solvers[name].h)
            dlt = [a[i] - prev[name][i] for i in range(6)]
            prev[name] = a
            # the audit of a turn runs at its first substep (a multiple of `report`)
            turn[name] = {"rel_l2_vs_plain_fp64": [float(f"{e:.3e}") for e in _rel_l2(
                              torch, solvers[name].state(), solvers["plain_fp64"].state())],
                          "weno_frac_by_direction": [round(v, 5) for v in red[name][9:12]],
                          "audit_at_substep": done - n,
                          "audit_plain_weno_frac": round(dlt[2] / max(dlt[1], 1), 5),
                          "audit_learned_weno_frac": round(dlt[3] / max(dlt[1], 1), 5),
                          "audit_mismatch_rate": round(dlt[5] / max(dlt[1], 1), 6),
                          "audit_missed_frac_of_plain_weno": round(dlt[4] / max(dlt[2], 1), 6)}
        turns.append(turn)
        _log(f"ramp{nx}x{ny}x{nz}: {turns[-1]}")
    forms = {}
    for name, sv in solvers.items():
        c = cases[name]
        prof = pk.ocfd_profile_read(sv.h)
        pk.ocfd_profile(sv.h, False)
        mean_frac = np.mean(np.array(fracs[name]), axis=0)
        forms[name] = {"gpt_substeps_per_s": round(c.N * steps / elapsed[name] / 1e9, 4),
                       "ms_per_substep": round(elapsed[name] / steps * 1e3, 3),
                       "avg_launch_us": _prof_avg_us(prof),
                       "weno_frac_mean_over_turns": [round(v, 5) for v in mean_frac],
                       "roofline": _sweep_roofline(prof, c.N, mean_frac, c.precision == "mixed")}
        if shape == (2048, 256, 256) and forms[name]["roofline"]["kernel"] == "sweep_xi":
            t = PMC_TRAFFIC_RAMP["mixed" if c.precision == "mixed" else "fp64"]
            forms[name]["roofline"]["traffic"] = 2 * t["fetch_kib"] * 1024 + t["write_kib"] * 1024
        _log(f"ramp{nx}x{ny}x{nz}: {name}: {forms[name]['gpt_substeps_per_s']} Gpt-substeps/s, "
             f"{forms[name]['avg_launch_us']}")
    for name in learned:
        a = pk.ocfd_sensor_audit(solvers[name].h)
        forms[name]["audit"] = {"runs": int(a[0]), "plain_weno_frac": round(a[2] / max(a[1], 1), 5),
                                "learned_weno_frac": round(a[3] / max(a[1], 1), 5),
                                "missed_frac_of_plain_weno": round(a[4] / max(a[2], 1), 6),
                                "mismatch_rate": round(a[5] / max(a[1], 1), 6)}
        forms[name]["training"] = nets[cases[name].sensor_inputs]["info"]
        forms[name]["rel_l2_vs_plain_fp64_after_100"] = (turns[0][name]["rel_l2_vs_plain_fp64"]
                                                          if turns and turns[0]["substeps"] == report else None)
        forms[name]["rel_l2_vs_plain_fp64_at_end"] = turns[-1][name]["rel_l2_vs_plain_fp64"] if turns else None
    drift100 = forms["learned_fp32"]["rel_l2_vs_plain_fp64_after_100"]
    drift_end = forms["learned_fp32"]["rel_l2_vs_plain_fp64_at_end"]
    for sv in solvers.values():
        sv.close()
    del solvers, xyz, inflow, U0
    torch.cuda.empty_cache()
    out = {"workload": f"Mach 2.9 24-degree compression ramp {nx}x{ny}x{nz} ({case.N} points), isothermal wall "
                       f"Tw 2.84, nonreflecting exit and top, Re_delta 5e4, C8 viscous, hybrid UD7 / WENO7: plain "
                       f"FP64 (pressure sensor) vs FP32 split/reconstruction + learned sensor every second RK "
                       f"step (audited every {report} substeps; inputs: the plain sensor's second differences; "
                       f"beside it the network once per RK step, and first-difference inputs); {steps} timed "
                       f"substeps each from the inflow state",
           "points": case.N, "forms": forms,
           "rel_l2_learned_vs_plain_after_100": drift100, "rel_l2_learned_vs_plain_at_end": drift_end,
           "plain_weno_frac_after_training_run": win, "training_run_substeps": train,
           "every_100_substeps": turns}
    return out


def cpu_baseline_ramp(threads: int, shape=(512, 256, 128), substeps=3):
    """The oracle, unchanged, on a slab of the ramp with the plain FP64 hybrid
    (UD7 / WENO7, pressure sensor) from the inflow state, metrics excluded; and
    on one core on a smaller slab.  Reported per grid-point substep."""
    import dataclasses
    import oracle
    import workloads
    out = {}
    for key, shp, nth in (("all", shape, threads), ("single_core", (256, 128, 32), 1)):
        c = dataclasses.replace(workloads.compression_ramp(shape=shp), scheme="hybrid", lowdiss="ud7")
        P = oracle.params_from_case(c, nthreads=nth)
        met = oracle.metrics(P, c.xyz)
        best = None
        for _ in range(2 if key == "all" else 1):
            t0 = time.perf_counter()
            oracle.advance(P, met, c.U0, substeps, c.dt, inflow=c.inflow)
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
        out[key] = {"value": c.N * substeps / best / 1e9, "cores": nth,
                    "sample": f"{substeps} substeps of the plain FP64 hybrid on a {shp[0]}x{shp[1]}x{shp[2]} "
                              f"slab of the ramp ({c.N * substeps} point-substeps), {best:.1f} s"}
    cpu = {"value": out["all"]["value"], "unit": "Gpt-substeps/s", "cores": out["all"]["cores"], "kind": "oracle",
           "sample": out["all"]["sample"] + "; rate per point-substep, extrapolated to the full grid",
           "single_core": out["single_core"]}
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
        cpu["cpu_model"] = model
    except Exception:
        pass
    return cpu


def secondary_c2(torch, pk, n, steps, warmup):
    """The plain FP64 method, WENO7 everywhere, on the two distorted periodic
    n^3 runs (Taylor-Green with sixth-order viscous terms, isentropic vortex
    Euler); one step = one substep of each run."""
    cases = make_cases(n)
    solvers = []
    for c in cases:
        s = pk.Solver(pk.params_from(c))
        s.set_grid(torch.from_numpy(c.xyz).cuda())
        s.set_state(torch.from_numpy(c.U0).cuda())
        solvers.append(s)
    for _ in range(warmup):
        for s, c in zip(solvers, cases):
            s.advance(1, c.dt)
    torch.cuda.synchronize()
    for s in solvers:
        pk.ocfd_profile(s.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, c in zip(solvers, cases):
            s.advance(1, c.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = [pk.ocfd_profile_read(s.h) for s in solvers]
    for s in solvers:
        pk.ocfd_profile(s.h, False)
        s.close()
    del solvers
    torch.cuda.empty_cache()
    tot = {}
    for p in prof:
        for k, (ms, cnt) in p.items():
            a = tot.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
    N = sum(c.N for c in cases) // len(cases)
    roof = _sweep_roofline(tot, N, [1.0, 1.0, 1.0], False, hybrid=False)
    if roof["kernel"] in PMC_TRAFFIC and n == 256:
        t = PMC_TRAFFIC[roof["kernel"]]
        roof["traffic"] = 2 * t["fetch_kib"] * 1024 + t["write_kib"] * 1024
    return {"workload": f"isentropic vortex (Euler) + Taylor-Green (C6 viscous) on {n}^3 distorted periodic grids, "
                        "plain FP64 method, SW + WENO7 everywhere, RK3; one step = one substep of each",
            "gpt_substeps_per_s": round(sum(c.N for c in cases) * steps / elapsed / 1e9, 4),
            "ms_per_step": round(elapsed / steps * 1e3, 4), "steps": steps,
            "avg_launch_us": _prof_avg_us(tot), "roofline": roof}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="substeps timed per form on the headline workload")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shape", type=str, default="2048,256,256", help="headline ramp grid")
    ap.add_argument("--train-substeps", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--n", type=int, default=256, help="grid points per direction of the secondary runs")
    ap.add_argument("--c2-steps", type=int, default=200)
    ap.add_argument("--forms", type=str, default="c2,hit,ramp",
                    help="comma list of extra comparisons: c2 (256^3 FP64 WENO7), hit (512^3 isotropic "
                         "turbulence forms), ramp (1024x160x128 forms); empty for none")
    ap.add_argument("--hit-n", type=int, default=512)
    ap.add_argument("--hit-develop", type=int, default=2500,
                    help="plain FP64 hybrid substeps before the forms are timed (t ~ 0.9 at 512^3)")
    ap.add_argument("--form-substeps", type=int, default=100)
    ap.add_argument("--ramp-shape", type=str, default="1024,160,128")
    ap.add_argument("--learned-overhead", action="store_true",
                    help="also time the learned sensor's kernels on the 256^3 Taylor-Green run")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 512 MiB device-to-device copy first, as the reference dispatch "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver keeps the whole domain on a single device, and this "
              "build has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_15333_amd as pk

    if args.calibration_copy:
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        _log("calibration copy: 536870912 bytes read, 536870912 bytes written")

    shape = tuple(int(v) for v in args.shape.split(","))
    head = headline_ramp(torch, pk, shape, args.train_substeps, args.epochs, args.steps, args.warmup)
    lf, pf = head["forms"]["learned_fp32"], head["forms"]["plain_fp64"]
    value = lf["gpt_substeps_per_s"]
    speedup = value / pf["gpt_substeps_per_s"]
    extra = [f for f in args.forms.split(",") if f]
    forms = {}
    if "c2" in extra:
        forms["c2_fp64_weno7_256cube"] = secondary_c2(torch, pk, args.n, args.c2_steps, args.warmup)
        _log(f"c2: {forms['c2_fp64_weno7_256cube']['gpt_substeps_per_s']} Gpt-substeps/s")
    if "hit" in extra:
        forms["isotropic_turbulence"] = form_hit_learned(torch, pk, args.hit_n, args.hit_develop, 50,
                                                         args.form_substeps)
    if "ramp" in extra:
        forms["compression_ramp"] = form_ramp_mixed(torch, pk, tuple(int(v) for v in args.ramp_shape.split(",")),
                                                    args.form_substeps)
    overhead = learned_overhead(torch, pk, args.n, 100) if args.learned_overhead else None

    cpu = None
    if not args.no_cpu_baseline:
        _log(f"oracle baseline on {args.cpu_threads} threads")
        cpu = cpu_baseline_ramp(args.cpu_threads)

    out = {
        "metric": "Gpt-substeps/s: plain FP64 vs FP32+learned-sensor form at stated L2 error",
        "value": value,
        "unit": "Gpt-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lf["ms_per_substep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 split/reconstruction, f64 metrics/flux difference/RK/reductions, bf16 MFMA sensor",
        "data": "synthetic",
        "config": {"workload": head["workload"], "points": head["points"], "parallelism": "single GPU"},
        "plain_fp64": {"value": pf["gpt_substeps_per_s"], "ms_per_step": pf["ms_per_substep"],
                       "dtype": "f64", "roofline": pf["roofline"]},
        "speedup_vs_plain_fp64": round(speedup, 3),
        "rel_l2_vs_plain_fp64_after_100_substeps": head["rel_l2_learned_vs_plain_after_100"],
        "rel_l2_vs_plain_fp64_at_end": head["rel_l2_learned_vs_plain_at_end"],
        "target": {"speedup_vs_plain_fp64": 2.0, "rel_l2_after_100_substeps": 1e-5,
                   "met": bool(speedup >= 2.0 and head["rel_l2_learned_vs_plain_after_100"] is not None and
                               max(head["rel_l2_learned_vs_plain_after_100"]) <= 1e-5)},
        "roofline": lf["roofline"],
        "cpu_baseline": cpu,
        "headline": head,
        "forms": forms,
    }
    if overhead is not None:
        out["learned_overhead"] = overhead
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
