#!/usr/bin/env python3
"""Throughput benchmark of the bulb-model flavor-evolution hot path on one GPU.

Workload: three-flavor multi-angle bulb model, 400 energy bins x 4000 emission
angles x {nu, nubar} = 3.2M beams, Dormand-Prince 5(4) with rtol 1e-9, evolved
from the neutrinosphere (r = 10 km) with synthetic Fermi-Dirac spectra; no
dataset is involved.  One "step" is one attempted adaptive step: every launch
of an attempt (the per-trajectory stage launches, the state update with the
step error, the step control with the power moments of the new state).
beam-steps = beams x accepted steps.

The headline value is the FP32-amplitude form (FP32 amplitudes in HBM and FP32
update arithmetic; moments, step error and phases in FP64).  The same grid is
also run with FP32 amplitudes and FP64 arithmetic and in plain FP64.  The line
also carries: the FP32 forms' probabilities against the FP64 form over two
radius windows with real flavor evolution, the two small workloads (the
two-flavor single-angle fixed-step run and the 200 x 1000 FP64 adaptive run)
with their oracle times, the extended bulb model, the paper's own exponential
stepper, the 64-run batched workload (graph replays) and the served Poisson
mix, and the oracle timed on the host's cores.

Prints one JSON line.  --gpus above 1 is not supported: the path runs on one
GPU (the angle-sharded multi-GPU design is described, not built).
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "beam-steps/s at 1 GPU (FP32-amp vs FP64) @1e-4 prob error; p50/p99 latency"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz =
# 78.6 TFLOP/s for FP64 and for unpacked FP32.  The build disables packed FP32
# arithmetic, so 78.6 is the reachable peak of both precisions here.
PEAK_VALU_TFS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
FORM_NAMES = {"fp32": 1, "fp32math64": 2, "fp64": 0}
DTYPE = {1: "f32", 2: "f32-storage/f64-math", 0: "f64"}

# Dormand-Prince 5(4): stages, update and error polynomial degrees in u = +-1/E
# (the update 1 + sum_m b_m D_m(u) reaches degree 6, the error sum_m e_m D_m(u)
# degree 7), and the power moments Q_0 .. Q_12 the stage densities need.
DP_S, DP_DN, DP_DE, DP_NQ = 7, 6, 7, 13


def kernel_names(prec: int, n: int = 3, nj: int = 2):
    """Short names of the launches of one attempt (single-run instantiations,
    as profile_summary.kernel_key writes them), in launch order."""
    ts = "double" if prec == 0 else "float"
    t = "float" if prec == 1 else "double"
    tf = "float" if prec == 1 else "double"
    # (the stage launches before the last hold no table of the arithmetic type)
    names = [f"k_traj<{n},DP54,{nj},{L},{tf if L == DP_S else 'double'}>" for L in range(1, DP_S + 1)]
    names.append(f"k_final<{ts},{t},{n},DP54,{nj}>")
    names.append(f"k_power<{ts},{n},DP54,{nj},false>")
    return names


def run_form(nuosc, W, torch, precision, steps, warmup):
    """Time `steps` attempts of one precision form on the run's own stream.

    Two passes over the same number of attempts: the first is timed as a
    whole (HIP events on the run's stream around it) and gives the
    throughput; in the second the library records HIP events around every
    launch on the same stream, which gives each launch's mean duration (each
    including the few microseconds an event record adds)."""
    w = W.multi_angle_3f_large(precision)
    run = nuosc.Run.with_torch(w)
    stream = run.torch_stream
    S = run.num_stages
    run.step(warmup)
    s0 = run.stats()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    run.enqueue_steps(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    s1 = run.stats()
    run.timing_enable(True)
    run.enqueue_steps(steps)
    beam, _, cnt = run.timing_read()
    run.timing_enable(False)
    accepted = s1["accepted"] - s0["accepted"]
    n = [max(int(c), 1) for c in cnt]
    out = dict(
        precision=precision,
        beams=run.nb,
        traj=run.na,
        attempts=steps,
        accepted=accepted,
        ms_per_step=total_ms / steps,
        value=run.nb * accepted / (total_ms / 1e3),
        launch_us=[1e3 * beam[st] / n[st] for st in range(1, S + 1)],
        names=kernel_names(precision),
        r_km=s1["r_km"],
        amp_bytes=4 if precision != W.FP64 else 8,
        n=run.n,
    )
    return run, out


def beam_model(form, idx):
    """Algorithmic HBM bytes and vector flops of launch `idx` (0-based) of an
    attempt, for the whole grid.

    Bytes follow the method's floor (one read of the state per derivative
    evaluation, one write of the new state): the state update reads psi_n and
    writes psi_{n+1}; the power-moment launch reads psi_{n+1} (the first
    evaluation of the next step); the per-trajectory launches touch no beam
    data.  Flops count one FMA as 2 (powers of u and the renormalisation's
    multiplies as 1):
      state update: per row of the n x n complex update matrix, 2n reals x
        (DN + 1) power-sum FMAs, then n complex multiply-adds (4 FMAs each);
        the same with degree DE in FP64 for the error; FP32 renormalisation;
      power moments, per energy bin (its neutrino and antineutrino beam,
        u = 1/E and -1/E): both density matrices (n diagonal, n(n-1)/2
        complex off-diagonal entries each), their even and odd combinations
        w rho +- wbar rhobar, the powers of u and NQ x n^2 FMAs for
        Q_0 .. Q_{NQ-1}; half of that per beam."""
    n, nb = form["n"], form["beams"]
    state = 2 * n * form["amp_bytes"] * nb
    S = DP_S
    if idx < S:
        return 0, 0
    if idx == S:
        upd = 2 * (2 * n * n * (DP_DN + 1) + 4 * n * n) + (DP_DN - 1)
        err = 2 * (2 * n * n * (DP_DE + 1) + 4 * n * n) + (DP_DE - 1) + 2 * n
        ren = (2 * 2 * n + 2 * n + 2) if form["precision"] != 0 else 0
        return 2 * state, (upd + err + ren) * nb
    nm = n * n
    dens = 2 * n + 2 * n + (n * (n - 1) // 2) * 2 * 2
    pair = 2 * dens + 5 * nm + DP_NQ + 2 * DP_NQ * nm
    return state, pair * nb // 2


def traffic_of(name):
    """Copy-calibrated rocprofv3 FETCH + WRITE bytes per launch of a kernel, or
    None when no counters were taken for the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        from paper_1907_05560_amd.profile_summary import kernel_source_hash

        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return t.get("bytes_per_launch", {}).get(name)
    except (OSError, ValueError):
        return None


def roofline(form):
    """Roofline of the dominant kernel (the launch with the longest mean
    duration; for the 3.2M-beam grid the state update, k_final).

    HBM view: algorithmic bytes per launch (beam_model) / the launch's mean
    duration, against 8 TB/s.  ALU view: the launch's vector flops / duration
    against the unpacked vector peak.  The bound is the view with the larger
    fraction of its peak; both views are kept.  traffic: the rocprofv3
    FETCH + WRITE bytes of that kernel (copy-calibrated), null without
    counters for the current kernel source; waste = traffic / algorithmic
    bytes."""
    dom = max(range(len(form["launch_us"])), key=lambda i: form["launch_us"][i])
    name = form["names"][dom]
    alg_bytes, flops = beam_model(form, dom)
    dur_s = form["launch_us"][dom] / 1e6
    gbs = alg_bytes / dur_s / 1e9
    tfs = flops / dur_s / 1e12
    hbm = {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
           "alg_bytes_per_launch": alg_bytes}
    alu = {"achieved": round(tfs, 2), "peak": PEAK_VALU_TFS, "unit": "TFLOP/s",
           "frac": round(tfs / PEAK_VALU_TFS, 4), "flops_per_launch": flops}
    traffic = traffic_of(name)
    use_alu = alu["frac"] > hbm["frac"]
    head = alu if use_alu else hbm
    out = {
        "bound": "alu" if use_alu else "hbm",
        "kernel": name,
        "achieved": head["achieved"],
        "peak": head["peak"],
        "unit": head["unit"],
        "frac": head["frac"],
        "traffic": traffic,
        "mean_launch_us": round(dur_s * 1e6, 2),
        "hbm": hbm,
        "alu": alu,
    }
    if traffic is not None and alg_bytes:
        out["waste"] = round(traffic / alg_bytes, 3)
        out["traffic_gbs"] = round(traffic / dur_s / 1e9, 1)
    return out


def step_roofline(form):
    """Whole-step figures: beam-steps/s against (1) the method's floor, one
    read of y_n per derivative evaluation plus one write of y_{n+1}:
    B_alg = 7 S bytes per beam-step (Dormand-Prince, first-same-as-last; S =
    2n amplitude reals), (2) the design's bytes per beam-step, the copy-
    calibrated rocprofv3 FETCH + WRITE bytes of every launch of an attempt
    (null without counters for the current kernel source), and (3) the
    vector flops per beam-step of the beam launches against the unpacked
    vector peak."""
    state = 2 * form["n"] * form["amp_bytes"]
    b_alg = DP_S * state
    v = form["value"]
    out = {"alg_bytes_per_beam_step": b_alg, "alg_ceiling": round(PEAK_HBM_GBS * 1e9 / b_alg),
           "frac_alg": round(v * b_alg / (PEAK_HBM_GBS * 1e9), 4), "design_bytes_per_beam_step": None,
           "frac_design": None}
    tr = [traffic_of(nm) for nm in form["names"]]
    if all(x is not None for x in tr):
        d = sum(tr) / form["beams"]
        out["design_bytes_per_beam_step"] = round(d, 1)
        out["frac_design"] = round(v * d / (PEAK_HBM_GBS * 1e9), 4)
    flops = sum(beam_model(form, i)[1] for i in range(len(form["names"]))) / form["beams"]
    tfs = v * flops / 1e12
    out.update({"flops_per_beam_step": round(flops), "valu_tflops": round(tfs, 2), "valu_peak": PEAK_VALU_TFS,
                "valu_frac": round(tfs / PEAK_VALU_TFS, 4)})
    return out


def host_info():
    """Cores this process may use and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cores_allowed": len(os.sched_getaffinity(0)), "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(W, attempts):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of the
    same workload: `attempts` adaptive step attempts of the full grid from
    10 km; and the same sample with its OpenMP build (bitwise the same
    results) on the threads OMP_NUM_THREADS allows.

    Every attempt costs the oracle the same (all stages of every beam).  A fresh
    run rejects its first tries while the step size settles, whereas every timed
    GPU attempt (after warm-up) is accepted; the rate is therefore quoted per
    attempt, beams x attempts / time, which is the GPU's beam-steps/s at one
    accepted step per attempt."""
    from oracle import oracle as O

    w = W.multi_angle_3f_large(W.FP64)
    out = {}
    for omp in (False, True):
        ref = O.Run(w, openmp=omp)
        t = time.perf_counter()
        ref.step_dp54(attempts)
        dt = time.perf_counter() - t
        acc = ref.stats()["accepted"]
        threads = O.num_threads(omp)
        out[omp] = {
            "value": ref.nb * attempts / dt,
            "unit": "beam-steps/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{attempts} step attempts ({acc} accepted) of the 400x4000x2 grid from r = 10 km, "
                      f"FP64, {'OpenMP build, ' if omp else ''}{threads} thread(s), {dt:.1f} s; rate per attempt",
        }
        ref.close()
    line = dict(out[False])
    line["openmp"] = out[True]
    return line


def timed_runs(nuosc, torch, w, attempts, reps):
    """Median wall time (s) of `attempts` attempts of a fresh run of `w` (run
    creation and its first moment launch outside the timed region), over
    `reps` runs after one warm-up run; and the last run's statistics."""
    ts = []
    stats = None
    for i in range(reps + 1):
        with nuosc.Run(w) as run:
            torch.cuda.synchronize()
            t = time.perf_counter()
            run.step(attempts)
            dt = time.perf_counter() - t
            stats = run.stats()
        if i:
            ts.append(dt)
    return statistics.median(ts), ts, stats


def small_configs(nuosc, W, torch, c1_attempts, reps=3):
    """The two small workloads, GPU against the oracle (serial and OpenMP
    builds), each GPU figure the median of `reps` runs after one warm-up:

    * two-flavor single-angle run, 200 beams, 1e4 fixed RK4 steps from 50 km
      to 250 km (started at 50 km, where the explicit step is stable in the
      co-rotating frame), FP64: the whole run;
    * three-flavor multi-angle 200 x 1000 x 2 = 400k beams, Dormand-Prince
      rtol 1e-9 from 10 km, FP64: the first `c1_attempts` attempts (the full
      10 -> 250 km run takes ~1e10 attempts)."""
    from oracle import oracle as O

    out = {}
    w0 = dict(W.single_angle_2f(), r_start_km=50.0)
    t0, ts0, st0 = timed_runs(nuosc, torch, w0, w0["n_fixed_steps"], reps)
    nb0 = W.n_beams(w0)
    oracle0 = {}
    for omp in (False, True):
        ref = O.Run(w0, openmp=omp)
        t = time.perf_counter()
        ref.step_rk4(w0["n_fixed_steps"])
        dt = time.perf_counter() - t
        oracle0["openmp" if omp else "serial"] = {"seconds": round(dt, 3), "threads": O.num_threads(omp),
                                                 "value": nb0 * w0["n_fixed_steps"] / dt}
    out["single_angle_2f_rk4"] = {
        "workload": "2-flavor single-angle bulb model, 100 energies x 2 species = 200 beams, RK4 1e4 fixed "
                    "steps 50 -> 250 km, FP64",
        "beams": nb0, "steps": w0["n_fixed_steps"], "seconds": round(t0, 4), "repetitions_s": [round(x, 4) for x in ts0],
        "value": nb0 * st0["accepted"] / t0, "unit": "beam-steps/s", "oracle": oracle0,
        "note": "launch-latency bound: 6 launches per step of 200 beams",
    }
    w1 = W.multi_angle_3f(200, 1000)
    t1, ts1, s = timed_runs(nuosc, torch, w1, c1_attempts, reps)
    nb1 = W.n_beams(w1)
    oracle1 = {}
    for omp in (False, True):
        ref = O.Run(w1, openmp=omp)
        t = time.perf_counter()
        ref.step_dp54(c1_attempts)
        dt = time.perf_counter() - t
        so = ref.stats()
        oracle1["openmp" if omp else "serial"] = {"seconds": round(dt, 3), "threads": O.num_threads(omp),
                                                 "accepted": so["accepted"], "value": nb1 * so["accepted"] / dt}
        ref.close()
    out["multi_angle_200x1000_fp64"] = {
        "workload": f"3-flavor multi-angle bulb model, 200 energies x 1000 angles x 2 species = 400k beams, "
                    f"Dormand-Prince rtol 1e-9, FP64, the first {c1_attempts} attempts from r = 10 km",
        "beams": nb1, "attempts": c1_attempts, "accepted": s["accepted"], "rejected": s["rejected"],
        "r_km": s["r_km"], "seconds": round(t1, 5), "repetitions_s": [round(x, 5) for x in ts1],
        "value": nb1 * s["accepted"] / t1, "unit": "beam-steps/s", "oracle": oracle1,
        "note": "the 19 MB state arrays fit in the 256 MB MALL; launch-latency bound at this size",
    }
    return out


def accuracy(nuosc, W, forms):
    """The FP32 forms against the FP64 form on the full 400 x 4000 x 2 grid over
    the two radius windows (the same windows on which the FP64 form is
    pinned to the oracle on a 24 x 240 grid): every run starts from the
    pure-flavor state at r0 and evolves to r1 adaptively.  Max and RMS |dP|
    over all beams and over the seeded 4096-beam subsample, at r1."""
    import numpy as np

    out = []
    for r0, r1 in W.ACCURACY_WINDOWS:
        base = W.window(W.multi_angle_3f_large(W.FP64), r0, r1)
        with nuosc.Run(base) as ref:
            p0 = ref.probabilities()
            t = time.perf_counter()
            ref.evolve(r1)
            t64 = time.perf_counter() - t
            p64 = ref.probabilities()
            s64 = ref.stats()
        idx = W.error_subsample(p64.size)
        entry = {"window_km": [r0, r1], "r_km": s64["r_km"], "fp64_accepted": s64["accepted"],
                 "fp64_rejected": s64["rejected"], "fp64_seconds": round(t64, 3),
                 "max_dP_over_window": float(np.abs(p64 - p0).max()),
                 "reference": "GPU FP64 form on the same grid (pinned to the oracle on a 24x240 grid over the "
                              "same window)", "forms": {}}
        for name in forms:
            prec = FORM_NAMES[name]
            if prec == W.FP64:
                continue
            with nuosc.Run(dict(base, precision=prec)) as run:
                t = time.perf_counter()
                run.evolve(r1)
                dt = time.perf_counter() - t
                p = run.probabilities()
                s = run.stats()
            d = p - p64
            entry["forms"][name] = {
                "max": float(np.abs(d).max()), "rms": float(np.sqrt((d ** 2).mean())),
                "subsample_max": float(np.abs(d[idx]).max()), "subsample_rms": float(np.sqrt((d[idx] ** 2).mean())),
                "accepted": s["accepted"], "rejected": s["rejected"], "r_km": s["r_km"], "seconds": round(dt, 3),
                "within_1e-4": bool(np.abs(d).max() <= 1e-4)}
        out.append(entry)
    return out


def energy_average_timing(run, torch, amp_bytes, reps=50):
    """The energy-averaged output (k_energy_average) on the run's current state:
    mean duration of `reps` launches queued back to back on the run's stream
    (device output), against the HBM roofline of its algorithmic bytes (the
    state read once, the per-bin flux table, the output)."""
    out = torch.empty(2 * run.na * run.n, dtype=torch.float64, device="cuda")
    stream = run.torch_stream
    run.enqueue_energy_average(out.data_ptr())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run.enqueue_energy_average(out.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    nbytes = run.nb * 2 * run.n * amp_bytes + (run.nb // run.na) * 8 + 2 * run.na * run.n * 8
    gbs = nbytes / us / 1e3
    return {"us": round(us, 2), "alg_bytes": nbytes, "achieved_gbs": round(gbs, 1),
            "peak_gbs": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 4)}


def extended(nuosc, W, torch, precision, attempts, warmup=5):
    """The extended bulb model (eq 3.18: 100 energies x 100 emission angles x
    32 azimuth bins x 2 species = 640k beams, four angle moments), started
    from the seeded azimuthally perturbed state: beam-steps/s over `attempts`
    attempts after `warmup`."""
    w = W.extended_bulb_3f(100, 100, 32, precision)
    run = nuosc.Run.with_torch(w)
    try:
        psi = W.azimuth_perturbed_states(3, run.nb, run.na, seed=W.SEED_BASE + 5)
        run.set_state(psi, None, w["r_start_km"])
        run.step(warmup)
        s0 = run.stats()
        stream = run.torch_stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        run.enqueue_steps(attempts)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        s1 = run.stats()
        acc = s1["accepted"] - s0["accepted"]
        return {"workload": "3-flavor extended bulb model, 100 E x 100 angles x 32 azimuth bins x 2 species",
                "beams": run.nb, "attempts": attempts, "accepted": acc, "ms_per_step": ms / attempts,
                "value": run.nb * acc / (ms / 1e3), "unit": "beam-steps/s"}
    finally:
        run.close()


SERVING_WINDOW_KM = 3e-5
EXP_VALU_FILE = os.path.join(ROOT, "profiles", "exp_valu.json")
# wavefront-instruction issue peak of the vector ALUs: 256 CUs x 4 SIMDs, one
# 64-lane FP64 (or unpacked FP32) instruction per SIMD every 4 cycles at 2.4 GHz
PEAK_VALU_WAVE_INSTR_S = 256 * 4 * 2.4e9 / 4


def exp_stepper(nuosc, W, torch, attempts, warmup=10):
    """The paper's own stepper (exponential steps of eq 3.10-3.12 in the
    half/full-step loop with averaging and max-error control) on the 400 x
    4000 x 2 grid, lab frame, FP64, rtol 1e-9, from 10 km: beam-steps/s over
    `attempts` attempts after `warmup`, per-launch kernel times, the HBM view
    of its state traffic (each of the three beam launches reads psi_n once,
    the third also writes psi_{n+1}) and, from the committed rocprofv3 VALU
    instruction counts of the same kernels, the fraction of the vector-ALU
    issue peak it reaches (the kernels are bound by VALU issue)."""
    from paper_1907_05560_amd.profile_summary import exp_source_hash

    w = W.exp_stepper_3f(400, 4000)
    run = nuosc.Run.with_torch(w)
    try:
        run.step(warmup)
        s0 = run.stats()
        stream = run.torch_stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        run.enqueue_steps(attempts)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        s1 = run.stats()
        run.timing_enable(True)
        run.enqueue_steps(attempts)
        beam, fin, cnt = run.timing_read()
        run.timing_enable(False)
        acc = s1["accepted"] - s0["accepted"]
        rej = s1["rejected"] - s0["rejected"]
        n = [max(int(c), 1) for c in cnt]
        launch_us = [round(1e3 * beam[i] / n[i], 2) for i in range(1, 4)]
        reduce_us = [round(1e3 * fin[i] / n[i], 2) for i in range(1, 4)]
        state = 2 * 3 * 8 * run.nb
        hbm_bytes = [state, state, 2 * state]
        hbm = [round(b / (u * 1e3), 1) for b, u in zip(hbm_bytes, launch_us)]
        out = {"workload": "the paper's exponential stepper, 3-flavor multi-angle bulb model, 400 E x 4000 angles "
                           "x 2 species, lab frame, FP64, rtol 1e-9, from r = 10 km",
               "beams": run.nb, "attempts": attempts, "accepted": acc, "rejected": rej,
               "ms_per_step": ms / attempts, "value": run.nb * acc / (ms / 1e3),
               "attempt_rate": run.nb * attempts / (ms / 1e3), "unit": "beam-steps/s",
               "launch_us": launch_us, "reduce_us": reduce_us,
               "hbm": {"alg_bytes_per_launch": hbm_bytes, "achieved_gbs": hbm, "peak_gbs": PEAK_HBM_GBS,
                       "frac": [round(g / PEAK_HBM_GBS, 4) for g in hbm]},
               "valu": None}
        if os.path.exists(EXP_VALU_FILE):
            t = json.load(open(EXP_VALU_FILE))
            if t.get("source_sha256_16") == exp_source_hash():
                ins = [t["valu_wave_instr_per_launch"].get(f"launch{i}") for i in (1, 2, 3)]
                if all(ins):
                    frac = [round(i / (u * 1e-6) / PEAK_VALU_WAVE_INSTR_S, 4) for i, u in zip(ins, launch_us)]
                    out["valu"] = {"wave_instr_per_launch": ins, "peak_wave_instr_s": PEAK_VALU_WAVE_INSTR_S,
                                   "issue_frac": frac}
        return out
    finally:
        run.close()


def batched(nuosc, W, torch, attempts):
    """The 64-run batched workload: every run admitted into one batch and
    advanced together; the timed batch steps replay the captured HIP graph."""
    from paper_1907_05560_amd import serving

    out = serving.run_batched(W.batched_runs(64), attempts, torch=torch)
    out["workload"] = ("64 seeded 3-flavor multi-angle runs (N_E in 50..400, N_A log-uniform in 100..4000), "
                       "FP32 amplitudes, Dormand-Prince rtol 1e-9 from r = 10 km")
    return out


def served(nuosc, W, seconds, precision, check_fraction):
    """The served Poisson mix: 20 requests/s for `seconds`, 10% of them on the
    400 x 4000 grid, each evolved from 10 km over a 3e-5 km window (offered
    load above one GPU's capacity, so the queue grows); the loop stops when
    the arrival period ends.  Latencies include queue wait.  The window is
    3e-5 km: ~2e9 beam-steps per request on average, ~3e10 beam-steps/s
    offered at 20 requests/s.  Then a seeded
    `check_fraction` of the completed requests is run alone (nuosc_create)
    and compared bitwise with its served result."""
    import numpy as np

    from paper_1907_05560_amd import serving

    reqs = W.serving_requests(duration_s=seconds, precision=precision, window_km=SERVING_WINDOW_KM)
    out = serving.serve(reqs, max_slots=64, duration_s=seconds)
    digests = out.pop("digests")
    done = sorted(digests)
    k = int(np.ceil(check_fraction * len(done))) if done else 0
    rng = np.random.default_rng(W.SEED_BASE + 6)
    pick = sorted(rng.choice(done, size=k, replace=False).tolist()) if k else []
    same = True
    t = time.perf_counter()
    for i in pick:
        w = dict(reqs[i])
        with nuosc.Run(w) as run:
            run.evolve(w["r_end_km"])
            same = same and serving.digest(run.probabilities()) == digests[i]
    out["mix_equals_alone"] = same
    out["alone_checked"] = len(pick)
    out["alone_check_seconds"] = round(time.perf_counter() - t, 2)
    out["window_km"] = reqs[0]["r_end_km"] - reqs[0]["r_start_km"]
    out["arrival_rate_per_s"] = len(reqs) / seconds
    out["mean_completed_beam_steps"] = out["beam_steps_completed"] / max(1, out["completed"])
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-attempts", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP32-vs-FP64 accuracy windows")
    ap.add_argument("--small-attempts", type=int, default=20,
                    help="attempts of the 200x1000 FP64 workload (0: skip both small workloads)")
    ap.add_argument("--extended-attempts", type=int, default=50,
                    help="attempts of the extended bulb model workload (0: skip)")
    ap.add_argument("--exp-attempts", type=int, default=30,
                    help="attempts of the paper's exponential stepper on the 400x4000 grid (0: skip)")
    ap.add_argument("--forms", default="fp32,fp32math64,fp64",
                    help="precision forms to run (the first is the headline value)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a device buffer of this size (for scaling HBM counters)")
    ap.add_argument("--batched-attempts", type=int, default=50,
                    help="attempts per batch step of the 64-run batched workload (0 = skip)")
    ap.add_argument("--serving-seconds", type=float, default=120.0,
                    help="seconds of Poisson arrivals in the serving runs (0 = skip)")
    ap.add_argument("--serving-check-fraction", type=float, default=0.1,
                    help="fraction of completed requests re-run alone for the bitwise check")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this path runs on one GPU "
              "(multi-GPU angle sharding is a design note, not built).", file=sys.stderr)
        return 2

    import torch

    from paper_1907_05560_amd import nuosc, workloads as W

    def say(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    torch.cuda.init()
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib * 2 ** 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    form_list = args.forms.split(",")
    order = [FORM_NAMES[f] for f in form_list]
    # The accuracy windows run first, so that the timed forms do not start on
    # a GPU that has been idle since the process began (measured: a 20-attempt
    # window timed right after creation and 5 warm-up attempts runs about 8%
    # slower than the same window after 0.3 s of load; short windows still
    # read a few percent above the long-run attempt time, as the run's
    # creation leaves the GPU idle again for a moment).
    acc = None
    if not args.no_accuracy and 0 in order:
        say(f"accuracy windows {W.ACCURACY_WINDOWS} km on the 400x4000 grid")
        acc = accuracy(nuosc, W, form_list)
        for e in acc:
            say(f"window {e['window_km']}: fp64 {e['fp64_accepted']} steps, P moves {e['max_dP_over_window']:.3e}; "
                + ", ".join(f"{k} max {v['max']:.3e} rms {v['rms']:.3e}" for k, v in e["forms"].items()))
    forms = {}
    averages = {}
    for name, prec in zip(form_list, order):
        say(f"{name}: {args.warmup} warmup + {args.steps} timed attempts")
        run, form = run_form(nuosc, W, torch, prec, args.steps, args.warmup)
        forms[prec] = form
        averages[name] = energy_average_timing(run, torch, form["amp_bytes"])
        run.close()
        say(f"{name}: {form['ms_per_step']:.4f} ms/step, {form['value']:.4e} beam-steps/s, launches "
            f"{[round(x, 1) for x in form['launch_us']]} us")

    head = forms[order[0]]
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "beam-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[order[0]],
        "data": "synthetic",
        "config": {
            "workload": "three-flavor multi-angle bulb model, 400 energies x 4000 angles x 2 species "
                        "= 3.2M beams, Dormand-Prince 5(4) rtol 1e-9 from r = 10 km",
            "beams": head["beams"],
            "parallelism": "single GPU",
        },
        "roofline": roofline(head),
        "accepted_per_attempt": head["accepted"] / head["attempts"],
        "step_roofline": step_roofline(head),
        "forms": {f: {"value": forms[FORM_NAMES[f]]["value"], "ms_per_step": forms[FORM_NAMES[f]]["ms_per_step"],
                      "dtype": DTYPE[FORM_NAMES[f]],
                      "launch_us": dict(zip(forms[FORM_NAMES[f]]["names"],
                                            [round(x, 2) for x in forms[FORM_NAMES[f]]["launch_us"]])),
                      "roofline": roofline(forms[FORM_NAMES[f]]),
                      "step_roofline": step_roofline(forms[FORM_NAMES[f]])}
                  for f in form_list},
        "energy_average": averages,
        "host": host_info(),
    }
    if acc is not None:
        line["accuracy"] = acc
    if args.small_attempts > 0:
        say("small workloads (2f single-angle RK4 run, 200x1000 FP64 window) and their oracle times")
        line["small_workloads"] = small_configs(nuosc, W, torch, args.small_attempts)
        for k, v in line["small_workloads"].items():
            say(f"{k}: {v['value']:.3e} beam-steps/s in {v['seconds']} s; oracle serial "
                f"{v['oracle']['serial']['seconds']} s, OpenMP {v['oracle']['openmp']['seconds']} s")
    if args.extended_attempts > 0:
        line["extended"] = {}
        for name, prec in (("fp32", W.FP32_AMP), ("fp64", W.FP64)):
            say(f"extended bulb model {name} ({args.extended_attempts} attempts)")
            ex = extended(nuosc, W, torch, prec, args.extended_attempts)
            line["extended"][name] = ex
            say(f"extended {name}: {ex['ms_per_step']:.3f} ms/step, {ex['value']:.3e} beam-steps/s")
    if args.exp_attempts > 0:
        say(f"exponential stepper ({args.exp_attempts} attempts)")
        ex = exp_stepper(nuosc, W, torch, args.exp_attempts)
        line["exp_stepper"] = ex
        say(f"exponential stepper: {ex['ms_per_step']:.3f} ms/attempt, {ex['value']:.3e} beam-steps/s, "
            f"launches {ex['launch_us']} us, reductions {ex['reduce_us']} us")
    if args.batched_attempts > 0:
        say(f"batched workload ({args.batched_attempts} attempts per batch step, graph replays)")
        line["batched"] = batched(nuosc, W, torch, args.batched_attempts)
        say(f"batched {line['batched']['value']:.3e} beam-steps/s, timed steps replayed "
            f"{line['batched']['timed_steps_replayed']}/{line['batched']['timed_steps']}")
    if args.serving_seconds > 0:
        line["serving"] = {}
        for name, prec in (("fp32", W.FP32_AMP), ("fp64", W.FP64)):
            say(f"serving {name} ({args.serving_seconds:g} s of arrivals)")
            sv = served(nuosc, W, args.serving_seconds, prec, args.serving_check_fraction)
            line["serving"][name] = sv
            say(f"serving {name}: {sv['completed']}/{sv['requests']} done, queue max {sv['max_queue']}, "
                f"p50 {sv['p50_s']:.3f} s, p99 {sv['p99_s']:.3f} s, {sv['value']:.3e} beam-steps/s, "
                f"graph share {sv['graph_share']:.2f}, alone check {sv['alone_checked']} "
                f"{'equal' if sv['mix_equals_alone'] else 'DIFFERENT'}")
    if not args.no_cpu_baseline:
        say(f"cpu baseline ({args.cpu_attempts} oracle attempts, serial and OpenMP)")
        line["cpu_baseline"] = cpu_baseline(W, args.cpu_attempts)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
