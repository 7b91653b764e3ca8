#!/usr/bin/env python3
"""Throughput benchmark of the bulb-model flavor-evolution hot path on one GPU.

Workload: three-flavor multi-angle bulb model, 400 energy bins x 4000 emission
angles x {nu, nubar} = 3.2M beams, Dormand-Prince 5(4) with rtol 1e-9, evolved
from the neutrinosphere (r = 10 km) with synthetic Fermi-Dirac spectra; no
dataset is involved.  One "step" is one attempted adaptive step: every stage
kernel (moment reductions, fused Hamiltonian + RK stage), the step-error
reduction and the on-device controller.  beam-steps = beams x accepted steps.

The headline value is the FP32-amplitude form (FP32 amplitudes in HBM, FP32
stage arithmetic, FP64 moments / error / phases).  The same grid is also run
with FP32 amplitudes and FP64 arithmetic and in plain FP64, on the same GPU.

Prints one JSON line.  --gpus above 1 is not supported: the path runs on one
GPU (the angle-sharded multi-GPU design is described, not built).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "beam-steps/s at 1 GPU (FP32-amp vs FP64) @1e-4 prob error; p50/p99 latency"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# Vector ALU peaks (256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz = 78.6
# TFLOP/s for FP64 and for unpacked FP32; packed FP32 doubles the FP32 figure).
PEAK_FP32_TFS = 157.3
PEAK_FP64_TFS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def run_form(nuosc, W, torch, precision, steps, warmup):
    """Time `steps` attempts of one precision form on the run's own stream.

    Two passes over the same number of attempts: the first is timed as a
    whole (HIP events around it) and gives the throughput; in the second the
    library records events around every beam kernel and control kernel,
    which gives the per-kernel durations (each including the few
    microseconds an event record adds on the stream)."""
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
    beam, fin, cnt = run.timing_read()
    run.timing_enable(False)
    accepted = s1["accepted"] - s0["accepted"]
    n = [max(int(c), 1) for c in cnt]
    out = dict(
        precision=precision,
        beams=run.nb,
        attempts=steps,
        accepted=accepted,
        ms_per_step=total_ms / steps,
        value=run.nb * accepted / (total_ms / 1e3),
        stage_ms=[beam[st] / n[st] for st in range(1, S + 1)],
        fin_ms=[fin[st] / n[st] for st in range(1, S + 1)],
        r_km=s1["r_km"],
        amp_bytes=4 if precision != W.FP64 else 8,
        n=run.n,
    )
    return run, out


# Nonzero counts of the tableau rows (stage inputs 1..S-1, then the solution
# weights) and of the error weights, for the flop model below.
_NNZ = {
    "rk4": dict(S=4, fsal=False, rows=[1, 1, 1], sol=4, err=0),
    "dp54": dict(S=7, fsal=True, rows=[1, 2, 3, 4, 5, 5], sol=5, err=6),
}


def stage_flops(n: int, integrator: str, stage: int, fp32_storage: bool) -> int:
    """Flops per beam of stage launch `stage` (FMA = 2) in the recompute design.

    One derivative k = -i (A + B/E) y: n^2 FMAs to form the Hermitian matrix,
    2n multiplies for its diagonal and n(n-1) complex multiply-adds (4 FMAs) for
    the off-diagonals.  Launch I evaluates k_0..k_{I-1}, forms the inputs of
    stages 1..I (2n reals x (nonzeros + 1) FMAs each), the moments of its output
    state (n diagonal terms of 5 flops, n(n-1)/2 off-diagonal pairs of 10), and
    the FP32 renormalisation of the new state, and the embedded error.  For a
    first-same-as-last pair the error is split: the launch that forms y_{n+1}
    also sums e_i k_i over i < S-1, and the final launch evaluates only
    k_{S-1} = f(y_{n+1}) and adds h e_{S-1} k_{S-1}."""
    t = _NNZ[integrator]
    S = t["S"]
    f_eval = 2 * n * n + 2 * n + 8 * n * (n - 1)
    split = t["fsal"] and t["err"] > 0
    if split and stage == S:
        return f_eval + 2 * n * 3
    flops = stage * f_eval
    last_row = min(stage, S - 1)
    for l in range(1, last_row + 1):
        nnz = t["rows"][l - 1]
        flops += 2 * n * (nnz + 1) * 2
    final = stage == S
    if final and not t["fsal"]:
        flops += 2 * n * (t["sol"] + 1) * 2
    if not final or not t["fsal"]:
        flops += 5 * n + 10 * n * (n - 1) // 2
    if final and t["err"] and not split:
        flops += 2 * n * (t["err"] * 2 + 1)
    if split and stage == S - 1:
        flops += 2 * n * (2 * (t["err"] - 1) - 1)
    if fp32_storage and stage == (S - 1 if t["fsal"] else S):
        flops += 6 * n + 2
    return flops


def roofline(form):
    """Roofline of the dominant kernel (the slowest stage launch).

    HBM view: algorithmic bytes per launch (every beam launch reads y_n once,
    N_b x 2n amplitude reals; the launch that forms y_{n+1} -- the last one,
    or the one before it for a first-same-as-last pair -- also writes it; in
    the pair, that launch also writes the partial error sum, N_b x 2n reals of
    the arithmetic type, and the final launch reads y_{n+1} and that sum) /
    the launch's mean duration.  ALU view: stage_flops x N_b / duration against the vector
    peak of the arithmetic type.  The reported bound is the view with the
    larger fraction of its peak; the other view is kept alongside."""
    S = len(form["stage_ms"])
    dom = max(range(S), key=lambda i: form["stage_ms"][i])
    stage = dom + 1
    state_bytes = 2 * form["n"] * form["amp_bytes"] * form["beams"]
    write_stage = S - 1 if S == 7 else S
    alg_bytes = state_bytes * (2 if stage == write_stage else 1)
    if S == 7 and stage >= S - 1:
        alg_bytes += 2 * form["n"] * (4 if form["precision"] == 1 else 8) * form["beams"]
    dur_s = form["stage_ms"][dom] / 1e3
    gbs = alg_bytes / dur_s / 1e9
    fp32_math = form["precision"] == 1
    flops = stage_flops(form["n"], "dp54" if S == 7 else "rk4", stage, form["amp_bytes"] == 4) * form["beams"]
    tfs = flops / dur_s / 1e12
    peak_alu = PEAK_FP32_TFS if fp32_math else PEAK_FP64_TFS
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            from paper_1907_05560_amd.profile_summary import kernel_source_hash

            t = json.load(open(TRAFFIC_FILE))
            key = f"stage{stage}_prec{form['precision']}"
            if t.get("kernel_source_sha256_16") == kernel_source_hash() and key in t.get("bytes_per_launch", {}):
                traffic = t["bytes_per_launch"][key]
        except (OSError, ValueError):
            traffic = None
    hbm = {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
           "alg_bytes_per_launch": alg_bytes}
    alu = {"achieved": round(tfs, 2), "peak": peak_alu, "unit": "TFLOP/s", "frac": round(tfs / peak_alu, 4),
           "alg_flops_per_launch": flops, "frac_of_unpacked_peak": round(tfs / PEAK_FP64_TFS, 4)}
    use_alu = alu["frac"] > hbm["frac"]
    head = alu if use_alu else hbm
    out = {
        "bound": "alu" if use_alu else "hbm",
        "kernel": f"k_stage stage {stage}/{S}",
        "achieved": head["achieved"],
        "peak": head["peak"],
        "unit": head["unit"],
        "frac": head["frac"],
        "traffic": traffic,
        "mean_launch_us": round(dur_s * 1e6, 2),
        "hbm": hbm,
        "alu": alu,
    }
    if traffic is not None:
        out["traffic_gbs"] = round(traffic / dur_s / 1e9, 1)
    return out


def step_roofline(form):
    """Whole-step figures (every launch of an attempt): beam-steps/s against
    (1) the method's floor, one read of y_n per derivative evaluation plus one
    write of y_{n+1}: B_alg = (evaluations + 1) x S bytes per beam-step
    (Dormand-Prince first-same-as-last: 7 S; classic RK4: 5 S), and (2) the
    design's bytes per beam-step, the copy-calibrated rocprofv3 FETCH + WRITE
    bytes of all its stage launches (null without counters for this kernel
    source); and the achieved vector-ALU rate of the stage_flops model."""
    S = len(form["stage_ms"])
    state = 2 * form["n"] * form["amp_bytes"]
    b_alg = (S if S == 7 else S + 1) * state
    v = form["value"]
    out = {"alg_bytes_per_beam_step": b_alg, "alg_ceiling": round(PEAK_HBM_GBS * 1e9 / b_alg),
           "frac_alg": round(v * b_alg / (PEAK_HBM_GBS * 1e9), 4), "design_bytes_per_beam_step": None,
           "frac_design": None}
    if os.path.exists(TRAFFIC_FILE):
        try:
            from paper_1907_05560_amd.profile_summary import kernel_source_hash

            t = json.load(open(TRAFFIC_FILE))
            keys = [f"stage{i}_prec{form['precision']}" for i in range(1, S + 1)]
            bpl = t.get("bytes_per_launch", {})
            if t.get("kernel_source_sha256_16") == kernel_source_hash() and all(k in bpl for k in keys):
                d = sum(bpl[k] for k in keys) / form["beams"]
                out["design_bytes_per_beam_step"] = round(d, 1)
                out["frac_design"] = round(v * d / (PEAK_HBM_GBS * 1e9), 4)
        except (OSError, ValueError):
            pass
    flops = sum(stage_flops(form["n"], "dp54" if S == 7 else "rk4", st, form["amp_bytes"] == 4)
                for st in range(1, S + 1))
    tfs = v * flops / 1e12
    peak = PEAK_FP32_TFS if form["precision"] == 1 else PEAK_FP64_TFS
    out.update({"flops_per_beam_step": flops, "valu_tflops": round(tfs, 2), "valu_peak": peak,
                "valu_frac": round(tfs / peak, 4)})
    return out


def cpu_baseline(W, attempts):
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of the
    same workload: `attempts` adaptive step attempts of the full grid from 10 km.

    Every attempt costs the oracle the same (all stages of every beam).  A fresh
    run rejects its first tries while the step size settles, whereas every timed
    GPU attempt (after warm-up) is accepted; the rate is therefore quoted per
    attempt, beams x attempts / time, which is the GPU's beam-steps/s at one
    accepted step per attempt."""
    from oracle import oracle as O

    w = W.multi_angle_3f_large(W.FP64)
    ref = O.Run(w)
    t = time.perf_counter()
    ref.step_dp54(attempts)
    dt = time.perf_counter() - t
    acc = ref.stats()["accepted"]
    return {
        "value": ref.nb * attempts / dt,
        "unit": "beam-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{attempts} step attempts ({acc} accepted) of the 400x4000x2 grid from r = 10 km, "
                  f"FP64, single thread, {dt:.1f} s; rate per attempt",
    }


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
    advanced together; aggregate beam-steps/s over `attempts` attempts."""
    from paper_1907_05560_amd import serving

    return serving.run_batched(W.batched_runs(64), attempts, torch=torch)


def served(nuosc, W, seconds, precision):
    """The serving workload for `seconds` of Poisson arrivals: latency
    percentiles, throughput, and a bitwise check of two completed requests
    against the same runs alone."""
    import numpy as np

    from paper_1907_05560_amd import serving

    reqs = W.serving_requests(duration_s=seconds, precision=precision)
    out = serving.serve(reqs, max_slots=64, keep=2, wall_limit_s=max(120.0, 4 * seconds))
    same = True
    for i, p in out.pop("kept"):
        w = dict(reqs[i])
        with nuosc.Run(w) as run:
            run.evolve(w["r_end_km"])
            same = same and bool(np.array_equal(run.probabilities(), p))
    out["mix_equals_alone"] = same
    return out


def subsample_error(nuosc, W, run32, run64):
    """FP32-form error against the FP64 form on the seeded 4096-beam subsample,
    at a common radius (the run that is behind evolves to the other's radius)."""
    import numpy as np

    r32, r64 = run32.stats()["r_km"], run64.stats()["r_km"]
    r = max(r32, r64)
    if r32 < r:
        run32.evolve(r)
    if r64 < r:
        run64.evolve(r)
    idx = W.error_subsample(run32.nb)
    d = run32.probabilities()[idx] - run64.probabilities()[idx]
    return {"max": float(np.abs(d).max()), "rms": float(np.sqrt((d ** 2).mean())),
            "subsample": int(idx.size), "r_km": r}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-attempts", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extended-attempts", type=int, default=50,
                    help="attempts of the extended bulb model workload (0: skip)")
    ap.add_argument("--exp-attempts", type=int, default=30,
                    help="attempts of the paper's exponential stepper on the 400x4000 grid (0: skip)")
    ap.add_argument("--forms", default="fp32,fp32math64,fp64",
                    help="precision forms to run (the first is the headline value)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a device buffer of this size (for scaling HBM counters)")
    ap.add_argument("--batched-attempts", type=int, default=50,
                    help="attempts of the 64-run batched workload (0 = skip)")
    ap.add_argument("--serving-seconds", type=float, default=20.0,
                    help="seconds of Poisson arrivals in the serving runs (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this path runs on one GPU "
              "(multi-GPU angle sharding is a design note, not built).", file=sys.stderr)
        return 2

    import torch

    from paper_1907_05560_amd import nuosc, workloads as W

    torch.cuda.init()
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib * 2 ** 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    names = {"fp32": W.FP32_AMP, "fp32math64": W.FP32_AMP_FP64_MATH, "fp64": W.FP64}
    order = [names[f] for f in args.forms.split(",")]
    forms = {}
    runs = {}
    for prec in order:
        print(f"bench: precision {prec}: {args.warmup} warmup + {args.steps} timed attempts", file=sys.stderr, flush=True)
        run, form = run_form(nuosc, W, torch, prec, args.steps, args.warmup)
        forms[prec] = form
        runs[prec] = run
        print(f"bench: precision {prec}: {form['ms_per_step']:.3f} ms/step, {form['value']:.3e} beam-steps/s, "
              f"beam kernels {[round(x * 1e3, 1) for x in form['stage_ms']]} us, "
              f"control {[round(x * 1e3, 1) for x in form['fin_ms']]} us", file=sys.stderr, flush=True)
    err = None
    if W.FP32_AMP in runs and W.FP64 in runs:
        err = subsample_error(nuosc, W, runs[W.FP32_AMP], runs[W.FP64])
    averages = {}
    for prec, r in runs.items():
        averages[{W.FP32_AMP: "fp32", W.FP32_AMP_FP64_MATH: "fp32math64", W.FP64: "fp64"}[prec]] = \
            energy_average_timing(r, torch, 4 if prec != W.FP64 else 8)
    for r in runs.values():
        r.close()

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
        "dtype": {W.FP32_AMP: "f32", W.FP32_AMP_FP64_MATH: "f32-storage/f64-math", W.FP64: "f64"}[order[0]],
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
        "forms": {f: {"value": forms[names[f]]["value"], "ms_per_step": forms[names[f]]["ms_per_step"],
                      "roofline": roofline(forms[names[f]]), "step_roofline": step_roofline(forms[names[f]])}
                  for f in args.forms.split(",")},
        "fp32_vs_fp64_error": err,
        "stage_us": {str(p): [round(x * 1e3, 2) for x in f["stage_ms"]] for p, f in forms.items()},
        "control_us": {str(p): [round(x * 1e3, 2) for x in f["fin_ms"]] for p, f in forms.items()},
        "energy_average": averages,
    }
    if args.extended_attempts > 0:
        line["extended"] = {}
        for name, prec in (("fp32", W.FP32_AMP), ("fp64", W.FP64)):
            print(f"bench: extended bulb model {name} ({args.extended_attempts} attempts)", file=sys.stderr,
                  flush=True)
            ex = extended(nuosc, W, torch, prec, args.extended_attempts)
            line["extended"][name] = ex
            print(f"bench: extended {name}: {ex['ms_per_step']:.3f} ms/step, {ex['value']:.3e} beam-steps/s",
                  file=sys.stderr, flush=True)
    if args.exp_attempts > 0:
        print(f"bench: exponential stepper ({args.exp_attempts} attempts)", file=sys.stderr, flush=True)
        ex = exp_stepper(nuosc, W, torch, args.exp_attempts)
        line["exp_stepper"] = ex
        print(f"bench: exponential stepper: {ex['ms_per_step']:.3f} ms/attempt, {ex['value']:.3e} beam-steps/s, "
              f"launches {ex['launch_us']} us, reductions {ex['reduce_us']} us", file=sys.stderr, flush=True)
    if args.batched_attempts > 0:
        print(f"bench: batched workload ({args.batched_attempts} attempts)", file=sys.stderr, flush=True)
        line["batched"] = batched(nuosc, W, torch, args.batched_attempts)
        print(f"bench: batched {line['batched']['value']:.3e} beam-steps/s", file=sys.stderr, flush=True)
    if args.serving_seconds > 0:
        line["serving"] = {}
        for name, prec in (("fp32", W.FP32_AMP), ("fp64", W.FP64)):
            print(f"bench: serving {name} ({args.serving_seconds:g} s of arrivals)", file=sys.stderr, flush=True)
            sv = served(nuosc, W, args.serving_seconds, prec)
            line["serving"][name] = sv
            print(f"bench: serving {name}: {sv['completed']}/{sv['requests']} done, p50 {sv['p50_s']:.3f} s, "
                  f"p99 {sv['p99_s']:.3f} s, {sv['value']:.3e} beam-steps/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print(f"bench: cpu baseline ({args.cpu_attempts} oracle attempts)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(W, args.cpu_attempts)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
