"""Serving loop over the batch ABI: continuous batching of bulb-model runs.

Requests (workload dicts with an ``arrival_s`` time) arrive on the wall clock.
Arrived requests wait in a FIFO queue and are admitted into the batch as soon
as a slot and an arena gap of their footprint are free (``nuosc_batch_admit``
refuses otherwise); every tick advances all active runs together by a few
step attempts in one graph-replayed launch sequence, and finished runs are
retired, their survival probabilities read back, and their slot and memory
reused.  All the stepping runs in the library's HIP kernels; this module only
schedules.

``run_batched`` advances a fixed set of runs together (the batched workload);
``serve`` runs the arrival loop and reports completion latency (arrival to
result on the host) percentiles, throughput and queue depth.
"""

from __future__ import annotations

import collections
import time
from typing import Dict, List, Optional

import numpy as np

from . import nuosc


def _budget(ws: List[Dict], slack: float = 1.25) -> int:
    return int(sum(nuosc.footprint_bytes(w) for w in ws) * slack) + (64 << 20)


def run_batched(ws: List[Dict], attempts: int, warmup: int = 2, torch=None) -> Dict:
    """Admit every run, take `warmup` attempts, then time `attempts` attempts of
    all runs together.  Returns aggregate beam-steps/s over the timed attempts."""
    w0 = ws[0]
    b = nuosc.Batch.with_torch(len(ws), int(w0["n_flavors"]), int(w0["precision"]), int(w0["integrator"]),
                               _budget(ws))
    try:
        slots = [b.admit(w) for w in ws]
        if None in slots:
            raise RuntimeError("batch arena too small for the workload")
        b.step(warmup)
        acc0 = {s: b.query(s)["accepted"] for s in slots}
        if torch is not None:
            torch.cuda.synchronize()
        t = time.perf_counter()
        b.step(attempts)
        dt = time.perf_counter() - t
        beams = {s: b.num_beams(s) for s in slots}
        acc = {s: b.query(s)["accepted"] - acc0[s] for s in slots}
        bs = sum(beams[s] * acc[s] for s in slots)
        return dict(runs=len(ws), beams=int(sum(beams.values())), attempts=attempts, seconds=dt,
                    beam_steps=int(bs), value=bs / dt, ms_per_step=dt * 1e3 / attempts)
    finally:
        b.close()


def serve(requests: List[Dict], max_slots: int = 64, hbm_budget: Optional[int] = None,
          attempts_per_tick: int = 4, wall_limit_s: float = 600.0, keep: int = 0) -> Dict:
    """Continuous-batching loop over `requests` (sorted by ``arrival_s``).

    Returns latency percentiles (seconds, arrival -> probabilities on the
    host), completed count, aggregate beam-steps/s over the loop, queue-depth
    samples, and the results of the first `keep` completed requests (index,
    probabilities) for spot checks."""
    if not requests:
        raise ValueError("no requests")
    w0 = requests[0]
    if hbm_budget is None:
        hbm_budget = _budget(sorted(requests, key=nuosc.footprint_bytes)[-max_slots:])
    b = nuosc.Batch.with_torch(max_slots, int(w0["n_flavors"]), int(w0["precision"]), int(w0["integrator"]),
                               hbm_budget)
    arrivals = collections.deque(sorted(range(len(requests)), key=lambda i: requests[i]["arrival_s"]))
    queue: collections.deque = collections.deque()
    active: Dict[int, int] = {}          # slot -> request index
    latency: Dict[int, float] = {}
    beam_steps = 0
    depth = []
    kept = []
    busy_refusals = 0
    t0 = time.perf_counter()
    try:
        while arrivals or queue or active:
            now = time.perf_counter() - t0
            if now > wall_limit_s:
                break
            while arrivals and requests[arrivals[0]]["arrival_s"] <= now:
                queue.append(arrivals.popleft())
            while queue:
                s = b.admit(requests[queue[0]])
                if s is None:
                    busy_refusals += 1
                    break
                active[s] = queue.popleft()
            depth.append((now, len(queue), len(active)))
            if not active:
                if arrivals:
                    time.sleep(max(0.0, requests[arrivals[0]]["arrival_s"] - (time.perf_counter() - t0)))
                continue
            b.step(attempts_per_tick)
            for s in list(active):
                q = b.query(s)
                if not q["done"]:
                    continue
                i = active.pop(s)
                nbs = b.num_beams(s)
                p = b.retire(s)
                latency[i] = time.perf_counter() - t0 - requests[i]["arrival_s"]
                beam_steps += nbs * q["accepted"]
                if q["status"] != nuosc.OK:
                    raise RuntimeError(f"request {i} stopped with status {q['status']}")
                if len(kept) < keep:
                    kept.append((i, p))
        elapsed = time.perf_counter() - t0
    finally:
        b.close()
    lat = np.array(sorted(latency.values())) if latency else np.array([np.nan])
    return dict(
        requests=len(requests),
        completed=len(latency),
        p50_s=float(np.percentile(lat, 50)),
        p99_s=float(np.percentile(lat, 99)),
        max_s=float(lat.max()),
        elapsed_s=elapsed,
        beam_steps=int(beam_steps),
        value=beam_steps / elapsed,
        max_queue=max((d[1] for d in depth), default=0),
        max_active=max((d[2] for d in depth), default=0),
        busy_refusals=busy_refusals,
        kept=kept,
    )
