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
import hashlib
import time
from typing import Dict, List, Optional

import numpy as np

from . import nuosc


def _budget(ws: List[Dict], slack: float = 1.25) -> int:
    return int(sum(nuosc.footprint_bytes(w) for w in ws) * slack) + (64 << 20)


def run_batched(ws: List[Dict], attempts: int, reps: int = 3, torch=None) -> Dict:
    """Admit every run, then step all of them together by `attempts` attempts
    per batch step: the first step launches directly, the second captures the
    launch sequence as a HIP graph and replays it, and the `reps` timed steps
    after them are graph replays.  Returns aggregate beam-steps/s over the
    timed steps (host wall clock, each step ends with the control blocks on
    the host) and the batch's graph statistics."""
    w0 = ws[0]
    b = nuosc.Batch.with_torch(len(ws), int(w0["n_flavors"]), int(w0["precision"]), int(w0["integrator"]),
                               _budget(ws))
    try:
        slots = [b.admit(w) for w in ws]
        if None in slots:
            raise RuntimeError("batch arena too small for the workload")
        b.step(attempts)
        b.step(attempts)
        before = b.graph_stats()
        acc0 = {s: b.query(s)["accepted"] for s in slots}
        if torch is not None:
            torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            b.step(attempts)
            times.append(time.perf_counter() - t)
        after = b.graph_stats()
        beams = {s: b.num_beams(s) for s in slots}
        acc = {s: b.query(s)["accepted"] - acc0[s] for s in slots}
        bs = sum(beams[s] * acc[s] for s in slots)
        dt = sum(times)
        return dict(runs=len(ws), beams=int(sum(beams.values())), attempts_per_step=attempts, timed_steps=reps,
                    seconds=dt, step_seconds=[round(x, 6) for x in times], beam_steps=int(bs), value=bs / dt,
                    ms_per_attempt=dt * 1e3 / (reps * attempts),
                    timed_steps_replayed=after["graph"] - before["graph"],
                    timed_steps_eager=after["eager"] - before["eager"], graph_stats=after)
    finally:
        b.close()


def digest(p: np.ndarray) -> str:
    """Digest of a probability array (bitwise comparisons without keeping it)."""
    return hashlib.sha256(np.ascontiguousarray(p).tobytes()).hexdigest()


def serve(requests: List[Dict], max_slots: int = 64, hbm_budget: Optional[int] = None,
          attempts_per_tick: int = 4, duration_s: Optional[float] = None, drain_s: float = 0.0) -> Dict:
    """Continuous-batching loop over `requests` (sorted by ``arrival_s``).

    Requests join a FIFO queue at their arrival time and are admitted as soon
    as a slot and an arena gap are free; every tick advances all active runs
    by `attempts_per_tick` attempts (a graph replay when the active set and
    count repeat) and retires the finished ones.  The loop ends when every
    request is done, or `drain_s` seconds after the last arrival time
    (`duration_s`, default: the last request's arrival), whichever is first;
    unfinished requests are reported, not dropped silently.

    Returns completion latencies (arrival to probabilities on the host, queue
    wait included) of the completed requests, the beam-steps done (completed
    requests and the accepted steps of the ones still active at the end), the
    queue depth and active count sampled once a second, the batch's graph
    statistics, and a digest of every completed request's probabilities."""
    if not requests:
        raise ValueError("no requests")
    w0 = requests[0]
    if hbm_budget is None:
        hbm_budget = _budget(sorted(requests, key=nuosc.footprint_bytes)[-max_slots:])
    if duration_s is None:
        duration_s = max(r["arrival_s"] for r in requests)
    b = nuosc.Batch.with_torch(max_slots, int(w0["n_flavors"]), int(w0["precision"]), int(w0["integrator"]),
                               hbm_budget)
    arrivals = collections.deque(sorted(range(len(requests)), key=lambda i: requests[i]["arrival_s"]))
    queue: collections.deque = collections.deque()
    active: Dict[int, int] = {}          # slot -> request index
    latency: Dict[int, float] = {}
    digests: Dict[int, str] = {}
    beam_steps = 0
    series = []                          # (t, queue depth, active) once a second
    next_sample = 0.0
    busy_refusals = 0
    ticks = 0
    t0 = time.perf_counter()
    try:
        while arrivals or queue or active:
            now = time.perf_counter() - t0
            if now > duration_s + drain_s:
                break
            while arrivals and requests[arrivals[0]]["arrival_s"] <= now:
                queue.append(arrivals.popleft())
            while queue:
                s = b.admit(requests[queue[0]])
                if s is None:
                    busy_refusals += 1
                    break
                active[s] = queue.popleft()
            if now >= next_sample:
                series.append((round(now, 2), len(queue), len(active)))
                next_sample += 1.0
            if not active:
                if arrivals:
                    time.sleep(max(0.0, requests[arrivals[0]]["arrival_s"] - (time.perf_counter() - t0)))
                continue
            b.step(attempts_per_tick)
            ticks += 1
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
                digests[i] = digest(p)
        elapsed = time.perf_counter() - t0
        partial = 0
        for s, i in active.items():
            partial += b.num_beams(s) * b.query(s)["accepted"]
        graph = b.graph_stats()
    finally:
        b.close()
    lat = np.array(sorted(latency.values())) if latency else np.array([np.nan])
    waits = [elapsed - requests[i]["arrival_s"] for i in list(queue) + list(active.values())]
    total = beam_steps + partial
    return dict(
        requests=len(requests),
        completed=len(latency),
        unfinished_active=len(active),
        unfinished_queued=len(queue),
        never_arrived=len(arrivals),
        p50_s=float(np.percentile(lat, 50)),
        p99_s=float(np.percentile(lat, 99)),
        max_s=float(lat.max()),
        unfinished_wait_max_s=float(max(waits)) if waits else 0.0,
        elapsed_s=elapsed,
        beam_steps=int(total),
        beam_steps_completed=int(beam_steps),
        value=total / elapsed,
        max_queue=max((d[1] for d in series), default=0),
        max_active=max((d[2] for d in series), default=0),
        queue_series=series,
        busy_refusals=busy_refusals,
        ticks=ticks,
        graph_stats=graph,
        graph_share=graph["graph"] / max(1, graph["graph"] + graph["eager"]),
        digests=digests,
    )
