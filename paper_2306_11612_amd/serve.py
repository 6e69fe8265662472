"""Serving volume-line updates over resident volumes.

Clients send TF-update requests (a volume, one alpha table per field, a plot
width); the server keeps every volume resident in HBM in Hilbert order and
answers each request with its bins.  Two policies:

* ``batch``: continuous batching.  Whenever one of the launch slots (an
  executor and its own stream) is free, the waiting requests are admitted in
  arrival order while they fit the device-memory budget (workspace and
  outputs, ``dvl_request_bytes``) and the batch limit, and run as one
  ``dvl_update_batch``: one launch per kernel phase for the whole batch, and
  the requests on one volume share each read of its cells.
* ``fifo``: the plain form: one request at a time, in arrival order.

The scheduling logic (``Scheduler``) is host code over an engine interface,
so it is tested without a GPU; ``GpuEngine`` is the engine over the C ABI.

    python -m paper_2306_11612_amd.serve --rates 50,200,1000 --duration 5
"""
from __future__ import annotations

import argparse
import gc
import collections
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    """One client request and its life cycle (times in seconds)."""
    rid: int
    volume: str
    alpha: np.ndarray                  # [M][n_tf] float32
    n_bins: int
    params: dict = field(default_factory=dict)
    arrival: float = 0.0
    admitted: float | None = None
    done: float | None = None
    bytes: int = 0
    out: object = None                 # engine-owned outputs while admitted

    @property
    def latency(self) -> float:
        return (self.done - self.arrival) if self.done is not None else math.nan


class Scheduler:
    """Admission by memory, continuous batching over `engine` slots.

    engine interface:
      n_slots                        launch slots that may run at once
      request_bytes(job) -> int      device bytes the job holds while admitted
      start(slot, jobs) -> handle    allocate outputs, enqueue the batch
      finished(handle) -> bool       non-blocking completion test
      release(jobs)                  outputs no longer needed
    """

    def __init__(self, engine, budget_bytes: int, max_batch: int = 32, policy: str = "batch",
                 keep_outputs: bool = False):
        if policy not in ("batch", "fifo"):
            raise ValueError(f"unknown policy {policy}")
        self.engine = engine
        self.budget = int(budget_bytes)
        self.max_batch = 1 if policy == "fifo" else int(max_batch)
        self.n_slots = 1 if policy == "fifo" else int(engine.n_slots)
        self.policy = policy
        self.keep_outputs = keep_outputs
        self.queue: collections.deque[Job] = collections.deque()
        self.running: dict[int, tuple[object, list[Job]]] = {}
        self.used = 0
        self.peak_used = 0
        self.completed: list[Job] = []
        self.batches: list[int] = []
        self.max_running = 0               # most slots seen busy at once (overlap on the device)
        self.max_shared = 0                # most requests of one batch on one volume (shared reads)

    def submit(self, job: Job):
        job.bytes = int(self.engine.request_bytes(job))
        if job.bytes > self.budget:
            raise ValueError(f"request {job.rid} needs {job.bytes} bytes, above the budget {self.budget}")
        self.queue.append(job)

    def idle(self) -> bool:
        return not self.queue and not self.running

    def _poll(self, now: float) -> list[Job]:
        finished = []
        for slot in list(self.running):
            handle, jobs = self.running[slot]
            if self.engine.finished(handle):
                del self.running[slot]
                for j in jobs:
                    j.done = now
                    self.used -= j.bytes
                if not self.keep_outputs:
                    self.engine.release(jobs)
                finished.extend(jobs)
        self.completed.extend(finished)
        return finished

    def _admit(self, now: float) -> list[Job]:
        batch = []
        while self.queue and len(batch) < self.max_batch:
            j = self.queue[0]
            if self.used + j.bytes > self.budget:
                break                      # strict arrival order: nothing overtakes
            self.queue.popleft()
            self.used += j.bytes
            j.admitted = now
            batch.append(j)
        self.peak_used = max(self.peak_used, self.used)
        return batch

    def step(self, now: float) -> list[Job]:
        """Collect finished batches, then fill every free slot."""
        finished = self._poll(now)
        for slot in range(self.n_slots):
            if slot in self.running or not self.queue:
                continue
            batch = self._admit(now)
            if not batch:
                break
            self.running[slot] = (self.engine.start(slot, batch), batch)
            self.batches.append(len(batch))
            self.max_running = max(self.max_running, len(self.running))
            per_volume = collections.Counter(j.volume for j in batch)
            self.max_shared = max(self.max_shared, max(per_volume.values()))
        return finished


def percentiles(lat: list[float]) -> dict:
    a = np.sort(np.asarray(lat, np.float64))
    if a.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None}
    q = lambda p: float(a[min(a.size - 1, int(math.ceil(p * a.size)) - 1)] * 1e3)
    return {"p50_ms": q(0.50), "p99_ms": q(0.99), "mean_ms": float(a.mean() * 1e3)}


def run_open_loop(sched: Scheduler, jobs: list[Job], clock=time.perf_counter, spin_s: float = 0.0) -> dict:
    """Drive `sched` with jobs whose `arrival` fields are offsets from the
    start (open loop: arrivals do not wait for completions)."""
    t0 = clock()
    pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
    for j in pending:
        j.arrival += t0
    while pending or not sched.idle():
        now = clock()
        while pending and pending[0].arrival <= now:
            sched.submit(pending.popleft())
        sched.step(now)
        if spin_s:
            time.sleep(spin_s)
    t1 = clock()
    lat = [j.latency for j in sched.completed]
    out = {"requests": len(sched.completed), "wall_s": t1 - t0,
           "throughput_rps": len(sched.completed) / max(t1 - t0, 1e-9),
           "mean_batch": float(np.mean(sched.batches)) if sched.batches else 0.0,
           "max_batch": int(max(sched.batches)) if sched.batches else 0,
           "max_running_slots": sched.max_running, "max_requests_on_one_volume": sched.max_shared,
           "peak_bytes": sched.peak_used}
    out.update(percentiles(lat))
    return out


# ---------------------------------------------------------------- GPU engine

class HostBins:
    """Pinned host copies of one request's bins (what a client receives)."""

    def __init__(self, torch, n_bins: int, n_fields: int):
        pin = dict(device="cpu", pin_memory=True)
        self.first = torch.empty(n_bins, dtype=torch.int32, **pin)
        self.last = torch.empty(n_bins, dtype=torch.int32, **pin)
        self.stats = torch.empty(4, n_fields, n_bins, dtype=torch.float32, **pin)   # mean, min, max, y

    def copy_from(self, b):
        self.first.copy_(b.first_cell, non_blocking=True)
        self.last.copy_(b.last_cell, non_blocking=True)
        for k, t in enumerate((b.mean, b.vmin, b.vmax, b.y)):
            self.stats[k].copy_(t, non_blocking=True)


class GpuEngine:
    """Engine over the C ABI: one executor and one stream (default priority)
    per slot, and pools of device outputs and pinned host copies per (fields,
    width).  A request is complete when its bins are on the host: the
    device-to-host copy is part of its latency."""

    def __init__(self, volumes: dict, n_slots: int = 2, copy_to_host: bool = True):
        import torch
        from . import dvl
        self.dvl = dvl
        self.torch = torch
        self.volumes = volumes
        self.n_slots = n_slots
        self.copy_to_host = copy_to_host
        self.slots = [(dvl.Executor(), torch.cuda.Stream()) for _ in range(n_slots)]
        self.pool: dict[tuple[int, int], list] = collections.defaultdict(list)

    def request_bytes(self, job: Job) -> int:
        return self.dvl.request_bytes(self.volumes[job.volume], job.n_bins)

    def _bins(self, M: int, W: int):
        p = self.pool[(M, W)]
        if p:
            return p.pop()
        b = self.dvl.Bins(W, M)
        b.host = HostBins(self.torch, W, M) if self.copy_to_host else None
        return b

    def start(self, slot: int, jobs: list[Job]):
        ex, stream = self.slots[slot]
        reqs = []
        for j in jobs:
            V = self.volumes[j.volume]
            j.out = self._bins(V.m, j.n_bins)
            reqs.append(self.dvl.Request(V, j.alpha, j.out, **j.params))
        # the stream must not read output buffers before earlier users of the pool are done
        stream.wait_stream(self.torch.cuda.current_stream())
        ex.update_batch(reqs, stream=stream)
        if self.copy_to_host:
            with self.torch.cuda.stream(stream):
                for j in jobs:
                    j.out.host.copy_from(j.out)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def finished(self, handle) -> bool:
        return handle.query()

    def release(self, jobs: list[Job]):
        for j in jobs:
            if j.out is not None:
                self.pool[(j.out.n_fields, j.out.n_bins)].append(j.out)
                j.out = None

    def close(self):
        for ex, _ in self.slots:
            ex.close()


def make_requests(volume_ids: list[str], n_fields: dict, rate: float, duration: float, max_requests: int,
                  seed: int, widths=(1024, 1920, 3840), n_tf: int = 256, tf_pool: int = 64) -> list[Job]:
    """Open-loop Poisson arrivals: exponential gaps at `rate`, volume uniform,
    width uniform over `widths`, every field's TF drawn from a seeded pool of
    piecewise-linear tables with 4-8 control points."""
    import synth
    from synth.noise import substream
    rng = np.random.default_rng(substream(seed, 4))
    n = int(min(max_requests, max(1, round(rate * duration))))
    gaps = rng.exponential(1.0 / rate, n)
    arrivals = np.cumsum(gaps) - gaps[0]
    tables = {}
    for vid in sorted(set(volume_ids)):
        M = n_fields[vid]
        tables[vid] = [np.stack([t.numpy() for t in synth.make_tfs(seed + 7919 * k + M, M, (4, 8), n_tf)])
                       for k in range(tf_pool)]
    jobs = []
    for i in range(n):
        vid = volume_ids[int(rng.integers(len(volume_ids)))]
        A = tables[vid][int(rng.integers(tf_pool))]
        W = int(widths[int(rng.integers(len(widths)))])
        jobs.append(Job(i, vid, A, W, arrival=float(arrivals[i])))
    return jobs


def main(argv=None):
    import os
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    from . import dvl
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", default="10,50,150,300", help="resident volumes, millions of cells")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--max-requests", type=int, default=2000)
    ap.add_argument("--policies", default="batch,fifo")
    ap.add_argument("--budget-gb", type=float, default=8.0)
    ap.add_argument("--max-batch", type=int, default=32)
    ap.add_argument("--slots", type=int, default=2)
    args = ap.parse_args(argv)

    def log(m):
        print(f"[serve] {m}", file=sys.stderr, flush=True)

    sizes = [int(s) for s in args.sizes.split(",")]
    volumes, n_fields = {}, {}
    for i, mc in enumerate(sizes):
        t = time.perf_counter()
        vol = synth.cfg5_volume(i, device="cuda", sizes=[mc * 1e6 for mc in sizes])
        V = dvl.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
        vid = f"amr4_{mc}m"
        volumes[vid], n_fields[vid] = V, V.m
        del vol
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"{vid}: {V.n} cells resident ({V.nbytes / 1e9:.2f} GB) in {time.perf_counter() - t:.1f} s")
    ids = sorted(volumes)
    engine = GpuEngine(volumes, n_slots=args.slots)
    try:
        # warm both paths (executor workspaces, kernels)
        warm = make_requests(ids, n_fields, 1000.0, 0.05, 50, synth.SEED + 99)
        for pol in args.policies.split(","):
            run_open_loop(Scheduler(engine, int(args.budget_gb * 1e9), args.max_batch, pol), warm)
            for j in warm:
                j.arrival, j.done, j.admitted = 0.0, None, None
        # the long-lived objects (torch, the volumes) go to the permanent
        # generation, so a full collection does not walk them between requests
        gc.collect()
        gc.freeze()
        for rate in [float(r) for r in args.rates.split(",")]:
            for pol in args.policies.split(","):
                jobs = make_requests(ids, n_fields, rate, args.duration, args.max_requests, synth.SEED + 5)
                sched = Scheduler(engine, int(args.budget_gb * 1e9), args.max_batch, pol)
                res = run_open_loop(sched, jobs)
                res.update({"policy": pol, "rate_rps": rate, "volumes": ids, "slots": sched.n_slots,
                            "budget_gb": args.budget_gb})
                print(json.dumps(res), flush=True)
                log(f"rate {rate:g} {pol}: p50 {res['p50_ms']:.2f} ms p99 {res['p99_ms']:.2f} ms "
                    f"throughput {res['throughput_rps']:.0f} req/s mean batch {res['mean_batch']:.1f}")
    finally:
        engine.close()
        for V in volumes.values():
            V.close()


if __name__ == "__main__":
    main()
