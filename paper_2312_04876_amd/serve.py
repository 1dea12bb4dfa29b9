"""Continuous-batching Louvain server.

Jobs (graphs) arrive at any time.  A scheduler thread admits queued jobs, in
arrival order, into batches as soon as an execution slot and device memory
are free: a batch takes every queued job that fits the memory budget (a job's
footprint is its share of a batch workspace plus its CSR), up to a job and
entry cap.  Each slot runs its batch as one union run (independent graphs,
each with its own convergence and stop tests, so a job's result is the one it
would get alone; bit for bit in deterministic mode) on its own stream, so
batches on different slots overlap on the device while new arrivals queue.
Latency is measured from submission to completion.

The scheduler knows nothing about GPUs: an executor provides footprints and
runs batches.  GpuExecutor runs them through the HIP library (graphs kept
resident on the device); tests drive the scheduler with a CPU executor.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional, Sequence


@dataclass
class Job:
    """A request: run Louvain on graph `key` of the executor's pool."""
    key: Any
    nnz: int
    n: int
    id: int = -1
    submitted: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0
    slot: int = -1
    batch: int = -1
    membership: Any = None
    modularity: float = float("nan")
    error: Optional[str] = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.finished - self.submitted


class Server:
    """Continuous batching over `slots` execution slots within `memory_budget` bytes.

    executor.footprint(job) -> bytes the job needs while its batch runs;
    executor.run(jobs, slot) -> list of (membership, modularity), one per job.
    """

    def __init__(self, executor, memory_budget: int, slots: int = 4, max_jobs: int = 512,
                 max_entries: int = 1 << 30, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(memory_budget)
        self.slots = int(slots)
        self.max_jobs = int(max_jobs)
        self.max_entries = int(max_entries)
        self.clock = clock
        self._cv = threading.Condition()
        self._queue: collections.deque = collections.deque()
        self._free_slots = list(range(self.slots))
        self._in_use = 0
        self._peak_use = 0
        self._next_id = 0
        self._batches = 0
        self._stop = False
        self._workers: List[threading.Thread] = []
        self.completed: List[Job] = []
        self._sched = threading.Thread(target=self._schedule, name="louvain-scheduler", daemon=True)
        self._sched.start()

    # -- client side
    def submit(self, job: Job) -> Job:
        with self._cv:
            if self._stop:
                raise RuntimeError("server is closed")
            job.id = self._next_id
            self._next_id += 1
            job.submitted = self.clock()
            if self.ex.footprint(job) > self.budget:
                job.error = "job needs more memory than the server's budget"
                job.finished = job.submitted
                job.done.set()
                self.completed.append(job)
                return job
            self._queue.append(job)
            self._cv.notify_all()
        return job

    def drain(self, timeout: Optional[float] = None) -> bool:
        """Wait until every submitted job has finished."""
        end = None if timeout is None else time.monotonic() + timeout
        with self._cv:
            while self._queue or len(self._free_slots) < self.slots:
                left = None if end is None else end - time.monotonic()
                if left is not None and left <= 0:
                    return False
                self._cv.wait(left)
        return True

    def close(self):
        self.drain()
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._sched.join()
        for w in self._workers:
            w.join()

    @property
    def peak_memory(self) -> int:
        return self._peak_use

    @property
    def batches(self) -> int:
        return self._batches

    # -- scheduler side
    def _take_batch(self) -> List[Job]:
        """Queued jobs, in arrival order, that fit the free memory (caller holds the lock)."""
        batch, mem, ent = [], 0, 0
        while self._queue and len(batch) < self.max_jobs:
            job = self._queue[0]
            need = self.ex.footprint(job)
            if self._in_use + mem + need > self.budget:
                break
            if batch and ent + job.nnz > self.max_entries:
                break
            self._queue.popleft()
            batch.append(job)
            mem += need
            ent += job.nnz
        return batch

    def _schedule(self):
        with self._cv:
            while True:
                while not self._stop and not (self._queue and self._free_slots):
                    self._cv.wait()
                if self._stop:
                    return
                batch = self._take_batch()
                if not batch:
                    # the head job waits for memory held by running batches
                    self._cv.wait()
                    continue
                slot = self._free_slots.pop()
                mem = sum(self.ex.footprint(j) for j in batch)
                self._in_use += mem
                self._peak_use = max(self._peak_use, self._in_use)
                bid = self._batches
                self._batches += 1
                now = self.clock()
                for j in batch:
                    j.admitted, j.slot, j.batch = now, slot, bid
                t = threading.Thread(target=self._work, args=(batch, slot, mem),
                                     name="louvain-slot%d" % slot, daemon=True)
                self._workers.append(t)
                t.start()

    def _work(self, batch: List[Job], slot: int, mem: int):
        err = None
        try:
            results = self.ex.run(batch, slot)
        except Exception as e:  # the batch fails as a whole; the server goes on
            results, err = None, "%s: %s" % (type(e).__name__, e)
        now = self.clock()
        with self._cv:
            for k, j in enumerate(batch):
                if results is not None:
                    j.membership, j.modularity = results[k]
                else:
                    j.error = err
                j.finished = now
                self.completed.append(j)
                j.done.set()
            self._in_use -= mem
            self._free_slots.append(slot)
            self._cv.notify_all()


def latency_stats(jobs: Sequence[Job]) -> Dict[str, float]:
    lat = sorted(j.latency for j in jobs if j.error is None)
    if not lat:
        return {"count": 0}

    def pct(p):
        k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[k]
    return {"count": len(lat), "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3,
            "max_ms": lat[-1] * 1e3, "mean_ms": sum(lat) / len(lat) * 1e3}


class GpuExecutor:
    """Runs batches through the HIP library; the pool's graphs stay resident on the device.

    pool: {key: graphgen.CSR}.  Each slot has its own stream.  params: Louvain parameters
    (deterministic mode by default, so a job's result is exactly its standalone result).
    """

    def __init__(self, pool: Dict[Any, Any], slots: int, device=None, **params):
        import numpy as np
        import torch

        from . import binding
        self.torch = torch
        self.binding = binding
        self.params = dict(params)
        self.params.setdefault("mode", "deterministic")
        self.device = device or torch.device("cuda:0")
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.graphs = {}
        for key, csr in pool.items():
            self.graphs[key] = (
                torch.from_numpy(csr.offsets32()).to(self.device),
                torch.from_numpy(np.ascontiguousarray(csr.targets, dtype=np.int32)).to(self.device),
                torch.from_numpy(np.ascontiguousarray(csr.weights, dtype=np.int32)).to(self.device),
                int(csr.weights[:csr.nnz].sum(dtype=np.int64)) if csr.nnz else 0)
        self._cp = binding.make_params(**self.params)
        torch.cuda.synchronize(self.device)

    def footprint(self, job: Job) -> int:
        # its part of a batch workspace (an upper bound: the batch's own size is the sum of
        # the per-job sizes minus the shared scalars) plus its copy in the union CSR
        ws = self.binding.batch_workspace_bytes(1, job.n, job.nnz, -1, self._cp)
        return ws + 4 * (job.n + 1) + 8 * job.nnz

    def run(self, jobs: List[Job], slot: int):
        torch = self.torch
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            offs, tgts, ws, go = [], [], [], [0]
            vbase, ebase = 0, 0
            for j in jobs:
                off, tgt, w, _ = self.graphs[j.key]
                offs.append(off[:-1] + ebase if j.n else off[:0])
                tgts.append(tgt + vbase)
                ws.append(w)
                vbase += j.n
                ebase += j.nnz
                go.append(vbase)
            offs.append(torch.tensor([ebase], dtype=torch.int32, device=self.device))
            off = torch.cat(offs).contiguous()
            tgt = torch.cat(tgts).contiguous() if ebase else torch.zeros(1, dtype=torch.int32,
                                                                          device=self.device)
            w = torch.cat(ws).contiguous() if ebase else torch.ones(1, dtype=torch.int32,
                                                                   device=self.device)
            tgt, w = tgt[:ebase], w[:ebase]
            ctx = self.binding.Louvain(off, tgt, w, stream=stream,
                                       graph_offsets=torch.tensor(go, dtype=torch.int32),
                                       **self.params)
            try:
                memb, _q, _st = ctx.run()
                qs, _c = ctx.batch_results()
                parts = ctx.split_membership(memb)
            finally:
                ctx.close()
        return list(zip(parts, qs))
