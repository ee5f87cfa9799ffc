"""Query serving over a resident pool of B2SR graphs.

Queries (BFS, SSSP, CC, TC on one of the pool's graphs) arrive over time.  The
server admits them against a device-memory budget and batches them
continuously:

* BFS queries on one graph share a session of 64 frontier bits
  (``BfsSession``): a query takes a free bit between two levels and leaves when
  its bit reaches no new vertex, so queries that arrive while others run join
  the running levels instead of waiting for them.  SSSP queries join the same
  sessions: with unit edge weights their distances are the BFS levels (Sec. V,
  the diagonal as zero and each edge costing one), so concurrent SSSP queries
  on a graph are one multi-source job of up to 64 sources, mixed with its BFS
  queries;
* CC and TC are whole-graph jobs run on worker threads, each with its own
  stream, so their kernels overlap the BFS sessions on the device.  Concurrent
  queries asking the same whole-graph question share one job, and CC and TC
  results are kept per graph (the graphs do not change).

Memory accounting: a BFS session holds ``session_bytes(g)`` while it has
queries; each admitted query holds its result (and, for jobs, its workspace)
until it finishes.  A query whose need exceeds the whole budget is rejected;
one that does not fit now waits, and later queries that do fit may go first.

The executor does the device work; ``GpuExecutor`` drives libb2sr.so.  The
scheduler itself is plain host logic that any executor with the same methods
can drive (the tests use an executor backed by a CPU reference and a fake
clock).
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

KINDS = ("bfs", "sssp", "cc", "tc")
SESSION_KINDS = ("bfs", "sssp")  # answered by the 64-source BFS sessions


@dataclass
class Query:
    qid: int
    kind: str
    graph: int
    source: int = 0
    arrival: float = 0.0
    status: str = "new"          # new, queued, running, done, rejected, cancelled
    admitted: float | None = None
    finished: float | None = None
    result: object = None
    joined_step: int | None = None
    waited_for_memory: bool = False   # admission found the budget full at least once

    @property
    def latency(self) -> float | None:
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class _Session:
    graph: int
    handle: object
    nbytes: int
    slots: dict = field(default_factory=dict)   # slot -> Query
    start: dict = field(default_factory=dict)   # slot -> session step at join
    steps: int = 0
    in_flight: int | None = None                # number of the step in flight
    extracting: list = field(default_factory=list)  # (query, token) awaiting completion


@dataclass
class _Job:
    key: tuple
    future: object
    nbytes: int
    queries: list = field(default_factory=list)


class Server:
    """Continuous-batching scheduler (see the module docstring)."""

    def __init__(self, executor, budget_bytes: int, clock=time.perf_counter, cache: bool = True,
                 on_done=None, keep_results: bool = True, scan_limit: int = 256):
        self.ex = executor
        # queries a round may find unable to start before it stops looking: a
        # long queue behind a full budget otherwise costs every round a pass
        # over all of it
        self.scan_limit = int(scan_limit)
        self.on_done = on_done
        self.keep_results = keep_results
        self.budget = int(budget_bytes)
        self.clock = clock
        self.cache_on = cache
        self.in_use = 0
        self.peak_in_use = 0
        self.queue: list[Query] = []
        self.sessions: dict[int, _Session] = {}
        self.jobs: dict[tuple, _Job] = {}
        self.cache: dict[tuple, object] = {}
        self.done: list[Query] = []
        self.steps_run = 0
        self.ticks = 0
        self.tick_seconds = 0.0

    # ---- client side ----------------------------------------------------------
    def submit(self, q: Query):
        if q.kind not in KINDS:
            raise ValueError(f"unknown query kind {q.kind!r}")
        if q.kind in ("bfs", "sssp") and not 0 <= q.source < self.ex.graph_n(q.graph):
            raise ValueError("source out of range")
        q.status = "queued"
        if self._need(q, fresh=True) > self.budget:
            self._finish(q, "rejected")
            return
        self.queue.append(q)

    def cancel(self, q: Query):
        """Drops a queued or running query; its slot and memory are freed."""
        if q.status == "queued":
            self.queue.remove(q)
            self._finish(q, "cancelled")
        elif q.status == "running":
            for s in self.sessions.values():
                for slot, sq in list(s.slots.items()):
                    if sq is q:
                        self.ex.cancel(s.handle, slot)
                        del s.slots[slot]
                        self._release(self.ex.result_bytes(q.kind, q.graph))
                        self._finish(q, "cancelled")
                        return
            for job in self.jobs.values():
                if q in job.queries:
                    job.queries.remove(q)
                    self._release(self.ex.result_bytes(q.kind, q.graph))
                    self._finish(q, "cancelled")
                    return

    @property
    def idle(self) -> bool:
        return not self.queue and not self.jobs and not any(
            s.slots or s.extracting or s.in_flight is not None for s in self.sessions.values())

    # ---- memory -----------------------------------------------------------------
    def _need(self, q: Query, fresh: bool = False) -> int:
        """Bytes admitting q would add now (fresh: assume nothing is running)."""
        res = self.ex.result_bytes(q.kind, q.graph)
        if q.kind in SESSION_KINDS:
            if not fresh and q.graph in self.sessions:
                return res
            return res + self.ex.session_bytes(q.graph)
        return res + self.ex.job_bytes(q.kind, q.graph)

    def _take(self, nbytes: int) -> bool:
        if self.in_use + nbytes > self.budget:
            return False
        self.in_use += nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        return True

    def _release(self, nbytes: int):
        self.in_use -= nbytes
        assert self.in_use >= 0

    def _finish(self, q: Query, status: str, result=None):
        q.status = status
        q.finished = self.clock()
        q.result = result
        if self.on_done is not None:
            self.on_done(q)
        if not self.keep_results:
            q.result = None
        self.done.append(q)

    # ---- one scheduling round ---------------------------------------------------
    def tick(self) -> int:
        """One round: retire finished work, admit, step every session that has
        queries and no step in flight.  Returns the number of actions taken."""
        t0 = time.perf_counter()
        self.ticks += 1
        before = len(self.done) + self.steps_run
        queued = len(self.queue)
        self._retire_sessions()
        self._retire_jobs()
        self._admit()
        for s in self.sessions.values():
            if s.slots and s.in_flight is None:
                self.ex.step(s.handle)
                s.steps += 1
                s.in_flight = s.steps
                self.steps_run += 1
        for g in [g for g, s in self.sessions.items() if not s.slots and not s.extracting and s.in_flight is None]:
            s = self.sessions.pop(g)
            self.ex.close_session(s.handle)
            self._release(s.nbytes)
        self.tick_seconds += time.perf_counter() - t0
        return len(self.done) + self.steps_run - before + (queued - len(self.queue))

    def _retire_sessions(self):
        for s in self.sessions.values():
            still = []
            for q, token in s.extracting:
                if self.ex.token_ready(token):
                    self._release(self.ex.result_bytes(q.kind, q.graph))
                    self._finish(q, "done", self.ex.token_result(token))
                else:
                    still.append((q, token))
            s.extracting = still
            if s.in_flight is None or not self.ex.ready(s.handle):
                continue
            step, s.in_flight = s.in_flight, None
            alive = self.ex.alive(s.handle)
            for slot, q in list(s.slots.items()):
                if s.start[slot] < step and not (alive >> slot) & 1:
                    token = self.ex.extract(s.handle, slot)
                    del s.slots[slot]
                    s.extracting.append((q, token))

    def _retire_jobs(self):
        for key in [k for k, j in self.jobs.items() if j.future.done()]:
            job = self.jobs.pop(key)
            result = job.future.result()
            self._release(job.nbytes)
            if self.cache_on and key[0] in ("cc", "tc"):
                self.cache[key] = result
            for q in job.queries:
                self._release(self.ex.result_bytes(q.kind, q.graph))
                self._finish(q, "done", result)

    def _admit(self):
        waiting = []
        for i, q in enumerate(self.queue):
            if len(waiting) >= self.scan_limit:
                waiting.extend(self.queue[i:])  # the rest keep their order for later rounds
                break
            if not self._admit_one(q):
                waiting.append(q)
        self.queue = waiting

    def _admit_one(self, q: Query) -> bool:
        now = self.clock()
        res = self.ex.result_bytes(q.kind, q.graph)
        if q.kind in SESSION_KINDS:
            s = self.sessions.get(q.graph)
            if s is not None:
                free = [k for k in range(64) if k not in s.slots]
                if not free:
                    return False
                if not self._take(res):
                    q.waited_for_memory = True
                    return False
            else:
                nb = self.ex.session_bytes(q.graph)
                if not self._take(nb + res):
                    q.waited_for_memory = True
                    return False
                s = _Session(q.graph, self.ex.open_session(q.graph), nb)
                self.sessions[q.graph] = s
                free = list(range(64))
            slot = free[0]
            self.ex.join(s.handle, slot, q.source)
            s.slots[slot] = q
            s.start[slot] = s.steps
            q.joined_step = s.steps
        else:
            key = (q.kind, q.graph) if q.kind in ("cc", "tc") else (q.kind, q.graph, q.source)
            if key in self.cache:
                q.status, q.admitted = "running", now
                self._finish(q, "done", self.cache[key])
                return True
            job = self.jobs.get(key)
            if job is not None:
                if not self._take(res):
                    q.waited_for_memory = True
                    return False
                job.queries.append(q)
            else:
                nb = self.ex.job_bytes(q.kind, q.graph)
                if not self._take(nb + res):
                    q.waited_for_memory = True
                    return False
                job = _Job(key, self.ex.submit(q.kind, q.graph, q.source), nb, [q])
                self.jobs[key] = job
        q.status, q.admitted = "running", now
        return True

    # ---- driving a stream of arrivals ------------------------------------------
    def run(self, queries, sleep=time.sleep, max_ticks: int | None = None, idle_wait: float = 5e-5):
        """Submits each query at its arrival time (clock seconds from the start)
        and ticks until every query has finished.  Returns the finished queries."""
        pending = sorted(queries, key=lambda q: q.arrival)
        t0 = self.clock()
        for q in pending:
            q.arrival += t0
        i = ticks = 0
        while i < len(pending) or not self.idle:
            now = self.clock()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            acted = self.tick()
            ticks += 1
            if max_ticks is not None and ticks >= max_ticks:
                raise RuntimeError("serving loop did not finish")
            if self.idle and i < len(pending):
                sleep(max(0.0, pending[i].arrival - self.clock()))
            elif not acted:
                sleep(idle_wait)  # nothing ready: let worker threads run
        return self.done

    def stats(self) -> dict:
        done = [q for q in self.done if q.status == "done"]
        lat = np.array([q.latency for q in done], dtype=np.float64)
        out = {"queries": len(self.done), "done": len(done),
               "rejected": sum(q.status == "rejected" for q in self.done),
               "cancelled": sum(q.status == "cancelled" for q in self.done),
               "bfs_steps": self.steps_run, "ticks": self.ticks, "tick_seconds": self.tick_seconds,
               "peak_bytes_in_use": self.peak_in_use, "budget_bytes": self.budget,
               "waited_for_memory": sum(q.waited_for_memory for q in self.done)}
        if lat.size:
            out["p50_ms"] = float(np.percentile(lat, 50) * 1e3)
            out["p99_ms"] = float(np.percentile(lat, 99) * 1e3)
            span = max(q.finished for q in done) - min(q.arrival for q in done)
            out["queries_per_s"] = len(done) / span if span > 0 else float("inf")
            per = {}
            for k in KINDS:
                lk = np.array([q.latency for q in done if q.kind == k])
                if lk.size:
                    per[k] = {"n": int(lk.size), "p50_ms": float(np.percentile(lk, 50) * 1e3),
                              "p99_ms": float(np.percentile(lk, 99) * 1e3)}
            out["per_kind"] = per
        return out


# ---- the device executor -------------------------------------------------------

class GpuExecutor:
    """Runs the server's work on the GPU through libb2sr.so.  ``graphs`` is a
    list of (A, L) B2SR pairs: A for BFS/SSSP/CC, L (the strict lower
    triangle, at tile width ``tc_tile(A.tile)``) for TC, built on first use
    when None (``csrs`` then holds the graphs' CSR)."""

    def __init__(self, graphs, csrs=None, streams: int = 4, workers: int = 2):
        import torch

        from . import (ALGO_CC, ALGO_SSSP, B2SR, BfsSession, b2sr_algo_workspace_bytes, b2sr_bfs_session_bytes)
        self._torch = torch
        self._B2SR, self._Session = B2SR, BfsSession
        self.graphs = [list(p) for p in graphs]
        self.csrs = csrs
        self._sess_bytes = [b2sr_bfs_session_bytes(A.n) for A, _ in self.graphs]
        self._job_bytes = {
            "sssp": [b2sr_algo_workspace_bytes(A, ALGO_SSSP) for A, _ in self.graphs],
            "cc": [b2sr_algo_workspace_bytes(A, ALGO_CC) for A, _ in self.graphs],
            "tc": [8 for _ in self.graphs],
        }
        self._streams = [torch.cuda.Stream() for _ in range(streams)]
        self._next = 0
        self._pool = ThreadPoolExecutor(workers)
        self._local = threading.local()
        self._l_lock = threading.Lock()
        self.job_seconds = {k: 0.0 for k in ("sssp", "cc", "tc")}  # wall time of jobs, by kind
        self.job_count = {k: 0 for k in ("sssp", "cc", "tc")}

    def graph_n(self, g: int) -> int:
        return self.graphs[g][0].n

    def session_bytes(self, g: int) -> int:
        return self._sess_bytes[g]

    def job_bytes(self, kind: str, g: int) -> int:
        return self._job_bytes[kind][g]

    def result_bytes(self, kind: str, g: int) -> int:
        return 8 if kind == "tc" else 4 * self.graphs[g][0].n

    # sessions
    def open_session(self, g: int):
        stream = self._streams[self._next % len(self._streams)]
        self._next += 1
        return self._Session(self.graphs[g][0], stream=stream)

    def join(self, h, slot: int, source: int):
        h.join(slot, source)

    def step(self, h):
        h.step()

    def ready(self, h) -> bool:
        return h.ready()

    def alive(self, h) -> int:
        return h.alive()

    def extract(self, h, slot: int):
        out = h.extract(slot)
        ev = self._torch.cuda.Event()
        ev.record(h.stream)
        return (out, ev)

    def token_ready(self, token) -> bool:
        return token[1].query()

    def token_result(self, token):
        return token[0]

    def cancel(self, h, slot: int):
        h.cancel(slot)

    def close_session(self, h):
        h.stream.synchronize()  # the workspace is freed with the handle
        h.close()

    # whole-graph jobs, each on its worker thread's own stream
    def _stream(self):
        s = getattr(self._local, "stream", None)
        if s is None:
            s = self._local.stream = self._torch.cuda.Stream()
        return s

    @staticmethod
    def tc_tile(tile: int) -> int:
        """Tile width of the triangle-count operand: T = 4 tiles hold too few
        bits per tile pair for the masked product, and their tile-column range
        outgrows the product's LDS bitmap on large graphs, so they move to 8."""
        return max(tile, 8)

    def _lower(self, g: int):
        with self._l_lock:
            A, L = self.graphs[g]
            if L is None:
                c = self.csrs[g]
                L = self._B2SR.from_csr(c.rowptr, c.colind, c.n, self.tc_tile(A.tile), lower=True)
                self.graphs[g][1] = L
            return L

    def _run(self, kind: str, g: int, source: int):
        from . import b2sr_cc, b2sr_sssp, spgemm_masked
        torch = self._torch
        s = self._stream()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            A = self.graphs[g][0]
            if kind == "sssp":
                out, _ = b2sr_sssp(A, source)
            elif kind == "cc":
                out, _ = b2sr_cc(A)
            else:
                L = self._lower(g)
                out = spgemm_masked(L, L, L)
            s.synchronize()
        with self._l_lock:
            self.job_seconds[kind] += time.perf_counter() - t0
            self.job_count[kind] += 1
        return out

    def submit(self, kind: str, g: int, source: int):
        return self._pool.submit(self._run, kind, g, source)

    def shutdown(self):
        self._pool.shutdown(wait=True)
