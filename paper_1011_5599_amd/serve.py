"""Continuous-batching server for HyperANF requests on one GPU.

A request is one graph, a register count m = 2^log2m and a hash seed. The server:
- admits arrived requests while their device footprint (graph, two register arrays,
  flags, sums; `hanf_footprint`) fits the HBM budget;
- puts the requests admitted together that share m (and, by default, a size class:
  footprints within a factor of 4) into one batch, whose passes advance all of them at
  once (cross-graph iteration batching; the disjoint-union batch of the library);
- keeps every batch's counters resident on the device until its last request is done, each
  batch on its own HIP stream, so batches admitted at different times overlap;
- polls without blocking (`hanf_poll`) and completes a request as soon as its own component
  reaches its fixpoint, even while the rest of its batch still iterates; its results are
  N_hat(0..T), T, the statistics and, optionally, the counters;
- returns a batch's memory to the budget when its last request is done, which lets waiting
  requests in; its context (stream and device buffers) is kept for the next batch, since
  freeing device memory would wait for every stream of the device.

Every request's results equal those of the same request run alone (the batch components
are independent runs).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import (HANF_BUSY, HANF_DONE, Batch, hanf_batch_info, hanf_batch_read_nt,
               hanf_batch_read_registers, hanf_batch_stats_all, hanf_enqueue, hanf_footprint, hanf_poll)


@dataclass
class Request:
    rid: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    log2m: int
    seed: int
    arrival: float = 0.0
    admitted: float | None = None
    finish: float | None = None
    nt: np.ndarray | None = None
    T: int | None = None
    stats: dict | None = None
    registers: np.ndarray | None = None

    @property
    def n(self):
        return len(self.row_ptr) - 1

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival


@dataclass
class _Flight:
    batch: Batch
    requests: list
    footprint: int
    open: set = field(default_factory=set)


def footprint(req: Request) -> int:
    """Device bytes a request needs inside a batch (its graph copy, expanded graph, run
    state; padding to 64 nodes included)."""
    n_pad = (req.n + 63) // 64 * 64
    return hanf_footprint(n_pad, len(req.col_idx), req.log2m, 1) + 4 * (len(req.col_idx) + req.n + 1)


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 96 << 30, max_batches: int = 4,
                 passes_per_poll: int = 2, keep_registers: bool = False, max_batch_requests: int = 64,
                 size_classes: bool = True, clock=time.perf_counter, **options):
        self.device = device
        self.budget = hbm_budget
        self.max_batches = max_batches
        self.passes_per_poll = passes_per_poll
        self.keep_registers = keep_registers
        self.max_batch_requests = max_batch_requests
        # With size classes, a batch also holds only requests whose footprints are within a
        # factor of 4 of each other: a batch's pass covers every component, so a small graph
        # batched with a large one would advance at the large one's pass time.
        self.size_classes = size_classes
        self.clock = clock
        self.options = options
        self.waiting = collections.deque()
        self.flights: list[_Flight] = []
        self.used = 0
        self.done: list[Request] = []
        self.max_flights = 0       # most batches in flight at once
        self.batch_sizes: list[int] = []
        self.idle_batches: list[Batch] = []
        self.host_s = {"admit": 0.0, "collect": 0.0, "poll": 0.0}

    # -- admission
    def submit(self, req: Request) -> None:
        if footprint(req) > self.budget:
            raise ValueError(f"request {req.rid} needs more than the HBM budget")
        self.waiting.append(req)

    def _admit(self):
        t0 = self.clock()
        try:
            self._admit_groups()
        finally:
            self.host_s["admit"] += self.clock() - t0

    def _admit_groups(self):
        while self.waiting and len(self.flights) < self.max_batches:
            m = self.waiting[0].log2m
            key = self._class(self.waiting[0])
            group, room = [], self.budget - self.used
            for r in list(self.waiting):
                if r.log2m != m or len(group) >= self.max_batch_requests or self._class(r) != key:
                    continue
                fp = footprint(r)
                if fp > room:
                    if not group:
                        return  # the oldest request does not fit yet: wait for memory
                    continue
                group.append(r)
                room -= fp
            if not group:
                return
            for r in group:
                self.waiting.remove(r)
            fp = sum(footprint(r) for r in group)
            bt = self.idle_batches.pop() if self.idle_batches else Batch(self.device, **self.options)
            now = self.clock()
            bt.load_graphs([(r.row_ptr, r.col_idx) for r in group], 1)
            bt.init(m, [r.seed for r in group])
            hanf_enqueue(bt.ctx, self.passes_per_poll)
            for r in group:
                r.admitted = now
            self.used += fp
            self.flights.append(_Flight(bt, group, fp, set(range(len(group)))))
            self.batch_sizes.append(len(group))
            self.max_flights = max(self.max_flights, len(self.flights))

    def _class(self, r: Request) -> int:
        return footprint(r).bit_length() // 2 if self.size_classes else 0

    # -- completion
    def _collect(self, fl: _Flight, finished_all: bool):
        _, T = hanf_batch_info(fl.batch.ctx)
        ready = [c for c in sorted(fl.open) if T[c] >= 0 or finished_all]
        if not ready:
            return []
        st = hanf_batch_stats_all(fl.batch.ctx)
        now = self.clock()
        out = []
        for c in ready:
            r = fl.requests[c]
            r.nt = hanf_batch_read_nt(fl.batch.ctx, c)
            r.T = len(r.nt) - 1
            r.stats = {k: v[c] for k, v in st.items()}
            if self.keep_registers:
                r.registers = hanf_batch_read_registers(fl.batch.ctx, c, r.n, r.log2m)
            r.finish = now
            fl.open.discard(c)
            out.append(r)
        return out

    def pump(self) -> list[Request]:
        """One round: admit what fits, poll every batch, keep the unfinished ones going.
        Returns the requests completed in this round."""
        self._admit()
        finished = []
        for fl in list(self.flights):
            t0 = self.clock()
            st, _ = hanf_poll(fl.batch.ctx)
            t1 = self.clock()
            self.host_s["poll"] += t1 - t0
            if st == HANF_BUSY:
                continue
            finished += self._collect(fl, st == HANF_DONE)
            self.host_s["collect"] += self.clock() - t1
            if st == HANF_DONE or not fl.open:
                self.idle_batches.append(fl.batch)
                self.used -= fl.footprint
                self.flights.remove(fl)
            else:
                hanf_enqueue(fl.batch.ctx, self.passes_per_poll)
        self.done += finished
        return finished

    def idle(self) -> bool:
        return not self.waiting and not self.flights

    def close(self):
        for fl in self.flights:
            fl.batch.close()
        for bt in self.idle_batches:
            bt.close()
        self.flights, self.idle_batches = [], []

    def warm_up(self, requests):
        """Serves copies of `requests` once (arrivals ignored) so that the contexts hold
        device buffers of the sizes the trace needs."""
        import copy
        reqs = [copy.copy(r) for r in requests]
        for r in reqs:
            r.arrival = 0.0
        self.serve_trace(reqs)
        self.done = []

    def serve_trace(self, requests: list[Request]) -> list[Request]:
        """Serves requests arriving at their `arrival` times (seconds from now, real time);
        returns them completed, with arrival/finish on the server clock."""
        t0 = self.clock()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        for r in pending:
            r.arrival += t0
        while pending or not self.idle():
            now = self.clock()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            self.pump()
            if not self.flights and pending:
                time.sleep(max(0.0, min(0.001, pending[0].arrival - self.clock())))
        return requests
