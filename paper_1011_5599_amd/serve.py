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
- counts against the budget the device memory every context actually holds
  (`hanf_device_bytes`: buffers in use and those its pool keeps for reuse, rounded up to
  size classes), plus, for a group being admitted, its footprints with the size-class slack;
- keeps a finished batch's context (stream and device buffers) for the next batch, since
  freeing device memory would wait for every stream of the device; when a waiting request
  does not fit, idle contexts are destroyed (largest first) to make room;
- if a batch stops at its pass cap (HANF_EMAXITER), its requests still open are run alone
  through the plain path, whose cap is the graph's n + 1, so no request is lost.

Every request's results equal those of the same request run alone (the batch components
are independent runs).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import (HANF_BUSY, HANF_DONE, HANF_EMAXITER, HANF_ENOMEM, Batch, HanfError, HyperANF,
               hanf_batch_info, hanf_batch_read_nt, hanf_batch_read_registers, hanf_batch_stats_all,
               hanf_device_bytes, hanf_enqueue, hanf_footprint, hanf_poll)


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
    batch_id: int | None = None    # the batch it was admitted in (0, 1, ... in admission order)
    alone: bool = False            # finished by a plain run after its batch hit the pass cap
    error: str | None = None       # set if the request could not be served

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


def footprint_of(n: int, arcs: int, log2m: int) -> int:
    """Device bytes a graph of n nodes and `arcs` arcs needs inside a batch (its graph copy,
    expanded graph, run state, N_hat history; padding to 64 nodes included)."""
    n_pad = (n + 63) // 64 * 64
    return hanf_footprint(n_pad, arcs, log2m, 1) + 4 * (arcs + n + 1)


def footprint(req: Request) -> int:
    return footprint_of(req.n, len(req.col_idx), req.log2m)


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 96 << 30, max_batches: int = 4,
                 passes_per_poll: int = 4, keep_registers: bool = False, max_batch_requests: int = 64,
                 size_classes: bool = True, clock=time.perf_counter, alloc_slack: float = 1.5,
                 **options):
        self.device = device
        self.budget = hbm_budget
        # the library rounds allocations up to size classes 2^k and 1.5 * 2^k (at most 1.5x)
        self.alloc_slack = alloc_slack
        self.max_batches = max_batches
        # passes enqueued per batch between polls: 4 keeps batches running while the host
        # uploads another request's graph, at the cost of at most 3 passes after a batch's
        # fixpoint (they leave at once); measured on MI355X, 48 requests at 1x and 2x the
        # sequential capacity: median latency 5.5 and 10.7 ms with 4, 8.1 and 13.8 with 2
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
        self.done: list[Request] = []
        self.n_batches = 0
        self.max_flights = 0       # most batches in flight at once
        self.batch_sizes: list[int] = []
        self.idle_batches: list[Batch] = []
        self.host_s = {"admit": 0.0, "collect": 0.0, "poll": 0.0}

    # -- device memory
    @property
    def used(self) -> int:
        """Footprints of the batches in flight (what their requests were admitted with)."""
        return sum(fl.footprint for fl in self.flights)

    def held(self) -> int:
        """Device bytes every context of the server holds (in flight and idle)."""
        return sum(hanf_device_bytes(bt.ctx)[0] for bt in self._contexts())

    def _contexts(self):
        return [fl.batch for fl in self.flights] + list(self.idle_batches)

    def _room(self) -> int:
        return self.budget - max(self.held(), self.used)

    def _need(self, fp: int) -> int:
        return int(self.alloc_slack * fp)

    def _drop_idle(self, need: int) -> bool:
        """Destroys idle contexts, those holding most first, until `need` bytes fit; True if
        any was destroyed."""
        dropped = False
        self.idle_batches.sort(key=lambda bt: hanf_device_bytes(bt.ctx)[0])
        while self.idle_batches and self._room() < need:
            self.idle_batches.pop().close()
            dropped = True
        return dropped

    # -- admission
    def submit(self, req: Request) -> None:
        if self._need(footprint(req)) > self.budget:
            raise ValueError(f"request {req.rid} needs more than the HBM budget")
        self.waiting.append(req)

    def _admit(self, finished: list):
        t0 = self.clock()
        try:
            self._admit_groups(finished)
        finally:
            self.host_s["admit"] += self.clock() - t0

    def _admit_groups(self, finished: list):
        first_group = True
        while self.waiting and len(self.flights) < self.max_batches:
            if not first_group:  # the batches in flight get their next passes before the next upload
                finished += self._poll_all()
            first_group = False
            first = self.waiting[0]
            m = first.log2m
            key = self._class(first)
            if self._room() < self._need(footprint(first)) and not self._drop_idle(self._need(footprint(first))):
                return  # the oldest request does not fit yet: wait for memory
            group, room = [], self._room()
            for r in list(self.waiting):
                if r.log2m != m or len(group) >= self.max_batch_requests or self._class(r) != key:
                    continue
                need = self._need(footprint(r))
                if need > room:
                    if not group:
                        return
                    continue
                group.append(r)
                room -= need
            if not group:
                return
            for r in group:
                self.waiting.remove(r)
            fp = sum(footprint(r) for r in group)
            bt = self.idle_batches.pop() if self.idle_batches else Batch(self.device, **self.options)
            now = self.clock()
            try:
                bt.load_graphs([(r.row_ptr, r.col_idx) for r in group], 1)
                bt.init(m, [r.seed for r in group])
                hanf_enqueue(bt.ctx, self.passes_per_poll)
            except HanfError as e:
                bt.close()
                if e.code != HANF_ENOMEM:
                    raise
                # device memory ran out (other processes, fragmentation): free the idle
                # contexts and retry later; with nothing in flight to wait for, give up
                for r in reversed(group):
                    self.waiting.appendleft(r)
                for idle in self.idle_batches:
                    idle.close()
                self.idle_batches = []
                if not self.flights:
                    for r in group:
                        self.waiting.remove(r)
                        r.error, r.finish = str(e), self.clock()
                        self.done.append(r)
                return
            for r in group:
                r.admitted = now
                r.batch_id = self.n_batches
            self.n_batches += 1
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

    def _run_alone(self, fl: _Flight) -> list:
        """The batch reached its pass cap: its open requests run one by one through the plain
        path (pass cap n + 1), with the same results they would have had in the batch."""
        out = []
        with HyperANF(self.device) as h:
            for c in sorted(fl.open):
                r = fl.requests[c]
                h.load(r.row_ptr, r.col_idx).init(r.log2m, r.seed)
                r.nt = h.run()
                r.T = len(r.nt) - 1
                r.stats = h.stats()
                if self.keep_registers:
                    r.registers = h.registers().copy()
                r.alone = True
                r.finish = self.clock()
                out.append(r)
        fl.open.clear()
        return out

    def pump(self) -> list[Request]:
        """One round: poll every batch and keep the unfinished ones going, then admit what
        fits (polling again between admitted groups: uploading a large graph holds the host for
        milliseconds, and the batches in flight must not run dry meanwhile). Returns the
        requests completed in this round."""
        finished = self._poll_all()
        self._admit(finished)
        self.done += finished
        return finished

    def _poll_all(self) -> list[Request]:
        """Polls every batch in flight: collects its finished requests, retires it when it is
        done, else enqueues its next passes."""
        finished = []
        for fl in list(self.flights):
            t0 = self.clock()
            capped = False
            try:
                st, _ = hanf_poll(fl.batch.ctx)
            except HanfError as e:
                if e.code != HANF_EMAXITER:
                    raise
                st, capped = HANF_DONE, True
            t1 = self.clock()
            self.host_s["poll"] += t1 - t0
            if st == HANF_BUSY:
                continue
            finished += self._collect(fl, st == HANF_DONE and not capped)
            if capped:
                finished += self._run_alone(fl)
            self.host_s["collect"] += self.clock() - t1
            if st == HANF_DONE or not fl.open:
                self.idle_batches.append(fl.batch)
                self.flights.remove(fl)
            else:
                hanf_enqueue(fl.batch.ctx, self.passes_per_poll)
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
