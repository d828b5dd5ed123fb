"""Serving on one GPU: continuous batching of k-NN requests over an index
resident in HBM, and HIP-graph capture of the whole query path.

A request is a block of queries with its own k, nprobe and re-rank depth
(Sec. 2.1 asks for the K nearest neighbours of each query; Sec. 4.1 probes
nprobe lists).  The server keeps `slots` batches in flight, each on its own
stream with a workspace allocated once, sized for `max_batch` queries at the
largest (nprobe, k, rerank_k) the server accepts; the number of slots is
capped by a memory budget (admission by memory).  Whenever a slot is free,
the queued requests that share the (k, nprobe, rerank_k) of the oldest one are
packed into it, up to `max_batch` queries, and the batch is launched; batches
on different slots overlap on the device.  Results of a query do not depend
on the batch it rides in: every step of the path (rotation, probe, int8
query, scan, selection, re-rank) is computed per query.

Every step runs in the library's kernels (`erq.Index.search`); this module
only moves tensors and events.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import erq


class SearchGraph:
    """erq_search captured in a HIP graph for a fixed batch shape.

    `run(q)` copies up to `nq` queries into the static input (zero rows pad
    the rest), replays the graph on the capture stream and returns views of
    the first rows of the static outputs.  The graph holds only kernel
    launches of the library (it clears memory with its own fill kernels)."""

    def __init__(self, index: erq.Index, nq: int, nprobe: int, k: int, rerank_k: int = 0,
                 stream: torch.cuda.Stream | None = None):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.index, self.nq, self.nprobe, self.k, self.rerank_k = index, nq, nprobe, k, rerank_k
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.q = torch.zeros((nq, index.dp), dtype=torch.float32, device=dev)
        self.ws = torch.empty(index.search_workspace_size(nq, nprobe, k, rerank_k), dtype=torch.uint8, device=dev)
        self.ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        self.dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        with torch.cuda.stream(self.stream):
            # one eager run first: the library's one-time kernel attributes are set outside capture
            self.index.search(self.q, nprobe, k, rerank_k, ws=self.ws, out=(self.ids, self.dist))
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="thread_local"):
            self.index.search(self.q, nprobe, k, rerank_k, ws=self.ws, out=(self.ids, self.dist))
        self.stream.synchronize()

    def run(self, q: torch.Tensor):
        m = q.shape[0]
        if m > self.nq:
            raise ValueError("batch larger than the captured shape")
        with torch.cuda.stream(self.stream):
            self.q[:m].copy_(q, non_blocking=True)
            if m < self.nq:
                self.q[m:].zero_()
            self.graph.replay()
        return self.ids[:m], self.dist[:m]


@dataclass
class Request:
    rid: int
    q: torch.Tensor            # m x dp FP32 on the device
    k: int
    nprobe: int
    rerank_k: int = 0
    arrival: float = 0.0       # seconds, on the server's clock
    ids: torch.Tensor | None = None
    dist: torch.Tensor | None = None
    done: float | None = None

    @property
    def key(self):
        return (self.k, self.nprobe, self.rerank_k)


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    ws: torch.Tensor
    qbuf: torch.Tensor
    event: torch.cuda.Event = field(default_factory=torch.cuda.Event)
    reqs: list = field(default_factory=list)
    busy: bool = False


class Server:
    """Continuous batching over `slots` streams (see the module docstring)."""

    def __init__(self, index: erq.Index, max_batch: int = 1024, max_nprobe: int = 128, max_k: int = 32,
                 max_rerank: int = 32, slots: int = 4, mem_budget: int = 8 << 30):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.index, self.max_batch = index, max_batch
        self.limits = (max_k, max_nprobe, max_rerank)
        per_slot = index.search_workspace_size(max_batch, max_nprobe, max_k, max_rerank)
        per_slot += max_batch * (index.dp * 4 + max_k * 12)
        self.slots_admitted = int(max(1, min(slots, mem_budget // max(per_slot, 1))))
        self.slots = []
        for _ in range(self.slots_admitted):
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(device=dev),
                ws=torch.empty(index.search_workspace_size(max_batch, max_nprobe, max_k, max_rerank),
                               dtype=torch.uint8, device=dev),
                qbuf=torch.empty((max_batch, index.dp), dtype=torch.float32, device=dev)))
        self.queue: deque[Request] = deque()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        k, nprobe, rr = req.key
        if k > self.limits[0] or nprobe > self.limits[1] or rr > self.limits[2]:
            raise ValueError("request exceeds the server's limits (k, nprobe, rerank_k)")
        if req.q.shape[0] > self.max_batch:
            raise ValueError("request larger than max_batch")
        self.queue.append(req)

    def _launch(self, slot: _Slot):
        head = self.queue[0]
        key, batch, m = head.key, [], 0
        keep = deque()
        while self.queue:
            r = self.queue.popleft()
            if r.key == key and m + r.q.shape[0] <= self.max_batch:
                batch.append(r)
                m += r.q.shape[0]
            else:
                keep.append(r)
        self.queue = keep
        k, nprobe, rr = key
        # the queries were written on the submitter's stream
        slot.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(slot.stream):
            o = 0
            for r in batch:
                slot.qbuf[o:o + r.q.shape[0]].copy_(r.q, non_blocking=True)
                o += r.q.shape[0]
            # outputs come from torch's caching allocator (no device allocation
            # once warm); the workspace and query buffer are the slot's own
            out = (torch.empty((m, k), dtype=torch.int64, device=slot.ws.device),
                   torch.empty((m, k), dtype=torch.float32, device=slot.ws.device))
            self.index.search(slot.qbuf[:m], nprobe, k, rr, ws=slot.ws, out=out)
            slot.event.record(slot.stream)
        slot.reqs = [(r, out) for r in batch]
        slot.offsets = np.cumsum([0] + [r.q.shape[0] for r in batch])
        slot.busy = True

    def _retire(self, slot: _Slot):
        t = self.now()
        cur = torch.cuda.current_stream()
        for i, (r, out) in enumerate(slot.reqs):
            if i == 0 or out is not slot.reqs[i - 1][1]:
                out[0].record_stream(cur)
                out[1].record_stream(cur)
            a, b = slot.offsets[i], slot.offsets[i + 1]
            r.ids, r.dist, r.done = out[0][a:b], out[1][a:b], t
        slot.reqs, slot.busy = [], False

    def step(self) -> int:
        """Retires finished batches and launches queued work on free slots;
        returns the number of batches in flight."""
        for s in self.slots:
            if s.busy and s.event.query():
                self._retire(s)
        for s in self.slots:
            if not s.busy and self.queue:
                self._launch(s)
        return sum(s.busy for s in self.slots)

    def drain(self):
        while self.queue or any(s.busy for s in self.slots):
            if self.step() and not self.queue:
                time.sleep(0)


def poisson_run(server: Server, queries: torch.Tensor, rate: float, n_requests: int, per_request: int,
                k: int, nprobes, rerank_k: int = 0, seed: int = 0):
    """Requests of `per_request` queries arrive as a Poisson process of `rate`
    requests per second, each with an nprobe drawn from `nprobes`; returns the
    finished requests and (p50, p99) latency in ms and the sustained QPS."""
    g = np.random.default_rng(seed)
    gaps = g.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps)
    nq = queries.shape[0]
    reqs = []
    for i in range(n_requests):
        lo = (i * per_request) % max(nq - per_request, 1)
        reqs.append(Request(i, queries[lo:lo + per_request], k, int(g.choice(nprobes)), rerank_k,
                            arrival=float(arrivals[i])))
    torch.cuda.synchronize()
    server.t0 = time.perf_counter()
    i = 0
    while i < len(reqs) or server.queue or any(s.busy for s in server.slots):
        t = server.now()
        while i < len(reqs) and reqs[i].arrival <= t:
            server.submit(reqs[i])
            i += 1
        server.step()
    torch.cuda.synchronize()
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    span = max(r.done for r in reqs) - reqs[0].arrival
    return reqs, float(np.percentile(lat, 50)), float(np.percentile(lat, 99)), n_requests * per_request / span
