"""Serving on one GPU: continuous batching of k-NN requests over an index
resident in HBM, and HIP-graph capture of the whole query path.

A request is a block of queries with its own k, nprobe and re-rank depth
(Sec. 2.1 asks for the K nearest neighbours of each query; Sec. 4.1 probes
nprobe lists).  The server keeps up to `slots` batches in flight, each on its
own stream.  Admission is by memory: every batch takes its search workspace,
sized exactly for its query count and its largest (nprobe, k, rerank_k), from
one device pool of `mem_budget` bytes, and a batch is launched only when a
stream is free and the pool has room for it.  Whenever that holds, queued
requests are packed in arrival order, whatever their (k, nprobe, rerank_k),
while the batch stays within `max_batch` queries and its workspace fits the
pool's largest free block; each query carries its own values into the batch
(erq_search's per-query arrays).  Batches on different streams overlap on the
device.  Results of a query do not depend on the batch it rides in: every step
of the path (rotation, probe, int8 query, scan, selection, re-rank) is
computed per query, and the selection is the exact top-k by (estimate, id).

Every step runs in the library's kernels (`erq.Index.search`); this module
only moves tensors and events.
"""
from __future__ import annotations

import gc
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
                 stream: torch.cuda.Stream | None = None, per_query: bool = False):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.index, self.nq, self.nprobe, self.k, self.rerank_k = index, nq, nprobe, k, rerank_k
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.q = torch.zeros((nq, index.dp), dtype=torch.float32, device=dev)
        self.ws = torch.empty(index.search_workspace_size(nq, nprobe, k, rerank_k), dtype=torch.uint8, device=dev)
        self.ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
        self.dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        # per_query: static per-query (nprobe, k, rerank_k) rows the caller fills before a replay
        self.params = torch.stack([torch.full((nq,), v, dtype=torch.int32, device=dev)
                                   for v in (nprobe, k, rerank_k)]) if per_query else None
        pq = dict(nprobe_q=self.params[0], k_q=self.params[1], rerank_q=self.params[2]) if per_query else {}
        with torch.cuda.stream(self.stream):
            # one eager run first: the library's one-time kernel attributes are set outside capture
            self.index.search(self.q, nprobe, k, rerank_k, ws=self.ws, out=(self.ids, self.dist), **pq)
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="thread_local"):
            self.index.search(self.q, nprobe, k, rerank_k, ws=self.ws, out=(self.ids, self.dist), **pq)
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
    done: float | None = None
    _res: tuple | None = None  # (the batch's output tensors, first row, end row), set when the batch retires

    @property
    def key(self):
        return (self.k, self.nprobe, self.rerank_k)

    # the request's rows of its batch's outputs, sliced on access (the
    # serving loop does no tensor work per request when a batch retires)
    @property
    def ids(self) -> torch.Tensor | None:
        if self._res is None:
            return None
        out, a, b = self._res
        return out[0][a:b, :self.k]

    @property
    def dist(self) -> torch.Tensor | None:
        if self._res is None:
            return None
        out, a, b = self._res
        return out[1][a:b, :self.k]


class _Pool:
    """First-fit allocator of 256-byte aligned blocks inside one device buffer."""

    def __init__(self, nbytes: int, device):
        self.size = int(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]                 # (offset, bytes), sorted, coalesced

    def largest(self) -> int:
        return max((n for _, n in self.free), default=0)

    def alloc(self, nbytes: int):
        n = (int(nbytes) + 255) & ~255
        for i, (o, m) in enumerate(self.free):
            if m >= n:
                self.free[i:i + 1] = [(o + n, m - n)] if m > n else []
                return o, n
        return None

    def release(self, o: int, n: int):
        self.free.append((o, n))
        self.free.sort()
        out = []
        for fo, fn in self.free:
            if out and out[-1][0] + out[-1][1] == fo:
                out[-1] = (out[-1][0], out[-1][1] + fn)
            else:
                out.append((fo, fn))
        self.free = out


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    qbuf: torch.Tensor                     # max_batch x dp queries of the batch
    pdev: torch.Tensor                     # 3 x max_batch per-query (nprobe, k, rerank_k)
    phost: torch.Tensor                    # pinned staging of pdev
    event: torch.cuda.Event = field(default_factory=torch.cuda.Event)
    reqs: list = field(default_factory=list)
    block: tuple | None = None             # the batch's workspace in the pool
    busy: bool = False


class Server:
    """Continuous batching with admission by memory (see the module docstring)."""

    def __init__(self, index: erq.Index, max_batch: int = 1024, max_nprobe: int = 128, max_k: int = 32,
                 max_rerank: int = 32, slots: int = 4, mem_budget: int = 1 << 30):
        dev = torch.device("cuda", torch.cuda.current_device())
        self.index, self.max_batch = index, max_batch
        self.limits = (max_k, max_nprobe, max_rerank)
        free, _ = torch.cuda.mem_get_info(dev)
        self.pool = _Pool(min(int(mem_budget), int(free * 0.8)), dev)
        full = index.search_workspace_size(max_batch, max_nprobe, max_k, max_rerank)
        # streams that a pool of this size can keep busy with full-size batches (at least one)
        self.slots_admitted = int(max(1, min(slots, self.pool.size // max(full, 1))))
        self.slots = []
        for _ in range(max(1, slots)):
            self.slots.append(_Slot(
                stream=torch.cuda.Stream(device=dev),
                qbuf=torch.empty((max_batch, index.dp), dtype=torch.float32, device=dev),
                pdev=torch.empty((3, max_batch), dtype=torch.int32, device=dev),
                phost=torch.empty((3, max_batch), dtype=torch.int32).pin_memory()))
        self.queue: deque[Request] = deque()
        self._need_memo: dict = {}             # workspace bytes by (queries, nprobe, k, rerank_k)
        self.t0 = time.perf_counter()
        self.batches = 0
        self.mixed_batches = 0                 # batches whose requests differ in (k, nprobe, rerank_k)

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def _need(self, m: int, np_: int, k: int, rr: int) -> int:
        key = (m, np_, k, rr)
        n = self._need_memo.get(key)
        if n is None:
            if len(self._need_memo) > 65536:
                self._need_memo.clear()
            n = self._need_memo[key] = self.index.search_workspace_size(m, np_, k, rr)
        return n

    def submit(self, req: Request):
        k, nprobe, rr = req.key
        if k > self.limits[0] or nprobe > self.limits[1] or rr > self.limits[2]:
            raise ValueError("request exceeds the server's limits (k, nprobe, rerank_k)")
        if rr and rr < k:
            raise ValueError("a re-rank depth must be 0 or at least k")
        if req.q.shape[0] > self.max_batch:
            raise ValueError("request larger than max_batch")
        if self._need(req.q.shape[0], nprobe, k, rr) > self.pool.size:
            raise ValueError("request needs more workspace than the server's memory budget")
        self.queue.append(req)

    def _launch(self, slot: _Slot) -> bool:
        """Packs queued requests (arrival order, any keys) into one batch whose
        workspace fits the pool's largest free block; False if even the oldest
        request does not fit now."""
        room = self.pool.largest()
        batch, m, mx = [], 0, (0, 0, 0)
        keep = deque()
        while self.queue:
            r = self.queue.popleft()
            k, np_, rr = r.key
            nmx = (max(mx[0], np_), max(mx[1], k), max(mx[2], rr))
            if m + r.q.shape[0] <= self.max_batch and self._need(m + r.q.shape[0], *nmx) <= room:
                batch.append(r)
                m += r.q.shape[0]
                mx = nmx
            else:
                keep.append(r)
        self.queue = keep
        if not batch:
            return False
        nprobe, k, rr = mx
        block = self.pool.alloc(self._need(m, nprobe, k, rr))
        assert block is not None
        o, nb = block
        ph = slot.phost.numpy()
        row = 0
        for r in batch:
            c = r.q.shape[0]
            ph[0, row:row + c] = r.nprobe
            ph[1, row:row + c] = r.k
            ph[2, row:row + c] = r.rerank_k
            row += c
        # the queries were written on the submitter's stream
        slot.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(slot.stream):
            slot.pdev[:, :m].copy_(slot.phost[:, :m], non_blocking=True)
            # the batch's queries gathered by one copy launch
            if len(batch) == 1:
                slot.qbuf[:m].copy_(batch[0].q, non_blocking=True)
            else:
                torch.cat([r.q for r in batch], dim=0, out=slot.qbuf[:m])
            # outputs come from torch's caching allocator (no device allocation
            # once warm); the workspace is the batch's block of the pool
            out = (torch.empty((m, k), dtype=torch.int64, device=slot.qbuf.device),
                   torch.empty((m, k), dtype=torch.float32, device=slot.qbuf.device))
            pd = slot.pdev[:, :m]
            self.index.search(slot.qbuf[:m], nprobe, k, rr, ws=self.pool.buf[o:o + nb], out=out,
                              nprobe_q=pd[0], k_q=pd[1], rerank_q=pd[2])
            slot.event.record(slot.stream)
        slot.reqs = [(r, out) for r in batch]
        slot.offsets = np.cumsum([0] + [r.q.shape[0] for r in batch])
        slot.block = block
        slot.busy = True
        self.batches += 1
        self.mixed_batches += len(set(r.key for r in batch)) > 1
        return True

    def _retire(self, slot: _Slot):
        t = self.now()
        cur = torch.cuda.current_stream()
        for i, (r, out) in enumerate(slot.reqs):
            if i == 0:
                out[0].record_stream(cur)
                out[1].record_stream(cur)
            r._res, r.done = (out, int(slot.offsets[i]), int(slot.offsets[i + 1])), t
        self.pool.release(*slot.block)
        slot.reqs, slot.block, slot.busy = [], None, False

    def step(self) -> int:
        """Retires finished batches and launches queued work on free streams
        while the pool has room; returns the number of batches in flight."""
        for s in self.slots:
            if s.busy and s.event.query():
                self._retire(s)
        for s in self.slots:
            if not s.busy and self.queue:
                if not self._launch(s):
                    break
        return sum(s.busy for s in self.slots)

    def drain(self):
        while self.queue or any(s.busy for s in self.slots):
            if self.step() and not self.queue:
                time.sleep(0)


def poisson_run(server: Server, queries: torch.Tensor, rate: float, n_requests: int, per_request: int,
                k, nprobes, rerank_k=0, seed: int = 0):
    """Requests of `per_request` queries arrive as a Poisson process of `rate`
    requests per second, each with a k drawn from `k` (an int or a tuple) and
    an nprobe drawn from `nprobes` (a tuple, or a dict k -> nprobe); `rerank_k`
    is an int or a dict k -> re-rank depth.  Returns the finished requests, (p50, p99) latency in ms
    and the sustained QPS."""
    g = np.random.default_rng(seed)
    gaps = g.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps)
    nq = queries.shape[0]
    ks = (k,) if isinstance(k, int) else tuple(k)
    reqs = []
    for i in range(n_requests):
        lo = (i * per_request) % max(nq - per_request, 1)
        kr = int(g.choice(ks))
        rr = rerank_k.get(kr, 0) if isinstance(rerank_k, dict) else rerank_k
        npr = int(nprobes[kr]) if isinstance(nprobes, dict) else int(g.choice(nprobes))
        reqs.append(Request(i, queries[lo:lo + per_request], kr, npr, rr, arrival=float(arrivals[i])))
    torch.cuda.synchronize()
    # no cyclic garbage collection inside the timed loop: a full collection
    # over the live tensors and requests pauses the host for milliseconds
    gc_on = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        server.t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or server.queue or any(s.busy for s in server.slots):
            t = server.now()
            while i < len(reqs) and reqs[i].arrival <= t:
                server.submit(reqs[i])
                i += 1
            server.step()
        torch.cuda.synchronize()
    finally:
        if gc_on:
            gc.enable()
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    span = max(r.done for r in reqs) - reqs[0].arrival
    return reqs, float(np.percentile(lat, 50)), float(np.percentile(lat, 99)), n_requests * per_request / span
