"""HIP-graph capture of the query path and continuous batching.

Results of a query do not depend on the batch it is computed in (every step
is per query, and the final top-k is ordered by (estimate, id)), so the
comparisons here are bit-exact: a graph replay against an eager call, and a
query served in a mixed batch against the same query searched alone.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2409_09913_amd import erq, serve, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def built():
    n, d, nl = 40000, 128, 64
    x = torch.from_numpy(synth.gmm(n, d, 16, 0.3, seed=21, stream=synth.S_BASE)).to(DEV)
    q = torch.from_numpy(synth.gmm(640, d, 16, 0.3, seed=21, stream=synth.S_QUERY)).to(DEV)
    P = torch.from_numpy(synth.haar_orthogonal(d, seed=22).astype(np.float32)).to(DEV)
    cent, assign = erq.kmeans(x, nl, iters=5)
    ix = erq.Index(d, 4, nl, P)
    ix.build(x, cent, assign, keep_raw=True)
    torch.cuda.synchronize()
    yield ix, q
    ix.close()


def _same(a_ids, a_d, b_ids, b_d, what):
    a_ids, b_ids = a_ids.cpu().numpy(), b_ids.cpu().numpy()
    a_d, b_d = a_d.cpu().numpy(), b_d.cpu().numpy()
    bad = np.nonzero((a_ids != b_ids).any(1) | (a_d.view(np.uint32) != b_d.view(np.uint32)).any(1))[0]
    assert bad.size == 0, f"{what}: rows {bad[:8]} differ"


@pytest.mark.parametrize("rerank_k", [0, 20])
def test_graph_replays_match_eager(built, rerank_k):
    ix, q = built
    say("graph replay rerank", rerank_k)
    nprobe, k = 16, 10
    g = serve.SearchGraph(ix, 256, nprobe, k, rerank_k)
    batches = [q[0:256], q[256:512], q[100:300], q[600:640], q[0:256]]
    for i, b in enumerate(batches):
        gi, gd = g.run(b)
        g.stream.synchronize()
        gi, gd = gi.clone(), gd.clone()
        # eager work of the program between replays, on its own stream
        ei, ed = ix.search(b.contiguous(), nprobe, k, rerank_k)
        other = ix.search(q[300:420].contiguous(), 32, k, rerank_k)
        torch.cuda.synchronize()
        _same(gi, gd, ei, ed, f"replay {i}")
        assert other[0].shape == (120, k)
    say("  5 replays identical to eager")


def test_server_alone_equals_mixed(built):
    ix, q = built
    say("server mixed batches")
    srv = serve.Server(ix, max_batch=192, max_nprobe=32, max_k=10, max_rerank=20, slots=3)
    assert srv.slots_admitted == 3
    g = np.random.default_rng(5)
    reqs, lo = [], 0
    for i in range(60):
        m = int(g.integers(1, 24))
        if lo + m > q.shape[0]:
            lo = 0
        k = int(g.choice([1, 5, 10]))
        rr = int(g.choice([0, 20]))
        reqs.append(serve.Request(i, q[lo:lo + m], k, int(g.choice([8, 16, 32])), rr))
        lo += m
    for r in reqs:
        srv.submit(r)
    srv.drain()
    torch.cuda.synchronize()
    say("  %d batches, %d with mixed (k, nprobe, rerank_k)" % (srv.batches, srv.mixed_batches))
    assert srv.mixed_batches > 0
    for r in reqs:
        assert r.ids is not None and r.ids.shape == (r.q.shape[0], r.k)
        for j in range(r.q.shape[0]):
            ai, ad = ix.search(r.q[j:j + 1].contiguous(), r.nprobe, r.k, r.rerank_k)
            _same(r.ids[j:j + 1], r.dist[j:j + 1], ai, ad, f"request {r.rid} query {j}")
    say("  %d queries identical alone and in the mix" % sum(r.q.shape[0] for r in reqs))


def test_server_admission_by_memory(built):
    """Batches take their workspace from a pool of the memory budget: with
    room for 2.5 full-size batches, at most 2 full-size batches are in flight
    at once, and every request still completes with its alone result."""
    ix, q = built
    per = ix.search_workspace_size(512, 64, 10, 20)
    srv = serve.Server(ix, max_batch=512, max_nprobe=64, max_k=10, max_rerank=20, slots=8,
                       mem_budget=int(2.5 * per))
    assert srv.slots_admitted == 2
    reqs = [serve.Request(i, q[(i * 97) % 128:(i * 97) % 128 + 512], 10, 64, 20) for i in range(6)]
    for r in reqs:
        srv.submit(r)
    peak = 0
    while srv.queue or any(s.busy for s in srv.slots):
        peak = max(peak, srv.step())
    torch.cuda.synchronize()
    assert peak <= 2
    for r in reqs[:2]:
        ai, ad = ix.search(r.q.contiguous(), r.nprobe, r.k, r.rerank_k)
        _same(r.ids, r.dist, ai, ad, f"request {r.rid}")
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, q[:4], 11, 16, 0))
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, q[:4], 10, 65, 0))
    with pytest.raises(ValueError):
        srv.submit(serve.Request(0, q[:513], 10, 16, 0))


def test_poisson_latency(built):
    ix, q = built
    say("poisson arrivals")
    srv = serve.Server(ix, max_batch=256, max_nprobe=64, max_k=10, max_rerank=20, slots=4)
    reqs, p50, p99, qps = serve.poisson_run(srv, q, rate=4000.0, n_requests=300, per_request=8, k=10,
                                            nprobes=(16, 64), rerank_k=20, seed=3)
    say("  p50 %.3f ms p99 %.3f ms, %.0f QPS" % (p50, p99, qps))
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert 0 < p50 <= p99
    for r in reqs[::37]:
        ai, ad = ix.search(r.q.contiguous(), r.nprobe, r.k, r.rerank_k)
        _same(r.ids, r.dist, ai, ad, f"request {r.rid}")
