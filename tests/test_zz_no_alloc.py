"""erq_search_static (the search on the library's static device scratch,
for callers that cannot allocate) against erq_search through the C ABI: two
calls in a row, the second with a smaller batch, each identical bit for bit
to erq_search with a workspace; a call that needs more than the scratch is
rejected before any device work."""
import sys

import numpy as np
import pytest
import torch

from paper_2409_09913_amd import erq, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b, what):
    ai, ad = a[0].cpu().numpy(), a[1].cpu().numpy()
    bi, bd = b[0].cpu().numpy(), b[1].cpu().numpy()
    np.testing.assert_array_equal(ai, bi, err_msg=what)
    np.testing.assert_array_equal(ad.view(np.uint32), bd.view(np.uint32), err_msg=what)


def test_search_static_matches_search():
    n, d, nl = 40000, 128, 64
    x = torch.from_numpy(synth.gmm(n, d, 16, 0.3, seed=61, stream=synth.S_BASE)).to(DEV)
    q = torch.from_numpy(synth.gmm(400, d, 16, 0.3, seed=61, stream=synth.S_QUERY)).to(DEV)
    P = torch.from_numpy(synth.haar_orthogonal(d, seed=62).astype(np.float32)).to(DEV)
    cent, assign = erq.kmeans(x, nl, iters=4)
    ix = erq.Index(d, 4, nl, P)
    ix.build(x, cent, assign, keep_raw=True)
    assert erq.static_scratch_bytes() == 64 << 20
    # call 1: 300 queries, re-rank; call 2: 37 queries with per-query values
    q1 = q[:300].contiguous()
    s1 = ix.search_static(q1, 16, 10, 20)
    r1 = ix.search(q1, 16, 10, 20)
    torch.cuda.synchronize()
    _same(s1, r1, "call 1")
    q2 = q[300:337].contiguous()
    g = np.random.default_rng(3)
    npq = torch.from_numpy(g.integers(1, 9, 37).astype(np.int32)).to(DEV)
    kq = torch.from_numpy(g.integers(1, 6, 37).astype(np.int32)).to(DEV)
    s2 = ix.search_static(q2, 8, 5, 0, nprobe_q=npq, k_q=kq)
    r2 = ix.search(q2, 8, 5, 0, nprobe_q=npq, k_q=kq)
    torch.cuda.synchronize()
    _same(s2, r2, "call 2")
    say("  two calls identical to erq_search")
    # a batch whose workspace exceeds the scratch is refused
    big = q.repeat(10, 1).contiguous()
    need = ix.search_workspace_size(big.shape[0], 16, 10, 0)
    assert need > erq.static_scratch_bytes()
    with pytest.raises(erq.ErqError) as e:
        ix.search_static(big, 16, 10, 0)
    assert e.value.code == erq.ERQ_ENOMEM
    ix.close()
