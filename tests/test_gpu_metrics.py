"""Inner-product and cosine metrics on the device (the paper's conclusion:
the method adapts to both), against the oracle's inner-product scan.

* Scan parity: an imported index with the inner-product metric against
  oracle.search_ip (int8 query), per candidate at 1e-4 of the terms of the
  estimate (|<c', q'>| + |f_rescale / 2 <y_bar, q'>|).
* erq_search on a device-built inner-product index: estimates element by
  element against oracle.search_ip with the search's own rotated queries and
  probe lists (largest inner products with the centroids), and the exact
  re-rank against oracle.rerank_ip.
* Cosine: rows and queries normalised by the library; the re-ranked values
  are the exact negated cosines of the returned ids, and recall@10 against
  the exact cosine k-NN is high.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2409_09913_amd import erq, synth
from parity_util import CandTerms, both_paths, compare_topk

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("B,kk", [(1, 10), (4, 10), (4, 100), (8, 32)])
def test_ip_scan_parity(B, kk):
    say("ip scan B", B, "kk", kk)
    n, nl, dp, nq, nprobe = 8000, 16, 192, 50, 5
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=300 + B)
    qrot = synth.random_rotated(nq, dp, seed=301 + B)
    probes = synth.random_probes(nq, nl, nprobe, seed=302 + B)
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P), metric="ip")
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    gi, ge = both_paths(ix, lambda: [t.cpu().numpy() for t in ix.scan(dev(qrot), dev(probes), kk)])
    oi, oe = oracle.search_ip(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=0)
    compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B, metric="ip"))
    ix.close()


@pytest.fixture(scope="module")
def built_ip():
    n, d, nl, nq = 60000, 256, 64, 40
    x = synth.gmm(n, d, 32, 0.3, seed=310, stream=synth.S_BASE, dp=d)
    q = synth.gmm(nq, d, 32, 0.3, seed=310, stream=synth.S_QUERY, dp=d)
    P = synth.haar_orthogonal(d, seed=311).astype(np.float32)
    xd = dev(x)
    cent, _ = erq.kmeans(xd, nl, iters=4)
    ix = erq.Index(d, 4, nl, dev(P), metric="ip")
    ix.build(xd, cent, keep_raw=True)
    torch.cuda.synchronize()
    off, ids, codes, fa, fr, _ = [t.cpu().numpy() for t in ix.export()]
    cent_np = cent.cpu().numpy()
    qd = dev(q)
    yield dict(ix=ix, x=x, q=q, qd=qd, cent=cent_np, off=off, ids=ids, codes=codes, fa=fa, fr=fr,
               crot=oracle.rotate(cent_np, P).astype(np.float32),
               qrot=erq.rotate(qd, dev(P), precision=2).cpu().numpy())
    ix.close()


def test_ip_search_elementwise(built_ip):
    b = built_ip
    nprobe, k = 12, 20
    gi, ge = both_paths(b["ix"], lambda: [t.cpu().numpy() for t in b["ix"].search(b["qd"], nprobe, k, 0)])
    probes = erq.coarse_probe(b["qd"], dev(b["cent"]), nprobe, metric="ip").cpu().numpy()
    # the probe lists are the largest inner products with the centroids (up to near-ties)
    op, od = oracle.probe_ip(b["q"], b["cent"], nprobe)
    assert np.mean([set(a) == set(o) for a, o in zip(probes, op)]) > 0.9
    oi, oe = oracle.search_ip(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"], probes, 4, k,
                              est_mode=0)
    compare_topk(gi, ge, oi, oe, CandTerms(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"],
                                           probes, 4, metric="ip"))
    # exact re-rank of the same candidates
    ri, rd = b["ix"].search(b["qd"], nprobe, 10, k)
    ri, rd = ri.cpu().numpy(), rd.cpu().numpy()
    xi, xd_ = oracle.rerank_ip(b["x"], b["q"], gi, 10)
    np.testing.assert_allclose(rd, xd_, rtol=1e-5, atol=1e-5)
    assert (ri == xi).mean() > 0.99
    ti, _ = oracle.knn_ip(b["x"], b["q"], 10)
    rec = np.mean([len(set(a) & set(t)) / 10 for a, t in zip(ri, ti)])
    say("  ip recall@10 after re-rank", rec)
    assert rec > 0.8


def test_cosine_search():
    n, d, nl, nq = 40000, 128, 48, 40
    x = synth.spherical_clusters(n, d, 32, seed=320) * np.float32(3.0)      # not unit length
    q = synth.spherical_clusters(nq, d, 32, seed=320, stream=synth.S_QUERY) * np.float32(0.5)
    xd, qd = dev(x), dev(q)
    ix = erq.Index(d, 5, nl, None, seed=321, metric="cosine")
    ix.build(xd, None, keep_raw=True)
    ri, rd = ix.search(qd, 16, 10, 40)
    ri, rd = ri.cpu().numpy(), rd.cpu().numpy()
    xn = x.astype(np.float64) / np.linalg.norm(x.astype(np.float64), axis=1, keepdims=True)
    qn = q.astype(np.float64) / np.linalg.norm(q.astype(np.float64), axis=1, keepdims=True)
    for i in range(nq):
        np.testing.assert_allclose(rd[i], -(xn[ri[i]] @ qn[i]), rtol=1e-5, atol=1e-5)
    ti, _ = oracle.knn_ip(xn.astype(np.float32), qn.astype(np.float32), 10)
    rec = np.mean([len(set(a) & set(t)) / 10 for a, t in zip(ri, ti)])
    say("  cosine recall@10", rec)
    assert rec > 0.8
    ix.close()
