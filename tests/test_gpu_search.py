"""The timed query path (erq_search) against the CPU oracle, element by
element, and the exactness of the integer products of the scan.

* The search's rotation (erq_rotate precision 2, the BF16 hi/lo three-product
  form) within its forward-error bound against the FP64 rotation.
* Integer products bit-exact: inputs chosen so that every FP32 operation of
  the estimator epilogue is exact (power-of-two delta and f_rescale, zero
  centroids, small integer query values), so each returned estimate equals
  the oracle's FP64 value bit for bit exactly when <y_u, q_int> is exact;
  kk covers every candidate, so every product of every query is checked.
  B = 1..8 at dp = 768 and B = 4, 8 at dp = 3072 (where |<y_u, q_int>| of
  full-range queries would exceed 2^24).
* erq_search on a device-built index (200,000 x 768, 256 lists, nprobe 16
  and 64): its estimates against oracle.search on the exported codes with the
  search's own int8 query decision (its rotated queries) and probe lists, per
  candidate at the tolerance of reading C-15, k = 10 and 100; its exact
  re-rank against oracle.rerank of the same candidates.
* Per-query nprobe / k / re-rank depth in one batch: every query's result is
  identical to the same query searched alone with its own values.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2409_09913_amd import erq, synth
from parity_util import CandTerms, compare_topk

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("dp,n", [(64, 37), (768, 300), (3072, 40)])
def test_rotate_search_precision_error_bound(dp, n):
    """Precision 2: each product off by at most 2^-16 |x_k P_kj| (split
    residuals and the dropped lo*lo term), plus FP32 accumulation of 3*dp
    terms."""
    say("rotate bf16x3", dp, n)
    P = synth.haar_orthogonal(dp, seed=dp + 1).astype(np.float32)
    x = synth.gmm(n, dp, 8, 0.3, seed=dp + 2, dp=dp)
    got = erq.rotate(dev(x), dev(P), precision=2).cpu().numpy().astype(np.float64)
    ref = oracle.rotate(x, P)
    mag = np.abs(x).astype(np.float64) @ np.abs(P).astype(np.float64)
    m = 3 * dp
    bound = (2.0 ** -15 + m * U32 / (1 - m * U32)) * mag
    assert np.all(np.abs(got - ref) <= bound)
    say("  max err / sum|x P|", float(np.max(np.abs(got - ref) / (mag + 1e-30))))


def _exact_case(dp, B, nl, nq, nprobe, seed):
    g = np.random.default_rng(seed)
    sizes = g.integers(40, 121, nl)
    n = int(sizes.sum())
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=seed, sizes=sizes)
    fa[:] = 0.0
    fr[:] = -0.125                                   # -2^-3
    crot[:] = 0.0
    # q' = q_int / 16: delta = 2^-4 exactly, one coordinate at +-127, the rest small
    qi = g.integers(-3, 4, (nq, dp))
    qi[np.arange(nq), g.integers(0, dp, nq)] = 127 * np.where(g.random(nq) < 0.5, -1, 1)
    qrot = (qi / 16.0).astype(np.float32)
    probes = synth.random_probes(nq, nl, nprobe, seed=seed + 1)
    return off, ids, codes, fa, fr, crot, qrot, probes


@pytest.mark.parametrize("dp,B", [(768, b) for b in range(1, 9)] + [(3072, 4), (3072, 8)])
def test_scan_int32_products_bit_exact(dp, B):
    say("int32 products bit-exact dp", dp, "B", B)
    nl, nq, nprobe, kk = 16, 48, 8, 1024
    off, ids, codes, fa, fr, crot, qrot, probes = _exact_case(dp, B, nl, nq, nprobe, seed=1000 * B + dp)
    P = synth.haar_orthogonal(dp, seed=3).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    gi, ge = ix.scan(dev(qrot), dev(probes), kk)
    torch.cuda.synchronize()
    gi, ge = gi.cpu().numpy(), ge.cpu().numpy()
    ix.close()
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=0)
    ncand = sum(int(off[l + 1] - off[l]) for l in probes.ravel())
    assert ncand == int((oi >= 0).sum()) and ncand <= nq * kk      # every candidate is returned
    np.testing.assert_array_equal(gi, oi)
    valid = oi >= 0
    # exact as values: FP32 of the GPU == FP64 of the oracle
    np.testing.assert_array_equal(ge[valid].astype(np.float64), oe[valid])
    say("  %d products exact" % ncand)


# ---------------------------------------------------------------------------
# erq_search on a device-built index
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def built768():
    n, d, nl, nq = 200_000, 768, 256, 48
    x = synth.gmm(n, d, 256, 0.3, zipf=True, lognormal_norm=0.2, seed=777, stream=synth.S_BASE)
    q = synth.gmm(nq, d, 256, 0.3, zipf=True, lognormal_norm=0.2, seed=777, stream=synth.S_QUERY)
    P = synth.haar_orthogonal(d, seed=778).astype(np.float32)
    xd = dev(x)
    cent, assign = erq.kmeans(xd, nl, iters=5)
    ix = erq.Index(d, 4, nl, dev(P))
    ix.build(xd, cent, assign, keep_raw=True)
    torch.cuda.synchronize()
    off, ids, codes, fa, fr, _ = [t.cpu().numpy() for t in ix.export()]
    cent_np = cent.cpu().numpy()
    crot = oracle.rotate(cent_np, P).astype(np.float32)        # the oracle's own rotated centroids
    qd = dev(q)
    qrot = erq.rotate(qd, dev(P), precision=2).cpu().numpy()   # the search's own rotation (int8 decision)
    yield dict(ix=ix, x=x, q=q, qd=qd, P=P, cent=cent_np, off=off, ids=ids, codes=codes, fa=fa, fr=fr,
               crot=crot, qrot=qrot)
    ix.close()


@pytest.mark.parametrize("nprobe", [16, 64])
def test_search_probe_lists_match_oracle(built768, nprobe):
    """The search's probe lists equal the FP64 nearest centroids, except
    where two centroid distances lie within the probe's error bound."""
    b = built768
    gp = erq.coarse_probe(b["qd"], dev(b["cent"]), nprobe).cpu().numpy()
    op, od = oracle.probe(b["q"], b["cent"], nprobe)
    q64, c64 = b["q"].astype(np.float64), b["cent"].astype(np.float64)
    d = q64.shape[1]
    cmax = float((c64 ** 2).sum(1).max())
    for i in range(len(gp)):
        if set(gp[i]) == set(op[i]):
            continue
        # error of ||q||^2 + ||c||^2 - 2 q.c: 2^-14 sum|q_i c_i| <= 2^-15 (||q||^2 + ||c||^2), plus the
        # FP32 sums; twice that between two distances
        tol = 2 * (2.0 ** -15 + 4 * d * U32) * (float(q64[i] @ q64[i]) + cmax)
        for j in set(gp[i]) ^ set(op[i]):
            dj = float(((q64[i] - c64[j]) ** 2).sum())
            assert abs(dj - od[i][-1]) <= tol, (i, j, dj, od[i][-1])


@pytest.mark.parametrize("nprobe,k", [(16, 10), (64, 10), (64, 100)])
def test_search_estimates_elementwise(built768, nprobe, k):
    b = built768
    say("search elementwise nprobe", nprobe, "k", k)
    gi, ge = b["ix"].search(b["qd"], nprobe, k, 0)
    gi, ge = gi.cpu().numpy(), ge.cpu().numpy()
    probes = erq.coarse_probe(b["qd"], dev(b["cent"]), nprobe).cpu().numpy()   # the search's probes
    oi, oe = oracle.search(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"], probes, 4, k,
                           est_mode=0)
    compare_topk(gi, ge, oi, oe, CandTerms(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"],
                                           probes, 4))
    same = np.mean([set(a) == set(o) for a, o in zip(gi, oi)])
    say("  identical id sets: %.3f of queries" % same)


def test_search_rerank_elementwise(built768):
    b = built768
    nprobe, k, rr = 64, 10, 20
    gi, gd = b["ix"].search(b["qd"], nprobe, k, rr)
    ci, _ = b["ix"].search(b["qd"], nprobe, rr, 0)             # the same scan's top-20 candidates
    gi, gd, ci = gi.cpu().numpy(), gd.cpu().numpy(), ci.cpu().numpy()
    oi, od = oracle.rerank(b["x"], b["q"], ci, k)
    np.testing.assert_allclose(gd, od, rtol=1e-5)
    x64, q64 = b["x"].astype(np.float64), b["q"].astype(np.float64)
    for i in range(len(gi)):
        if np.array_equal(gi[i], oi[i]):
            continue
        for j in set(gi[i].tolist()) ^ set(oi[i].tolist()):
            d = float(((x64[j] - q64[i]) ** 2).sum())
            assert abs(d - od[i][-1]) <= 1e-5 * od[i][-1], (i, j)


def test_search_per_query_parameters(built768):
    """One batch with per-query nprobe, k and re-rank depth: every query's
    row equals the same query searched alone with its own values."""
    b = built768
    ix, q = b["ix"], b["qd"]
    nq = q.shape[0]
    g = np.random.default_rng(11)
    npq = g.integers(1, 33, nq).astype(np.int32)
    kq = g.integers(1, 21, nq).astype(np.int32)
    rq = np.where(g.random(nq) < 0.5, 0, kq + g.integers(0, 21, nq)).astype(np.int32)
    ids, dist = ix.search(q, 32, 20, 40, nprobe_q=dev(npq), k_q=dev(kq), rerank_q=dev(rq))
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    for i in range(nq):
        ai, ad = ix.search(q[i:i + 1].contiguous(), int(npq[i]), int(kq[i]), int(rq[i]))
        ai, ad = ai.cpu().numpy()[0], ad.cpu().numpy()[0]
        np.testing.assert_array_equal(ids[i, :kq[i]], ai, err_msg=f"query {i}")
        np.testing.assert_array_equal(dist[i, :kq[i]].view(np.uint32), ad.view(np.uint32))
        assert (ids[i, kq[i]:] == -1).all() and np.isinf(dist[i, kq[i]:]).all()
    say("  %d queries identical alone and in the batch" % nq)


def test_import_rejects_ids_out_of_range():
    dp, nl, n = 64, 3, 50
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, 4, seed=5)
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, 4, nl, dev(P))
    bad = ids.copy()
    bad[7] = n                                    # a row number past the end
    with pytest.raises(erq.ErqError) as e:
        ix.import_(dev(off), dev(bad), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    assert e.value.code == erq.ERQ_EINVAL
    bad[7] = -3
    with pytest.raises(erq.ErqError):
        ix.import_(dev(off), dev(bad), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    assert ix.info()["n"] == n
    ix.close()
