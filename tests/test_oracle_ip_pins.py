"""Pins of the oracle's inner-product metric (the paper's conclusion: the
method adapts to inner product and cosine), CPU only.

<o_r, q_r> = <c, q_r> + ||r|| <o, q'> with <o, q'> estimated by
<o_bar, q'>/<o_bar, o> (Lemma 2.1).  Pins: the estimate is exact when q' is a
multiple of the member's own rotated residual (the estimator is linear in q'
and exact on o itself); it is unbiased over random rotations; the int8
estimate stays within the int8 rounding bound of the float one; probe, k-NN
and re-rank equal numpy's largest inner products.
"""
import math

import numpy as np

import oracle
from paper_2409_09913_amd import synth


def _rows(g, n, dp):
    r = g.standard_normal((n, dp))
    return r


def test_ip_exact_along_the_residual():
    g = np.random.default_rng(31)
    for B in (1, 3, 4, 8):
        dp, nl, per = 64, 3, 40
        n = nl * per
        rr = _rows(g, n, dp)                                   # rotated residuals r'
        codes, fa, fr, co = oracle.quantize(rr, B, norm2=(rr * rr).sum(1))
        off = np.arange(0, n + 1, per, dtype=np.int64)
        ids = np.arange(n, dtype=np.int64)
        crot = g.standard_normal((nl, dp)).astype(np.float32)
        for v in (0, 55, 119):
            alpha = 0.7
            q = (alpha * rr[v]).astype(np.float32)[None, :]
            l = v // per
            probes = np.array([[l]], np.int32)
            # <o_r, q_r> = <c', q'> + <r', q'>, exact for q' along r'
            exact = float(crot[l].astype(np.float64) @ q[0].astype(np.float64)) + float(q[0].astype(np.float64) @ rr[v])
            for mode, kw in ((2, {}), (1, {"cos_oo": co})):
                oi, od = oracle.search_ip(off, ids, codes, fa.astype(np.float32), fr.astype(np.float32), crot, q,
                                          probes, B, per, est_mode=mode, **kw)
                got = -od[0][list(oi[0]).index(v)]
                assert abs(got - exact) <= 2e-6 * (abs(exact) + float(rr[v] @ rr[v])), (B, v, mode, got, exact)


def test_ip_unbiased_over_rotations():
    D, M, B = 64, 1500, 2
    g = np.random.default_rng(32)
    o_r = g.standard_normal(D)
    q_r = g.standard_normal(D) + 0.5 * o_r
    c = 0.3 * g.standard_normal(D)
    r = o_r - c
    ests = np.empty(M)
    for m in range(M):
        P = synth.haar_orthogonal(D, seed=7000 + m)
        rp = (r @ P)[None, :]
        codes, fa, fr, co = oracle.quantize(rp, B, norm2=np.array([r @ r]))
        q = (q_r @ P).astype(np.float32)[None, :]
        crot = (c @ P).astype(np.float32)[None, :]
        oi, od = oracle.search_ip(np.array([0, 1], np.int64), np.array([0], np.int64), codes, fa.astype(np.float32),
                                  fr.astype(np.float32), crot, q, np.array([[0]], np.int32), B, 1, est_mode=2)
        ests[m] = -od[0, 0]
    assert abs(ests.mean() - o_r @ q_r) < 4 * ests.std() / math.sqrt(M)


def test_ip_int8_within_rounding_bound():
    g = np.random.default_rng(33)
    B, dp, n, nl, nq = 4, 128, 3000, 12, 6
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=33)
    qrot = synth.random_rotated(nq, dp, seed=33)
    probes = synth.random_probes(nq, nl, 4, seed=33)
    Y = codes.astype(np.float64) - ((1 << B) - 1) / 2.0
    i2, d2 = oracle.search_ip(off, ids, codes, fa, fr, crot, qrot, probes, B, n, est_mode=2)
    i0, d0 = oracle.search_ip(off, ids, codes, fa, fr, crot, qrot, probes, B, n, est_mode=0)
    for q in range(nq):
        e2 = dict(zip(i2[q].tolist(), d2[q].tolist()))
        e0 = dict(zip(i0[q].tolist(), d0[q].tolist()))
        _, delta, _ = oracle.query_quant(qrot[q])
        pos = np.empty(n, np.int64)
        pos[ids] = np.arange(n)
        for i in list(e2)[:200]:
            if i < 0:
                continue
            p = pos[i]
            bound = 0.5 * abs(fr[p]) * delta / 2 * np.abs(Y[p]).sum()
            assert abs(e0[i] - e2[i]) <= bound * (1 + 1e-6) + 1e-9


def test_ip_probe_knn_rerank_match_numpy():
    g = np.random.default_rng(34)
    x = g.standard_normal((500, 64)).astype(np.float32)
    q = g.standard_normal((7, 64)).astype(np.float32)
    cent = x[:40]
    pr, pd = oracle.probe_ip(q, cent, 5)
    ip = q.astype(np.float64) @ cent.astype(np.float64).T
    np.testing.assert_array_equal(pr, np.argsort(-ip, axis=1, kind="stable")[:, :5])
    ki, kd = oracle.knn_ip(x, q, 10)
    ipx = q.astype(np.float64) @ x.astype(np.float64).T
    np.testing.assert_array_equal(ki, np.argsort(-ipx, axis=1, kind="stable")[:, :10])
    np.testing.assert_allclose(-kd, np.sort(ipx, axis=1)[:, ::-1][:, :10], rtol=1e-12)
    cand = np.argsort(-ipx, axis=1)[:, :30][:, ::-1].copy()
    cand[:, 0] = -1
    ri, rd = oracle.rerank_ip(x, q, cand, 10)
    np.testing.assert_array_equal(ri, ki)
