"""Pins of the oracle's MSB-first two-stage scan (Sec. 4.2, Eq. 4.2,
Lemma 2.1), CPU only.

* Without pruning (eps0 huge) the two-stage scan, which completes each full
  estimate from the reused most-significant-bit product (Eq. 4.2), returns
  the one-stage scan's ids and estimates bit for bit; orc_search computes
  <y_u, q_int> directly, so a wrong shift, mask or split fails here.
* The most significant bits are the 1-bit RaBitQ code (the B = 1 quantiser
  of the same residual), and the 1-bit estimate equals the one-stage scan of
  those codes with the B = 1 factors (f_rescale computed by the quantiser from
  <x, r'>, not from ||r'||_1).
* Lemma 2.1: the error of the 1-bit estimate, scaled by the bound's factor,
  behaves like a standard normal variable (the analysis behind the lemma):
  the bound fails on about 2(1 - Phi(eps0)) of the pairs, below
  exp(-eps0^2 / 2) (the lemma's form with c0 = 1/2) at every eps0 tested,
  and not trivially loose (about 32% at eps0 = 1).
* With eps0 = 4 no member of the one-stage top-kk is lost while most
  candidates are pruned; at eps0 = 1.9 every lost member has a lower bound
  above the one-stage kk-th estimate (only a bound failure drops it).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2409_09913_amd import synth


def _index(n, d, nl, nq, B, seed):
    x = synth.gmm(n, d, 32, 0.3, seed=seed, dp=d)
    q = synth.gmm(nq, d, 32, 0.3, seed=seed, stream=synth.S_QUERY, dp=d)
    P = synth.haar_orthogonal(d, seed=seed + 1)
    cent = x[:nl].astype(np.float64)
    assign = oracle.probe(x, cent.astype(np.float32), 1)[0][:, 0].astype(np.int32)
    codes, fa, fr, _, rr = oracle.encode(x, cent, assign, P.astype(np.float32), B)
    order = np.argsort(assign, kind="stable")
    off = np.zeros(nl + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(assign, minlength=nl))
    return dict(off=off, ids=order.astype(np.int64), codes=codes[order], fa=fa[order].astype(np.float32),
                fr=fr[order].astype(np.float32), l1=np.abs(rr[order]).sum(1), rr=rr[order],
                crot=oracle.rotate(cent, P).astype(np.float32), qrot=oracle.rotate(q, P).astype(np.float32),
                cent=cent.astype(np.float32), q=q, B=B)


@pytest.fixture(scope="module", params=[3, 4, 8])
def idx(request):
    return _index(20000, 128, 16, 40, request.param, seed=11)


def _probes(b, nprobe):
    return oracle.probe(b["q"], b["cent"], nprobe)[0].astype(np.int32)


def test_without_pruning_equals_one_stage(idx):
    b = idx
    probes = _probes(b, 6)
    oi, oe = oracle.search(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"], probes, b["B"],
                           50, est_mode=0)
    ti, te, nf = oracle.search_two_stage(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["l1"], b["crot"],
                                         b["qrot"], probes, b["B"], 50, 1e300)
    np.testing.assert_array_equal(ti, oi)
    np.testing.assert_array_equal(te, oe)
    # members equal to their centroid (r = 0) have an exact 1-bit estimate and may still be dropped
    tot = np.array([sum(b["off"][l + 1] - b["off"][l] for l in pr) for pr in probes])
    assert np.all(nf >= tot - len(b["cent"]))


def test_msb_stage_is_rabitq(idx):
    b = idx
    B = b["B"]
    c1, fa1, fr1, _ = oracle.quantize(b["rr"], 1, norm2=(b["rr"] ** 2).sum(1))
    msb = (b["codes"] >> (B - 1)).astype(np.uint8)
    np.testing.assert_array_equal(msb, c1)
    probes = _probes(b, 4)
    oi, oe = oracle.search(b["off"], b["ids"], c1, fa1.astype(np.float32), fr1.astype(np.float32), b["crot"],
                           b["qrot"], probes, 1, 200, est_mode=0)
    e1, _ = oracle.msb_bounds(b["off"], b["ids"], b["codes"], b["fa"], b["l1"], b["crot"], b["qrot"], probes, B,
                              oi, 2.0)
    ok = oi >= 0
    # the 1-bit factors of the quantiser are stored in FP32 here; the stage's from f_add and l1 in FP64
    np.testing.assert_allclose(e1[ok], oe[ok], rtol=1e-5, atol=1e-5 * np.abs(oe[ok]).max())


def test_lemma_bound_failure_rate():
    d, n, nq = 256, 20000, 50
    g = np.random.default_rng(5)
    x = g.standard_normal((n, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    q = g.standard_normal((nq, d))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    x, q = x.astype(np.float32), q.astype(np.float32)
    P = synth.haar_orthogonal(d, seed=7)
    codes, fa, _, _, rr = oracle.encode(x, np.zeros((1, d)), np.zeros(n, np.int32), P.astype(np.float32), 3)
    off, ids = np.array([0, n], np.int64), np.arange(n, dtype=np.int64)
    true = ((q.astype(np.float64)[:, None, :] - x.astype(np.float64)[None, :, :]) ** 2).sum(2)
    rates = {}
    for eps in (1.0, 1.5, 1.9, 2.5, 3.0, 4.0):
        e1, lb = oracle.msb_bounds(off, ids, codes, fa, np.abs(rr).sum(1), np.zeros((1, d), np.float32),
                                   oracle.rotate(q, P).astype(np.float32), np.zeros((nq, 1), np.int32), 3,
                                   np.tile(ids, (nq, 1)), eps)
        rates[eps] = float((np.abs(e1 - true) > (e1 - lb)).mean())
        assert rates[eps] <= math.exp(-eps * eps / 2), (eps, rates[eps])
        gauss = math.erfc(eps / math.sqrt(2))          # 2 (1 - Phi(eps))
        assert abs(rates[eps] - gauss) <= 0.25 * gauss + 2e-4, (eps, rates[eps], gauss)
    assert rates[1.0] > 0.25
    assert all(rates[a] > rates[b] for a, b in zip((1.0, 1.5, 1.9, 2.5, 3.0), (1.5, 1.9, 2.5, 3.0, 4.0)))


@pytest.mark.parametrize("eps0", [4.0, 1.9])
def test_pruning_keeps_the_neighbours(idx, eps0):
    b = idx
    kk = 20
    probes = _probes(b, 6)
    oi, oe = oracle.search(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"], probes, b["B"],
                           kk, est_mode=0)
    ti, te, nf = oracle.search_two_stage(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["l1"], b["crot"],
                                         b["qrot"], probes, b["B"], kk, eps0)
    tot = np.array([sum(b["off"][l + 1] - b["off"][l] for l in pr) for pr in probes])
    assert nf.sum() < 0.3 * tot.sum()
    _, lb = oracle.msb_bounds(b["off"], b["ids"], b["codes"], b["fa"], b["l1"], b["crot"], b["qrot"], probes,
                              b["B"], oi, eps0)
    for i in range(len(oi)):
        got = dict(zip(ti[i].tolist(), te[i].tolist()))
        for j, (v, e) in enumerate(zip(oi[i], oe[i])):
            if v in got:
                assert got[v] == e                       # the same full estimate
            else:
                assert eps0 < 4 and lb[i, j] > oe[i, -1], (i, v)
    if eps0 == 4.0:
        np.testing.assert_array_equal(ti, oi)
