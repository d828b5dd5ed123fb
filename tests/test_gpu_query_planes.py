"""The int8 query in two planes (q' ~= delta (q_hi + q_lo / 254), B >= 5) on
the device against the oracle's two-plane scan (est_mode 3).

* Scan parity on imported random indexes, B = 5..8, dp 128 and 768, kk up to
  1024, per candidate at the tolerance of reading C-15; the pair-grouped
  pipeline and the small-batch path bit-identical.
* The exact fallback with two planes: lists of tied estimates too long for
  any bound, ids in the oracle's order.
* erq_search on a device-built B = 8 index element by element against the
  oracle with the search's own rotated queries and probe lists; its
  estimates sit far closer to the float-query estimates than one plane's.
* Save / load keeps the setting; refusals.
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


def _imported(n, nl, dp, B, seed, sizes=None):
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=seed, sizes=sizes)
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    ix.set_query_planes(2)
    return ix, (off, ids, codes, fa, fr, crot)


@pytest.mark.parametrize("B,dp,kk", [(5, 128, 10), (6, 128, 10), (7, 128, 10), (8, 128, 10), (8, 768, 10),
                                     (8, 256, 100), (6, 256, 1024), (8, 192, 1)])
def test_two_plane_scan_parity(B, dp, kk):
    say("two-plane scan B", B, "dp", dp, "kk", kk)
    nl, nq, nprobe = 20, 60, 5
    ix, (off, ids, codes, fa, fr, crot) = _imported(8000, nl, dp, B, seed=700 + B + dp + kk)
    qrot = synth.random_rotated(nq, dp, seed=701 + B)
    probes = synth.random_probes(nq, nl, nprobe, seed=702 + B)
    probes[:5, nprobe // 2:] = -1                         # some queries probe fewer lists
    gi, ge = both_paths(ix, lambda: [t.cpu().numpy() for t in ix.scan(dev(qrot), dev(probes), kk)])
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=3)
    compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    ix.close()


@pytest.mark.parametrize("kk", [16, 100])
def test_two_plane_exact_fallback_ties(kk):
    """All members of a list tie exactly; lists of 9000 and 5000 members keep
    more than 4096 candidates at or below every bound, so the exact fallback
    (with both planes) produces the result."""
    say("two-plane fallback kk", kk)
    dp, B, nl = 64, 8, 3
    sizes = np.array((9000, 5000, 40))
    off, ids, codes, fa, fr, crot = synth.random_index(int(sizes.sum()), nl, dp, B, seed=60 + kk, sizes=sizes)
    for l in range(nl):
        lo, hi = off[l], off[l + 1]
        codes[lo:hi] = codes[lo]
        fa[lo:hi] = fa[lo]
        fr[lo:hi] = fr[lo]
    qrot = synth.random_rotated(12, dp, seed=61)
    probes = np.tile(np.arange(nl, dtype=np.int32), (12, 1))
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    ix.set_query_planes(2)
    ix.set_small_batch(0)                                  # the pair-grouped pipeline and its fallback
    erq.profile_enable(2)
    erq.profile_read("scan_redo_pairs", reset=True)
    try:
        gi, ge = ix.scan(dev(qrot), dev(probes), kk)
        torch.cuda.synchronize()
        redo, _ = erq.profile_read("scan_redo_pairs", reset=True)
    finally:
        erq.profile_read("scan", reset=True)
        erq.profile_enable(False)
    gi, ge = gi.cpu().numpy(), ge.cpu().numpy()
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=3)
    np.testing.assert_array_equal(gi, oi)
    compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    assert redo > 0
    say("  pairs rescanned by the exact fallback", redo)
    ix.close()


@pytest.fixture(scope="module")
def built8():
    n, d, nl, nq = 60000, 256, 48, 64
    x = synth.gmm(n, d, 64, 0.3, seed=810, dp=d)
    q = synth.gmm(nq, d, 64, 0.3, seed=810, stream=synth.S_QUERY, dp=d)
    P = synth.haar_orthogonal(d, seed=811).astype(np.float32)
    cent = x[:nl].copy()
    assign = oracle.probe(x, cent, 1)[0][:, 0].astype(np.int32)
    ix = erq.Index(d, 8, nl, dev(P))
    ix.build(dev(x), dev(cent), dev(assign), precision=0, keep_raw=True)
    torch.cuda.synchronize()
    off, ids, codes, fa, fr, _ = [t.cpu().numpy() for t in ix.export()]
    crot = oracle.rotate(cent, P).astype(np.float32)
    qd = dev(q)
    qrot = erq.rotate(qd, dev(P), precision=2).cpu().numpy()   # the search's own rotation
    yield dict(ix=ix, q=q, qd=qd, P=P, cent=cent, off=off, ids=ids, codes=codes, fa=fa, fr=fr, crot=crot, qrot=qrot)
    ix.close()


@pytest.mark.parametrize("nprobe,k", [(6, 10), (16, 100)])
def test_two_plane_search_elementwise(built8, nprobe, k):
    b = built8
    ix = b["ix"]
    ix.set_query_planes(2)
    gi, ge = both_paths(ix, lambda: [t.cpu().numpy() for t in ix.search(b["qd"], nprobe, k, 0)])
    probes = erq.coarse_probe(b["qd"], dev(b["cent"]), nprobe).cpu().numpy()
    args = (b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], b["qrot"], probes, 8)
    oi, oe = oracle.search(*args, k, est_mode=3)
    compare_topk(gi, ge, oi, oe, CandTerms(*args))
    # estimates of the returned candidates against the float-query estimator, one plane and two
    fi, fe = oracle.search(*args, 4000, est_mode=2)
    ix.set_query_planes(1)
    hi_, he = ix.search(b["qd"], nprobe, k, 0)
    hi_, he = hi_.cpu().numpy(), he.cpu().numpy()
    d1, d2 = [], []
    for i in range(len(gi)):
        ref = dict(zip(fi[i].tolist(), fe[i].tolist()))
        d2 += [abs(e - ref[v]) for v, e in zip(gi[i].tolist(), ge[i].tolist()) if v in ref]
        d1 += [abs(e - ref[v]) for v, e in zip(hi_[i].tolist(), he[i].tolist()) if v in ref]
    say("  mean |estimate - float-query estimate|: one plane %.3g, two planes %.3g" % (np.mean(d1), np.mean(d2)))
    assert np.mean(d2) < 0.05 * np.mean(d1)


def test_two_plane_save_load_and_refusals(built8, tmp_path):
    b = built8
    b["ix"].set_query_planes(2)
    path = str(tmp_path / "planes.erq")
    b["ix"].save(path)
    iy = erq.Index.load_file(path)
    a = b["ix"].search(b["qd"], 8, 10, 20)
    c = iy.search(b["qd"], 8, 10, 20)
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and torch.equal(a[1].view(torch.int32), c[1].view(torch.int32))
    iy.close()
    for bits in (1, 4):
        ix = erq.Index(128, bits, 4, None, seed=1)
        with pytest.raises(erq.ErqError) as e:
            ix.set_query_planes(2)
        assert e.value.code == erq.ERQ_EUNSUPPORTED
        ix.close()
    ix = erq.Index(128, 8, 4, None, seed=1)
    with pytest.raises(erq.ErqError) as e:
        ix.set_query_planes(3)
    assert e.value.code == erq.ERQ_EINVAL
    ix.set_two_stage(2.0)
    with pytest.raises(erq.ErqError) as e:
        ix.set_query_planes(2)
    assert e.value.code == erq.ERQ_EUNSUPPORTED
    ix.set_two_stage(0.0)
    ix.set_query_planes(2)
    with pytest.raises(erq.ErqError) as e:
        ix.set_two_stage(2.0)
    assert e.value.code == erq.ERQ_EUNSUPPORTED
    ix.close()
