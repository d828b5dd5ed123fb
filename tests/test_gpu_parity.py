"""GPU parity of every stage of the hot path against the CPU oracle, called
through the C ABI on identical seeded inputs.

Bars: codes, ids and integer products bit-exact; FP32 distances within
1e-4 relative to the magnitude of the terms that form them (a difference of
large terms can be close to 0 or negative); rotations within the forward
error bound of an FP32 (or BF16-input) dot product of length dp.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2409_09913_amd import erq, synth
from parity_util import CandTerms, both_paths, compare_topk as _compare_topk

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


# ---------------------------------------------------------------------------
# rotation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dp,n", [(64, 33), (128, 300), (768, 517), (1536, 130)])
def test_rotate_fp32_error_bound(dp, n):
    say("rotate fp32", dp, n)
    P = synth.haar_orthogonal(dp, seed=dp).astype(np.float32)
    x = synth.gmm(n, dp, 8, 0.3, seed=dp, dp=dp)
    got = erq.rotate(dev(x), dev(P)).cpu().numpy().astype(np.float64)
    ref = oracle.rotate(x, P)
    mag = np.abs(x).astype(np.float64) @ np.abs(P).astype(np.float64)
    gam = dp * U32 / (1 - dp * U32)
    assert np.all(np.abs(got - ref) <= gam * mag + 1e-30)
    say("  max rel err", float(np.max(np.abs(got - ref) / (mag + 1e-30))))


def test_rotate_bf16_error_bound():
    dp, n = 768, 257
    P = synth.haar_orthogonal(dp, seed=3).astype(np.float32)
    x = synth.gmm(n, dp, 8, 0.3, seed=4, dp=dp)
    got = erq.rotate(dev(x), dev(P), precision=1).cpu().numpy().astype(np.float64)
    ref = oracle.rotate(x, P)
    mag = np.abs(x).astype(np.float64) @ np.abs(P).astype(np.float64)
    # inputs rounded to BF16 (rel. 2^-9 each), products exact, FP32 accumulation
    bound = (2 * 2.0 ** -9 + 2.0 ** -18) * mag + (dp * U32 / (1 - dp * U32)) * mag * (1 + 2.0 ** -7)
    assert np.all(np.abs(got - ref) <= bound)
    rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say("  bf16 mean row rel err", float(rel.mean()))


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------
def _quantize_compare(r, B, norm2=None):
    codes, fa, fr, co = erq.quantize(dev(r), B, None if norm2 is None else dev(norm2.astype(np.float32)))
    torch.cuda.synchronize()
    codes = codes.cpu().numpy()
    rc, rfa, rfr, rco = oracle.quantize(r.astype(np.float64), B,
                                        None if norm2 is None else norm2.astype(np.float32).astype(np.float64))
    bad = np.nonzero((codes != rc).any(1))[0]
    assert bad.size == 0, f"B={B}: {bad.size} rows differ, first {bad[:5]}"
    np.testing.assert_allclose(fa.cpu().numpy(), rfa.astype(np.float32), rtol=2e-7, atol=0)
    np.testing.assert_allclose(fr.cpu().numpy(), rfr.astype(np.float32), rtol=4e-7, atol=0)
    np.testing.assert_allclose(co.cpu().numpy(), rco.astype(np.float32), rtol=4e-7, atol=0)


@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 6, 7, 8])
def test_quantize_bitexact_dp128(B):
    say("quantize dp128 B", B)
    r = synth.random_rotated(200, 128, seed=B)
    _quantize_compare(r, B)


@pytest.mark.parametrize("dp,B,n", [(64, 4, 100), (768, 4, 300), (768, 8, 40), (960, 3, 64), (960, 7, 16),
                                    (1536, 5, 24), (3072, 4, 12), (3072, 2, 8)])
def test_quantize_bitexact_sizes(dp, B, n):
    say("quantize", dp, B, n)
    g = np.random.default_rng(dp + B)
    r = synth.random_rotated(n, dp, seed=dp * 10 + B)
    norm2 = (r.astype(np.float64) ** 2).sum(1) * g.uniform(0.5, 2.0, n)
    _quantize_compare(r, B, norm2)


@pytest.mark.parametrize("B", [1, 2, 4, 8])
def test_quantize_edge_rows(B):
    say("quantize edge rows B", B)
    for dp in (64, 192):
        r = synth.edge_rows(dp, seed=B)
        _quantize_compare(r, B)


def test_quantize_anisotropic_and_ties():
    """Rows built to create long runs of exactly tied critical values."""
    g = np.random.default_rng(5)
    rows = []
    for _ in range(20):
        v = (2.0 ** g.integers(-4, 4, 256)) * np.where(g.random(256) < 0.5, -1, 1)
        rows.append(v)
    for _ in range(10):
        rows.append(g.integers(-3, 4, 256).astype(np.float64))
    r = np.asarray(rows, np.float32)
    for B in (3, 5, 8):
        _quantize_compare(r, B)


# ---------------------------------------------------------------------------
# packing round trip
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 6, 7, 8])
def test_pack_roundtrip(B):
    dp, n, nl = 192, 1000, 9
    sizes = np.array([0, 1, 31, 32, 33, 100, 203, 300, 300])
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=B, sizes=sizes)
    P = synth.haar_orthogonal(dp, seed=1).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    cent = np.zeros((nl, dp), np.float32)
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(cent), dev(crot))
    o2, i2, c2, fa2, fr2, cr2 = [t.cpu().numpy() for t in ix.export()]
    np.testing.assert_array_equal(o2, off)
    np.testing.assert_array_equal(i2, ids)
    np.testing.assert_array_equal(c2, codes)
    np.testing.assert_array_equal(fa2, fa)
    np.testing.assert_array_equal(fr2, fr)
    assert ix.info()["code_bytes"] == 4 * dp * B * sum((s + 31) // 32 for s in sizes)
    ix.close()


# ---------------------------------------------------------------------------
# scan (int8 matrix cores + estimator + top-k)
# ---------------------------------------------------------------------------
def _scan_case(n, nl, dp, B, nq, nprobe, kk, seed, sizes=None, empty_lists=0, pad_probes=0, q_at_centroid=0):
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, B, seed=seed, sizes=sizes,
                                                       empty_lists=empty_lists)
    qrot = synth.random_rotated(nq, dp, seed=seed + 7)
    probes = synth.random_probes(nq, nl, nprobe, seed=seed)
    for i in range(pad_probes):
        probes[i, nprobe // 2:] = -1
    for i in range(q_at_centroid):
        qrot[nq - 1 - i] = crot[probes[nq - 1 - i, 0]]
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    # the pipeline and (up to 1024 queries) the small-batch path, bit-identical
    run = lambda: [t.cpu().numpy() for t in ix.scan(dev(qrot), dev(probes), kk)]
    gi, ge = both_paths(ix, run) if nq <= 1024 else run()
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=0)
    _compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    ix.close()
    return gi, oi


@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 6, 7, 8])
def test_scan_parity_bits(B):
    say("scan B", B)
    _scan_case(n=6000, nl=24, dp=128, B=B, nq=70, nprobe=6, kk=10, seed=B)


@pytest.mark.parametrize("kk", [1, 10, 16, 17, 32, 33, 64, 100, 257, 1000, 1024])
def test_scan_parity_kk(kk):
    say("scan kk", kk)
    _scan_case(n=8000, nl=16, dp=192, B=4, nq=50, nprobe=5, kk=kk, seed=100 + kk)


@pytest.mark.parametrize("kk", [0, 1025])
def test_scan_rejects_kk_out_of_range(kk):
    """kk outside [1, 1024] fails before any launch."""
    say("scan kk rejected", kk)
    dp, nl, n = 128, 4, 200
    off, ids, codes, fa, fr, crot = synth.random_index(n, nl, dp, 4, seed=1)
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, 4, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    with pytest.raises(erq.ErqError) as e:
        ix.scan(dev(synth.random_rotated(3, dp, seed=3)), dev(synth.random_probes(3, nl, 2, seed=4)), kk)
    assert e.value.code in (erq.ERQ_EUNSUPPORTED, erq.ERQ_EINVAL)
    ix.close()


def test_scan_parity_dp768_many_tiles():
    say("scan dp768")
    sizes = np.array([1, 2, 31, 32, 33, 64, 65, 500, 1000, 1500, 2000, 3000, 1871, 0, 17, 384])
    _scan_case(n=int(sizes.sum()), nl=len(sizes), dp=768, B=4, nq=120, nprobe=8, kk=20, seed=7, sizes=sizes)


def test_scan_edge_cases():
    """Empty lists, padded probe rows (-1), queries equal to a centroid
    (s' = 0, delta = 0), kk larger than the candidate count."""
    say("scan edges")
    _scan_case(n=3000, nl=32, dp=128, B=5, nq=40, nprobe=4, kk=10, seed=11, empty_lists=6,
               pad_probes=5, q_at_centroid=3)
    sizes = np.array([3, 0, 2, 1])
    gi, oi = _scan_case(n=6, nl=4, dp=64, B=8, nq=5, nprobe=2, kk=16, seed=12, sizes=sizes)
    assert (gi == -1).any()


@pytest.mark.parametrize("small", [False, True], ids=["pipeline", "small-batch"])
@pytest.mark.parametrize("kk,sizes", [(16, (300, 500, 40)), (32, (300, 500, 40)), (100, (300, 500, 40)),
                                      (10, (9000, 5000, 40)), (32, (9000, 5000, 40)), (100, (9000, 5000, 40)),
                                      (1000, (9000, 5000, 40))])
def test_scan_exact_ties_by_id(kk, sizes, small):
    """Every member of a list is a copy of one code row with the same factors,
    so all its estimates tie exactly (in FP32 and FP64): the top-kk must take
    the smallest ids of a tied group, in id order (reading C-16).  With lists
    of 9000 and 5000 tied members no bound can shrink a query's candidates
    below its buffer's 4096 entries, so the exact fallback runs (its pair
    count is read back).  The small-batch path (12 queries) must give the
    same ids."""
    say("scan exact ties kk", kk, "sizes", sizes, "small", small)
    dp, B, nl = 64, 4, 3
    sizes = np.array(sizes)
    off, ids, codes, fa, fr, crot = synth.random_index(int(sizes.sum()), nl, dp, B, seed=40 + kk, sizes=sizes)
    for l in range(nl):
        lo, hi = off[l], off[l + 1]
        codes[lo:hi] = codes[lo]
        fa[lo:hi] = fa[lo]
        fr[lo:hi] = fr[lo]
    qrot = synth.random_rotated(12, dp, seed=41)
    probes = np.tile(np.arange(nl, dtype=np.int32), (12, 1))
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    ix.set_small_batch(32 if small else 0)
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
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=0)
    np.testing.assert_array_equal(gi, oi)
    _compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    say("  pairs rescanned by the exact fallback", redo)
    # the fallback must have run when some query has more than 4096
    # candidates at or below its kk-th estimate (a tied group no bound splits)
    _, all_e = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, int(sizes.sum()), est_mode=0)
    if not small and any((all_e[i] <= oe[i][min(kk, int(sizes.sum())) - 1]).sum() > 4096 for i in range(len(qrot))):
        assert redo > 0
    ix.close()


@pytest.mark.parametrize("small", [False, True], ids=["pipeline", "small-batch"])
@pytest.mark.parametrize("kk", [1, 7, 22, 64])
def test_scan_small_tie_groups(kk, small):
    """Members come in groups of three copies of one code row with the same
    factors, so estimates tie in threes and the kk-th often falls inside a
    group: the top-kk must take its smallest ids (reading C-16).  Buffers
    stay under 1024 entries and kk <= 64, the case the select ranks with
    one sort across the wave."""
    say("scan small tie groups kk", kk, "small", small)
    dp, B, nl = 128, 4, 3
    sizes = np.array([300, 240, 180])
    off, ids, codes, fa, fr, crot = synth.random_index(int(sizes.sum()), nl, dp, B, seed=90 + kk, sizes=sizes)
    for l in range(nl):
        for lo in range(off[l], off[l + 1], 3):
            hi = min(lo + 3, off[l + 1])
            codes[lo:hi] = codes[lo]
            fa[lo:hi] = fa[lo]
            fr[lo:hi] = fr[lo]
    qrot = synth.random_rotated(20, dp, seed=91)
    probes = np.tile(np.arange(nl, dtype=np.int32), (20, 1))
    P = synth.haar_orthogonal(dp, seed=3).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    ix.set_small_batch(32 if small else 0)
    gi, ge = ix.scan(dev(qrot), dev(probes), kk)
    gi, ge = gi.cpu().numpy(), ge.cpu().numpy()
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=0)
    np.testing.assert_array_equal(gi, oi)
    _compare_topk(gi, ge, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    ix.close()


def test_scan_many_queries_per_list():
    """More than 32 queries per list (several query tiles per list)."""
    say("scan many queries")
    _scan_case(n=4000, nl=8, dp=256, B=3, nq=300, nprobe=4, kk=10, seed=13)


# ---------------------------------------------------------------------------
# coarse probe, rerank
# ---------------------------------------------------------------------------
def test_scan_long_lists_buffer_overflow():
    # lists of 20000 members are split into chunks of 2048 members per work
    # item; with kk = 32 the first bound (from 8 x 128 members) lets about
    # 10k candidates per query through, more than a query's buffer holds, so
    # the overflowing round is rescanned with the tighter bound
    say("scan long lists + overflow")
    sizes = np.full(16, 20000, np.int64)
    _scan_case(n=int(sizes.sum()), nl=16, dp=64, B=4, nq=70, nprobe=16, kk=32, seed=77, sizes=sizes)


def test_scan_one_huge_list():
    # one list far longer than the rest (a skewed k-means partition)
    say("scan huge list")
    sizes = np.array([37696] + [300] * 23, np.int64)
    _scan_case(n=int(sizes.sum()), nl=24, dp=128, B=4, nq=90, nprobe=3, kk=10, seed=78, sizes=sizes)


def test_coarse_probe_parity():
    say("probe")
    dp, nl, nq, nprobe = 256, 300, 200, 17
    cent = synth.gmm(nl, 200, 30, 0.5, seed=21, dp=dp)
    q = synth.gmm(nq, 200, 30, 0.5, seed=21, stream=synth.S_QUERY, dp=dp)
    pg, dg = erq.coarse_probe(dev(q), dev(cent), nprobe, with_dist=True)
    pg, dg = pg.cpu().numpy(), dg.cpu().numpy()
    po, do = oracle.probe(q, cent, nprobe)
    # FP32 error bound of ||q||^2 + ||c||^2 - 2 q.c
    qn = (q.astype(np.float64) ** 2).sum(1)
    cn = (cent.astype(np.float64) ** 2).sum(1)
    for i in range(nq):
        tol = 4 * dp * U32 * (qn[i] + cn.max()) + 1e-12
        assert np.all(np.abs(dg[i] - do[i]) <= tol)
        if set(pg[i]) != set(po[i]):
            kth = do[i][-1]
            for j in set(pg[i]) ^ set(po[i]):
                dd = ((q[i].astype(np.float64) - cent[j].astype(np.float64)) ** 2).sum()
                assert abs(dd - kth) <= 2 * tol
        else:
            np.testing.assert_array_equal(np.sort(pg[i]), np.sort(po[i]))


@pytest.mark.parametrize("nl,nprobe", [(1, 1), (63, 7), (64, 64), (65, 10), (300, 17), (1000, 88), (1024, 256),
                                       (1025, 100), (2048, 1), (3000, 128), (4096, 88), (4096, 256), (4096, 300),
                                       (5000, 96), (9000, 40)])
def test_probe_selection_exact_ties(nl, nprobe):
    """The nprobe nearest centroids, ascending by (distance, column), where the
    distances are small integers (exact in FP32 and in the BF16 planes) with
    many ties, so the rows decide ties among equal distances by column.
    Covers each register-tile width of the selection kernel (rows of up to
    1024, 2048, 4096 and 8192 entries, and longer rows read from memory) and
    ragged row lengths."""
    say("probe ties", nl, nprobe)
    g = np.random.default_rng(nl * 7 + nprobe)
    dp, nq = 64, 37
    cent = np.zeros((nl, dp), np.float32)
    cent[:, :6] = g.integers(-2, 3, (nl, 6))
    q = np.zeros((nq, dp), np.float32)
    q[:, :6] = g.integers(-2, 3, (nq, 6))
    q[0] = 0.0
    pg, dg = erq.coarse_probe(dev(q), dev(cent), nprobe, with_dist=True)
    pg, dg = pg.cpu().numpy(), dg.cpu().numpy()
    exact = ((q[:, None, :6].astype(np.int64) - cent[None, :, :6].astype(np.int64)) ** 2).sum(-1)
    cols = np.arange(nl)
    for i in range(nq):
        order = np.lexsort((cols, exact[i]))[:nprobe]
        np.testing.assert_array_equal(pg[i], order)
        np.testing.assert_array_equal(dg[i], exact[i][order].astype(np.float32))


@pytest.mark.parametrize("nl,nprobe", [(700, 84), (5000, 200), (9000, 40)])
def test_probe_selection_all_equal(nl, nprobe):
    """Every centroid is the same vector, so every distance of a row is the
    same value (no radix pass has anything to split): the selection must
    return the first nprobe columns in order."""
    say("probe all equal", nl, nprobe)
    g = np.random.default_rng(nl)
    cent = np.tile(g.standard_normal((1, 64)).astype(np.float32), (nl, 1))
    q = g.standard_normal((9, 64)).astype(np.float32)
    pg = erq.coarse_probe(dev(q), dev(cent), nprobe).cpu().numpy()
    np.testing.assert_array_equal(pg, np.tile(np.arange(nprobe, dtype=pg.dtype), (9, 1)))


def test_rerank_parity():
    say("rerank")
    dp, n, nq, kc, k = 192, 2000, 30, 50, 10
    x = synth.gmm(n, dp, 10, 0.5, seed=31, dp=dp)
    q = synth.gmm(nq, dp, 10, 0.5, seed=31, stream=synth.S_QUERY, dp=dp)
    g = np.random.default_rng(3)
    cand = np.stack([g.choice(n, kc, replace=False) for _ in range(nq)]).astype(np.int64)
    cand[0, :5] = -1
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, 4, 1, dev(P))
    off = np.array([0, n], np.int64)
    ix.import_(dev(off), dev(np.arange(n, dtype=np.int64)), dev(np.zeros((n, dp), np.uint8)),
               dev(np.ones(n, np.float32)), dev(-np.ones(n, np.float32)), dev(np.zeros((1, dp), np.float32)))
    ix.set_raw(dev(x))
    gi, gd = ix.rerank(dev(q), dev(cand), k)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    oi, od = oracle.rerank(x, q, cand, k)
    np.testing.assert_allclose(gd, od, rtol=1e-5)
    _same_up_to_exact_ties(gi, gd, oi, od, x, q)
    # ids outside [0, n) count as missing
    bad = cand.copy()
    bad[:, 1] = n
    bad[:, 2] = n + 12345
    gi2, gd2 = ix.rerank(dev(q), dev(bad), k)
    bad2 = bad.copy()
    bad2[bad2 >= n] = -1
    oi2, od2 = oracle.rerank(x, q, bad2, k)
    np.testing.assert_allclose(gd2.cpu().numpy(), od2, rtol=1e-5)
    _same_up_to_exact_ties(gi2.cpu().numpy(), gd2.cpu().numpy(), oi2, od2, x, q)
    ix.close()


def _same_up_to_exact_ties(gi, gd, oi, od, x, q, rel=1e-5):
    """Re-ranked ids equal the oracle's except where two exact FP64 distances
    lie within the FP32 rounding of each other (either order is correct)."""
    for i in range(gi.shape[0]):
        if np.array_equal(gi[i], oi[i]):
            continue
        kth = od[i][-1]
        for j in set(gi[i].tolist()) ^ set(oi[i].tolist()):
            d = float(((x[j].astype(np.float64) - q[i].astype(np.float64)) ** 2).sum())
            assert abs(d - kth) <= rel * kth, (i, j, d, kth)
        # inside the list only equal-distance neighbours may swap
        np.testing.assert_allclose(gd[i], od[i], rtol=rel)


# ---------------------------------------------------------------------------
# end to end on the tiny GMM workload (10,000 x 128, B = 4)
# ---------------------------------------------------------------------------
def test_build_list_order_deterministic():
    """Members are laid out by list with ids ascending within each list, one
    list longer than 16,384 members included, and two builds of the same
    input export the same index bit for bit."""
    say("build list order")
    dp, nl, n = 64, 8, 60000
    g = np.random.default_rng(91)
    x = synth.gmm(n, dp, 8, 0.5, seed=92, dp=dp)
    assign = g.integers(1, nl, n).astype(np.int32)
    assign[g.choice(n, 20000, replace=False)] = 0
    cent = np.stack([x[assign == l].astype(np.float64).mean(0) for l in range(nl)]).astype(np.float32)
    P = synth.haar_orthogonal(dp, seed=93).astype(np.float32)
    outs = []
    for _ in range(2):
        ix = erq.Index(dp, 4, nl, dev(P))
        ix.build(dev(x), dev(cent), dev(assign))
        outs.append([t.cpu().numpy() for t in ix.export()])
        ix.close()
    for a, b in zip(*outs):
        assert a.tobytes() == b.tobytes()
    off, ids = outs[0][0], outs[0][1]
    np.testing.assert_array_equal(np.diff(off), np.bincount(assign, minlength=nl))
    for l in range(nl):
        seg = ids[off[l]:off[l + 1]]
        np.testing.assert_array_equal(seg, np.nonzero(assign == l)[0])


def test_end_to_end_tiny():
    say("end to end tiny")
    x, q = synth.tiny_gmm()
    dp = x.shape[1]
    P = synth.haar_orthogonal(dp).astype(np.float32)
    c = x.astype(np.float64).mean(0, keepdims=True).astype(np.float32)
    ix = erq.Index(dp, 4, 1, dev(P))
    ix.build(dev(x), dev(c), keep_raw=True)
    off, ids, codes, fa, fr, crot = [t.cpu().numpy() for t in ix.export()]
    assert np.array_equal(ids, np.arange(x.shape[0]))
    # codes against the oracle's FP64 pipeline: rotation rounding may move a
    # coordinate across a boundary, so compare the objective they attain
    oc, ofa, ofr, oco, orr = oracle.encode(x, c.astype(np.float64), np.zeros(len(x), np.int32), P, 4)
    same = (codes == oc).all(1).mean()
    obj_g = np.array([oracle.objective(orr[i], 4, codes[i]) for i in range(0, len(x), 50)])
    obj_o = np.array([oracle.objective(orr[i], 4, oc[i]) for i in range(0, len(x), 50)])
    assert np.all(obj_g >= obj_o * (1 - 1e-6))
    np.testing.assert_allclose(fa, ofa.astype(np.float32), rtol=1e-5)
    say("  identical code rows", same)
    # search: estimated top-10 and re-ranked top-10 against exact k-NN
    ti, td = oracle.knn(x, q, 10)
    ids0, d0 = ix.search(dev(q), 1, 10, 0)
    ids1, d1 = ix.search(dev(q), 1, 10, 32)
    ids0, ids1 = ids0.cpu().numpy(), ids1.cpu().numpy()
    r0 = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(ids0, ti)])
    r1 = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(ids1, ti)])
    say("  recall@10 no rerank", r0, "rerank32", r1)
    assert r0 > 0.55 and r1 > 0.93
    np.testing.assert_allclose(d1.cpu().numpy()[:, 0], td[:, 0], rtol=1e-4)
    ix.close()


@pytest.mark.parametrize("B,planes,nq,kk,nprobe", [(4, 1, 1, 10, 8), (4, 1, 7, 100, 12), (4, 1, 32, 1, 5),
                                                   (3, 1, 20, 1024, 4), (8, 2, 13, 10, 8), (6, 2, 32, 64, 3),
                                                   (1, 1, 5, 10, 4), (4, 1, 300, 10, 16), (5, 2, 1024, 100, 6)])
def test_small_batch_path_identical(B, planes, nq, kk, nprobe):
    """The small-batch path (exact per-query top-kk over probe slices, one
    merge) and the pair-grouped pipeline return the same ids and the same
    FP32 estimates bit for bit, on Zipf lists with ragged tails and queries
    that probe fewer lists; both match the oracle."""
    say("small batch path B", B, "planes", planes, "nq", nq, "kk", kk)
    dp, nl = 192, 16
    sizes = synth.zipf_list_sizes(9000, nl, lo=1, seed=90 + B)
    off, ids, codes, fa, fr, crot = synth.random_index(int(sizes.sum()), nl, dp, B, seed=91 + B, sizes=sizes)
    qrot = synth.random_rotated(nq, dp, seed=92 + B)
    probes = synth.random_probes(nq, nl, nprobe, seed=93 + B)
    probes[: nq // 3, nprobe // 2:] = -1
    P = synth.haar_orthogonal(dp, seed=2).astype(np.float32)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.import_(dev(off), dev(ids), dev(codes), dev(fa), dev(fr), dev(np.zeros((nl, dp), np.float32)), dev(crot))
    if planes == 2:
        ix.set_query_planes(2)
    ix.set_small_batch(0)
    a_i, a_e = [t.cpu().numpy() for t in ix.scan(dev(qrot), dev(probes), kk)]
    ix.set_small_batch(max(nq, 32))
    assert ix.small_batch() == max(nq, 32)
    b_i, b_e = [t.cpu().numpy() for t in ix.scan(dev(qrot), dev(probes), kk)]
    np.testing.assert_array_equal(a_i, b_i)
    np.testing.assert_array_equal(a_e.view(np.uint32), b_e.view(np.uint32))
    oi, oe = oracle.search(off, ids, codes, fa, fr, crot, qrot, probes, B, kk, est_mode=3 if planes == 2 else 0)
    _compare_topk(b_i, b_e, oi, oe, CandTerms(off, ids, codes, fa, fr, crot, qrot, probes, B))
    ix.close()
