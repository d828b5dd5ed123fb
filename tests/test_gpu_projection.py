"""Random projection to dc < dp dimensions before quantising (App. C) on the
device, against the oracle (oracle.encode_proj, oracle.search with codes
narrower than the rotated queries).

* Build: the codes attain the oracle's objective on the first dc
  coordinates of the FP64 rotated residual (FP32 rotation rounding may move
  a coordinate across a boundary); f_add = ||r||^2 over all dp; f_rescale
  (scaled by dp/dc) within the FP32 rotation's error for identical codes.
* Scan (erq_scan, full-width rotated queries: the per-pair ||s'||^2 over all
  dp) and search (erq_search, queries rotated to dc coordinates only) against
  oracle.search on the exported codes, per candidate at the tolerance of
  reading C-15.
* Save / load keeps the code dimension; the call is refused on a built
  index, for a dc that is not a multiple of 64 in [64, dp], and for the
  inner-product metrics.
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


def _case(dp, nl, n, nq, seed):
    x = synth.gmm(n, dp, 32, 0.3, seed=seed, dp=dp)
    q = synth.gmm(nq, dp, 32, 0.3, seed=seed, stream=synth.S_QUERY, dp=dp)
    P = synth.haar_orthogonal(dp, seed=seed + 1).astype(np.float32)
    cent = x[:nl].copy()                                  # list centres: the first nl rows
    assign = oracle.probe(x, cent, 1)[0][:, 0].astype(np.int32)   # nearest centre (FP64)
    return x, q, P, cent, assign


@pytest.fixture(scope="module", params=[(128, 4), (192, 7)], ids=["dc128-B4", "dc192-B7"])
def built(request):
    dc, B = request.param
    dp, nl, n, nq = 256, 24, 24000, 40
    say("projection build dp", dp, "dc", dc, "B", B)
    x, q, P, cent, assign = _case(dp, nl, n, nq, seed=300 + dc + B)
    ix = erq.Index(dp, B, nl, dev(P))
    ix.set_projection(dc)
    assert ix.code_dim() == dc
    ix.build(dev(x), dev(cent), dev(assign), precision=0)
    torch.cuda.synchronize()
    off, ids, codes, fa, fr, _ = [t.cpu().numpy() for t in ix.export()]
    assert codes.shape == (n, dc)
    crot = oracle.rotate(cent, P).astype(np.float32)       # the oracle's own rotated centres (all dp)
    yield dict(ix=ix, x=x, q=q, P=P, cent=cent, assign=assign, dc=dc, B=B, off=off, ids=ids, codes=codes,
               fa=fa, fr=fr, crot=crot)
    ix.close()


def test_projection_build_matches_oracle(built):
    b = built
    dc, B = b["dc"], b["B"]
    oc, ofa, ofr = oracle.encode_proj(b["x"], b["cent"].astype(np.float64), b["assign"], b["P"], B, dc)
    # the device's arrays in row order
    pos = np.empty_like(b["ids"])
    pos[b["ids"]] = np.arange(len(b["ids"]))
    gc, gfa, gfr = b["codes"][pos], b["fa"][pos], b["fr"][pos]
    np.testing.assert_allclose(gfa, ofa, rtol=1e-5)
    rr = oracle.rotate(b["x"].astype(np.float64) - b["cent"][b["assign"]].astype(np.float64), b["P"])[:, :dc]
    for i in range(0, len(gc), 40):
        og, oo = oracle.objective(rr[i], B, gc[i]), oracle.objective(rr[i], B, oc[i])
        assert og >= oo * (1 - 1e-6), (i, og, oo)
    same = (gc == oc).all(1)
    assert same.mean() > 0.9
    np.testing.assert_allclose(gfr[same], ofr[same], rtol=2e-4)
    # list membership and ids follow the oracle's assignment
    np.testing.assert_array_equal(np.diff(b["off"]), np.bincount(b["assign"], minlength=len(b["cent"])))
    say("  identical code rows %.4f" % same.mean())


@pytest.mark.parametrize("nprobe,kk", [(4, 10), (12, 100)])
def test_projection_scan_matches_oracle(built, nprobe, kk):
    b = built
    qrot = erq.rotate(dev(b["q"]), dev(b["P"]), precision=0)      # full width: ||s'||^2 over every dp
    probes = oracle.probe(b["q"], b["cent"], nprobe)[0].astype(np.int32)
    gi, ge = both_paths(b["ix"], lambda: [t.cpu().numpy() for t in b["ix"].scan(qrot, dev(probes), kk)])
    qr = qrot.cpu().numpy()
    oi, oe = oracle.search(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], qr, probes, b["B"], kk,
                           est_mode=0)
    compare_topk(gi, ge, oi, oe, CandTerms(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], qr,
                                           probes, b["B"]))


@pytest.mark.parametrize("nprobe,k", [(6, 10), (16, 50)])
def test_projection_search_matches_oracle(built, nprobe, k):
    b = built
    qd = dev(b["q"])
    gi, ge = both_paths(b["ix"], lambda: [t.cpu().numpy() for t in b["ix"].search(qd, nprobe, k, 0)])
    probes = erq.coarse_probe(qd, dev(b["cent"]), nprobe).cpu().numpy()     # the search's probes
    qrot = erq.rotate(qd, dev(b["P"]), precision=2).cpu().numpy()           # its first dc columns: the search's
    oi, oe = oracle.search(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], qrot, probes, b["B"], k,
                           est_mode=0)
    compare_topk(gi, ge, oi, oe, CandTerms(b["off"], b["ids"], b["codes"], b["fa"], b["fr"], b["crot"], qrot,
                                           probes, b["B"]))
    same = np.mean([set(a) == set(o) for a, o in zip(gi, oi)])
    say("  identical id sets: %.3f of queries" % same)


def test_projection_save_load(built, tmp_path):
    b = built
    path = str(tmp_path / "proj.erq")
    b["ix"].save(path)
    iy = erq.Index.load_file(path)
    assert iy.code_dim() == b["dc"]
    for u, v in zip(b["ix"].export(), iy.export()):
        assert torch.equal(u.cpu().view(torch.uint8), v.cpu().view(torch.uint8))
    qd = dev(b["q"])
    a = b["ix"].search(qd, 8, 10, 0)
    c = iy.search(qd, 8, 10, 0)
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and torch.equal(a[1].view(torch.int32), c[1].view(torch.int32))
    iy.close()


def test_projection_refusals(built):
    with pytest.raises(erq.ErqError) as e:
        built["ix"].set_projection(64)                    # the index already holds vectors
    assert e.value.code == erq.ERQ_EINVAL
    ix = erq.Index(256, 4, 4, None, seed=1)
    for dc in (0, 32, 100, 320):
        with pytest.raises(erq.ErqError) as e:
            ix.set_projection(dc)
        assert e.value.code == erq.ERQ_ESHAPE
    ix.set_projection(256)                                # dc = dp: no projection
    assert ix.code_dim() == 256
    ix.close()
    iz = erq.Index(256, 4, 4, None, seed=1, metric="ip")
    with pytest.raises(erq.ErqError) as e:
        iz.set_projection(128)
    assert e.value.code == erq.ERQ_EUNSUPPORTED
    iz.close()
