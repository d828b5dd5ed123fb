"""The library's k-means (erq_kmeans) and the index build's list layout.

* Zero rounds return the seeded initial centroids (distinct rows) and the
  nearest-centroid assignment to them; the assignment agrees with exact FP64
  nearest centroids except where two distances lie within the probe's error
  bound.
* One round: every centroid is the plain FP64 mean of its list under that
  assignment (numpy), and an empty list keeps its centroid.
* Two runs give the same centroids and lists bit for bit, and a build
  without centroids uses the library's k-means with the index's seed.
"""
import numpy as np
import pytest
import torch

from paper_2409_09913_amd import erq, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def test_kmeans_lloyd_step_matches_plain_means():
    n, d, nl = 20000, 64, 40
    x = synth.gmm(n, d, 8, 0.3, seed=4, stream=synth.S_BASE, dp=d)
    xd = torch.from_numpy(x).to(DEV)
    c0, a0 = erq.kmeans(xd, nl, iters=0, seed=7)
    c0, a0 = c0.cpu().numpy(), a0.cpu().numpy()
    # initial centroids are distinct rows of x
    rows = [np.nonzero((x == c0[j]).all(1))[0] for j in range(nl)]
    assert all(len(r) >= 1 for r in rows) and len({int(r[0]) for r in rows}) == nl
    # nearest centroid, exact up to the probe's error bound
    x64, c64 = x.astype(np.float64), c0.astype(np.float64)
    D = (x64 ** 2).sum(1)[:, None] + (c64 ** 2).sum(1)[None, :] - 2 * x64 @ c64.T
    best = D.argmin(1)
    bad = np.nonzero(best != a0)[0]
    tol = 2 * (2.0 ** -15 + 4 * d * U32) * ((x64 ** 2).sum(1) + (c64 ** 2).sum(1).max())
    assert np.all(D[bad, a0[bad]] - D[bad, best[bad]] <= tol[bad])
    # one round: plain means of the lists of that assignment
    c1, _ = erq.kmeans(xd, nl, iters=1, seed=7)
    c1 = c1.cpu().numpy()
    for j in range(nl):
        m = a0 == j
        ref = x64[m].mean(0) if m.any() else c64[j]
        np.testing.assert_allclose(c1[j], ref, rtol=1e-6, atol=1e-7)


def test_kmeans_repeatable_and_used_by_build():
    x = torch.from_numpy(synth.gmm(200000, 128, 64, 0.3, seed=9, stream=synth.S_BASE)).to(DEV)
    runs = [erq.kmeans(x, 512, iters=4, seed=11) for _ in range(2)]
    assert torch.equal(runs[0][1], runs[1][1])
    assert torch.equal(runs[0][0].view(torch.int32), runs[1][0].view(torch.int32))
    # the build's lists: ascending row ids within each list, sizes of the assignment
    ix = erq.Index(128, 4, 512, None, seed=5)
    ix.build(x[:50000].contiguous())
    off, ids = ix.export()[:2]
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    assert off[-1] == 50000 and (np.diff(off) >= 0).all()
    for l in range(0, 512, 37):
        seg = ids[off[l]:off[l + 1]]
        assert (np.diff(seg) > 0).all()
    ix.close()
