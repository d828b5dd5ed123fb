"""The k-means that builds the IVF lists for the tests and the benchmark.

On the CPU: one Lloyd step of `ivf.kmeans` against a plain per-list mean
written out with numpy.  On the GPU: two runs on the same input give the same
centroids and lists bit for bit (the per-list sums are accumulated in a fixed
order), so an index, and the recall measured on it, is reproducible.
"""
import numpy as np
import pytest
import torch

from paper_2409_09913_amd import ivf, synth


def _lloyd_numpy(x, cent):
    d = ((x[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
    a = d.argmin(1)
    out = cent.copy()
    for j in range(cent.shape[0]):
        m = a == j
        if m.any():
            out[j] = x[m].mean(0)
    return out, a


def test_kmeans_step_matches_plain_means():
    x = synth.gmm(3000, 16, 8, 0.3, seed=4, stream=synth.S_BASE).astype(np.float64)
    xt = torch.from_numpy(x)
    nl = 24
    g = torch.Generator(device="cpu").manual_seed(7)
    idx = torch.randperm(x.shape[0], generator=g)[:nl]
    c1, a1 = ivf.kmeans(xt, nl, iters=1, seed=7)
    ref, _ = _lloyd_numpy(x, x[idx.numpy()])
    np.testing.assert_allclose(c1.numpy(), ref, rtol=0, atol=1e-12)
    _, aref = _lloyd_numpy(x, ref)
    # the returned assignment is to the updated centroids
    assert (a1.numpy() == aref).mean() > 0.999


@pytest.mark.gpu
def test_kmeans_repeatable_on_device():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(synth.gmm(200000, 128, 64, 0.3, seed=9, stream=synth.S_BASE)).to(dev)
    runs = [ivf.kmeans(x, 512, iters=4) for _ in range(2)]
    c0, a0 = runs[0]
    c1, a1 = runs[1]
    assert torch.equal(a0, a1)
    assert torch.equal(c0.view(torch.int32), c1.view(torch.int32))
