"""IVF list construction for the benchmark and the tests: Lloyd k-means on the
device with plain torch tensor ops (Sec. 4.1 builds the lists with KMeans).

This is index preparation, outside the quantise / scan path: it produces the
centroids and the row -> list assignment that both the HIP library
(erq_index_build) and the CPU oracle receive as inputs.  Readings: seeded
random initial centroids (distinct rows), a fixed number of Lloyd iterations,
ties to the lowest centroid id (torch.argmin), an empty cluster keeps its
previous centroid.  The per-list sums are accumulated in a fixed order
(torch's deterministic index_add_, which sorts by list before summing), so
the same input and seed give the same centroids and lists on every run.
"""
from __future__ import annotations

import torch


def _assign(x, cent, chunk=65536):
    cn = (cent * cent).sum(1)
    out = torch.empty(x.shape[0], dtype=torch.int64, device=x.device)
    for i in range(0, x.shape[0], chunk):
        xb = x[i:i + chunk]
        d = cn[None, :] - 2.0 * (xb @ cent.T)
        out[i:i + chunk] = torch.argmin(d, dim=1)
    return out


def _list_sums(x, a, nlist):
    prev = torch.are_deterministic_algorithms_enabled()
    torch.use_deterministic_algorithms(True)
    try:
        return torch.zeros((nlist, x.shape[1]), dtype=x.dtype, device=x.device).index_add_(0, a, x)
    finally:
        torch.use_deterministic_algorithms(prev)


def kmeans(x: torch.Tensor, nlist: int, iters: int = 10, seed: int = 240909913):
    """Returns (centroids nlist x dp float32, assign int32) on x's device."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randperm(x.shape[0], generator=g)[:nlist].to(x.device)
    cent = x[idx].clone()
    for _ in range(iters):
        a = _assign(x, cent)
        sums = _list_sums(x, a, nlist)
        cnt = torch.bincount(a, minlength=nlist).to(x.dtype)
        nz = cnt > 0
        cent[nz] = sums[nz] / cnt[nz, None]
    a = _assign(x, cent)
    return cent.contiguous(), a.to(torch.int32).contiguous()
