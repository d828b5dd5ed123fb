"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds none of the method's arithmetic: it only draws random
numbers (NumPy Philox, counter-based, chunked so any block of rows can be
regenerated on its own) and shapes them like the workloads the paper measures
on.  The random orthogonal matrix P that the method samples (Sec. 3.2.1) is
drawn here and handed to both the GPU library and the oracle as an input.

Recipes (named by what they are, with their sizes):
  * gmm(...)         Gaussian mixture, component means ~ N(0, I), isotropic
                     sigma, equal or Zipf(s=1) weights, optional per-vector
                     rescale to a LogNormal(0, 0.2) norm.
  * anisotropic(...) Gaussian with per-dimension variance i^-0.5.
  * spherical_clusters(...) unit vectors around uniform directions
                     (embedding-like).
  * gmm_device(...), clustered_anisotropic_device(...): the same kinds of
                     rows drawn on the GPU with a seeded torch generator, for
                     workloads too large to draw on the host (5M x 3072).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED = 240909913
CHUNK = 1 << 16

# stream offsets
S_BASE, S_QUERY, S_ROT, S_KMEANS, S_ARRIVAL, S_MEANS, S_AUX = 0, 1, 2, 3, 4, 5, 6


def rng(seed: int, stream: int = 0, block: int = 0) -> np.random.Generator:
    """Counter-based generator for (seed, stream, block)."""
    key = np.array([np.uint64(seed) ^ (np.uint64(stream) << np.uint64(40)), np.uint64(block)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def pad_dim(d: int) -> int:
    """Dimension padded to a multiple of 64 (Sec. 5.1)."""
    return 64 * ((d + 63) // 64)


def haar_orthogonal(dp: int, seed: int = SEED) -> np.ndarray:
    """Random orthogonal dp x dp matrix, Haar distributed: QR of a standard
    Gaussian matrix with the signs of R's diagonal folded into Q (Mezzadri,
    "How to generate random matrices from the classical compact groups",
    2007).  Returned in FP64; callers store it as FP32."""
    g = rng(seed, S_ROT).standard_normal((dp, dp))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def _zipf_weights(k: int) -> np.ndarray:
    w = 1.0 / np.arange(1, k + 1, dtype=np.float64)
    return w / w.sum()


def _parallel_rows(n: int, fill, dtype=np.float32, d: int = 1, workers: int = 8) -> np.ndarray:
    out = np.empty((n, d), dtype)
    blocks = [(b, b * CHUNK, min(n, (b + 1) * CHUNK)) for b in range((n + CHUNK - 1) // CHUNK)]

    def work(t):
        b, lo, hi = t
        fill(b, out[lo:hi])

    if len(blocks) <= 1:
        for t in blocks:
            work(t)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(work, blocks))
    return out


def gmm(n: int, d: int, ncomp: int, sigma: float = 0.3, zipf: bool = False,
        lognormal_norm: float | None = None, seed: int = SEED, stream: int = S_BASE,
        dp: int | None = None, return_labels: bool = False):
    """n rows of a ncomp-component Gaussian mixture in d dims, zero-padded to dp.
    Means ~ N(0, I) (drawn once per seed), noise sigma * N(0, I); weights equal
    or Zipf(s=1); optional rescale of every row to a norm ~ LogNormal(0, s)."""
    dp = dp or pad_dim(d)
    means = rng(seed, S_MEANS).standard_normal((ncomp, d)).astype(np.float32)
    w = _zipf_weights(ncomp) if zipf else np.full(ncomp, 1.0 / ncomp)
    cdf = np.cumsum(w)
    cdf[-1] = 1.0
    labels = np.empty(n, np.int32)

    def fill(b, blk):
        g = rng(seed, stream, b)
        m = blk.shape[0]
        lab = np.searchsorted(cdf, g.random(m), side="right").astype(np.int32)
        lab = np.minimum(lab, ncomp - 1)
        lo = b * CHUNK
        labels[lo:lo + m] = lab
        x = means[lab] + np.float32(sigma) * g.standard_normal((m, d), dtype=np.float32)
        if lognormal_norm is not None:
            rho = np.exp(lognormal_norm * g.standard_normal(m)).astype(np.float32)
            nrm = np.linalg.norm(x, axis=1)
            nrm[nrm == 0] = 1
            x *= (rho / nrm)[:, None]
        blk[:, :d] = x
        blk[:, d:] = 0

    x = _parallel_rows(n, fill, d=dp)
    return (x, labels) if return_labels else x


def anisotropic(n: int, d: int, seed: int = SEED, stream: int = S_BASE, dp: int | None = None):
    """Gaussian with variance i^-0.5 in dimension i (1-based), zero-padded."""
    dp = dp or pad_dim(d)
    sd = (np.arange(1, d + 1, dtype=np.float64) ** -0.25).astype(np.float32)

    def fill(b, blk):
        g = rng(seed, stream, b)
        blk[:, :d] = g.standard_normal((blk.shape[0], d), dtype=np.float32) * sd
        blk[:, d:] = 0

    return _parallel_rows(n, fill, d=dp)


def spherical_clusters(n: int, d: int, ncomp: int, tau: float = 1.0, seed: int = SEED,
                       stream: int = S_BASE, dp: int | None = None):
    """Unit vectors normalize(mu_j + tau * g / sqrt(d)), mu_j uniform on the sphere."""
    dp = dp or pad_dim(d)
    mu = rng(seed, S_MEANS).standard_normal((ncomp, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    mu = mu.astype(np.float32)

    def fill(b, blk):
        g = rng(seed, stream, b)
        m = blk.shape[0]
        lab = g.integers(0, ncomp, m)
        x = mu[lab] + np.float32(tau / np.sqrt(d)) * g.standard_normal((m, d), dtype=np.float32)
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        blk[:, :d] = x
        blk[:, d:] = 0

    return _parallel_rows(n, fill, d=dp)


# --------------------------------------------------------------------------
# Configurations (sizes of the workloads the paper's experiments use).
# --------------------------------------------------------------------------
def tiny_gmm(seed: int = SEED):
    """10,000 x 128 base, 100 queries; 16-component GMM, sigma 0.3, equal weights."""
    x = gmm(10_000, 128, 16, 0.3, seed=seed, stream=S_BASE)
    q = gmm(100, 128, 16, 0.3, seed=seed, stream=S_QUERY)
    return x, q


def embed768(n: int = 1_000_000, nq: int = 10_000, seed: int = SEED):
    """1,000,000 x 768 base and 10,000 queries; 1024-component GMM with Zipf
    weights, sigma 0.3, each row rescaled to a LogNormal(0, 0.2) norm."""
    x = gmm(n, 768, 1024, 0.3, zipf=True, lognormal_norm=0.2, seed=seed, stream=S_BASE)
    q = gmm(nq, 768, 1024, 0.3, zipf=True, lognormal_norm=0.2, seed=seed, stream=S_QUERY)
    return x, q


# --------------------------------------------------------------------------
# Synthetic index contents and probe lists (for stage-isolated parity tests).
# --------------------------------------------------------------------------
def zipf_list_sizes(n: int, nlist: int, lo: int = 1, seed: int = SEED) -> np.ndarray:
    """nlist sizes summing to n, skewed like Zipf(1) with a random order."""
    w = _zipf_weights(nlist) * 0.5 + 0.5 / nlist
    sizes = np.maximum(lo, np.floor(w * n).astype(np.int64))
    diff = n - sizes.sum()
    g = rng(seed, S_AUX, 1)
    while diff != 0:
        j = g.integers(0, nlist)
        if diff > 0:
            sizes[j] += 1
            diff -= 1
        elif sizes[j] > lo:
            sizes[j] -= 1
            diff += 1
    g.shuffle(sizes)
    return sizes


def random_index(n: int, nlist: int, dp: int, B: int, seed: int = SEED, sizes=None,
                 empty_lists: int = 0):
    """Index contents with uniform random codes and plausible factors:
    list offsets, ids (a random permutation), codes y_u in [0, 2^B), f_add > 0,
    f_rescale < 0 and rotated centroids.  Used to drive the scan arithmetic."""
    g = rng(seed, S_AUX, 2)
    if sizes is None:
        sizes = zipf_list_sizes(n, nlist, seed=seed)
    sizes = np.asarray(sizes, np.int64).copy()
    if empty_lists:
        idx = g.choice(nlist, empty_lists, replace=False)
        moved = sizes[idx].sum()
        sizes[idx] = 0
        sizes[np.argmax(sizes)] += moved
    off = np.zeros(nlist + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    ids = g.permutation(n).astype(np.int64)
    codes = g.integers(0, 1 << B, (n, dp), dtype=np.uint8)
    f_add = (g.random(n) * 2 + 0.1).astype(np.float32)
    f_rescale = (-(g.random(n) * 0.5 + 0.05)).astype(np.float32)
    crot = g.standard_normal((nlist, dp), dtype=np.float32)
    return off, ids, codes, f_add, f_rescale, crot


def random_probes(nq: int, nlist: int, nprobe: int, seed: int = SEED) -> np.ndarray:
    """nprobe distinct list ids per query."""
    g = rng(seed, S_AUX, 3)
    out = np.empty((nq, nprobe), np.int32)
    for i in range(nq):
        out[i] = g.choice(nlist, nprobe, replace=False)
    return out


def random_rotated(n: int, dp: int, seed: int = SEED, block: int = 4, scale: float = 1.0):
    """FP32 rows standing in for rotated residuals r' (stage-isolated tests)."""
    return (scale * rng(seed, S_AUX, block).standard_normal((n, dp))).astype(np.float32)


def edge_rows(dp: int, seed: int = SEED) -> np.ndarray:
    """Adversarial FP32 rows for the quantiser: zeros, one-hot, equal
    magnitudes, power-of-two ratios (exact ties of critical values), signed
    zeros, huge and tiny scales, a single non-zero in the last dimension."""
    g = rng(seed, S_AUX, 5)
    rows = []
    rows.append(np.zeros(dp))
    oh = np.zeros(dp); oh[3 % dp] = -2.5; rows.append(oh)
    rows.append(np.ones(dp))
    rows.append(np.where(g.random(dp) < 0.5, -1.0, 1.0))
    pw = 2.0 ** g.integers(-3, 4, dp) * np.where(g.random(dp) < 0.5, -1.0, 1.0); rows.append(pw)
    sz = np.zeros(dp); sz[::2] = -0.0; sz[1::2] = 0.75; rows.append(sz)
    rows.append(g.standard_normal(dp) * 1e30)
    rows.append(g.standard_normal(dp) * 1e-30)
    last = np.zeros(dp); last[-1] = 1e-3; rows.append(last)
    few = np.zeros(dp); few[:5] = [3.0, -1.5, 0.75, 3.0, -6.0]; rows.append(few)
    mix = g.standard_normal(dp); mix[g.random(dp) < 0.5] = 0.0; rows.append(mix)
    q = np.round(g.standard_normal(dp) * 4) / 4; rows.append(q)
    return np.asarray(rows, dtype=np.float32)


# --------------------------------------------------------------------------
# Device-side draws for the largest workloads (seeded torch generators).
# --------------------------------------------------------------------------
def gmm_device(n: int, d: int, ncomp: int, sigma: float = 0.3, zipf: bool = False, seed: int = SEED,
               stream: int = S_BASE, device="cuda", chunk: int = 1 << 18):
    """n x d rows of the Gaussian mixture of gmm() (same component means),
    drawn on `device` in chunks; returns (rows float32, labels int64)."""
    import torch
    means = torch.from_numpy(rng(seed, S_MEANS).standard_normal((ncomp, d)).astype(np.float32)).to(device)
    w = _zipf_weights(ncomp) if zipf else np.full(ncomp, 1.0 / ncomp)
    wt = torch.from_numpy(w).to(device)
    g = torch.Generator(device=device).manual_seed(int(seed) * 16 + stream)
    x = torch.empty((n, d), dtype=torch.float32, device=device)
    lab = torch.empty(n, dtype=torch.int64, device=device)
    for lo in range(0, n, chunk):
        m = min(chunk, n - lo)
        lb = torch.multinomial(wt, m, replacement=True, generator=g)
        x[lo:lo + m] = means[lb] + sigma * torch.randn((m, d), device=device, generator=g)
        lab[lo:lo + m] = lb
    return x, lab


def spherical_clusters_device(n: int, d: int, ncomp: int, tau: float = 1.0, seed: int = SEED,
                              stream: int = S_BASE, device="cuda", chunk: int = 1 << 18):
    """n unit vectors normalize(mu_j + tau * g / sqrt(d)) of spherical_clusters()
    (same centres mu_j, uniform on the sphere, equal weights), drawn on `device`
    in chunks; returns rows float32."""
    import torch
    mu = rng(seed, S_MEANS).standard_normal((ncomp, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    mu = torch.from_numpy(mu.astype(np.float32)).to(device)
    g = torch.Generator(device=device).manual_seed(int(seed) * 16 + stream)
    x = torch.empty((n, d), dtype=torch.float32, device=device)
    for lo in range(0, n, chunk):
        m = min(chunk, n - lo)
        lb = torch.randint(0, ncomp, (m,), device=device, generator=g)
        y = mu[lb] + (tau / float(np.sqrt(d))) * torch.randn((m, d), device=device, generator=g)
        x[lo:lo + m] = y / torch.linalg.vector_norm(y, dim=1, keepdim=True)
    return x


def clustered_anisotropic_device(sizes, d: int, noise: float = 0.5, seed: int = SEED, device="cuda",
                                 chunk: int = 1 << 18):
    """Clusters of the given sizes around centres drawn from the Gaussian with
    variance i^-0.5 in dimension i; members = centre + noise * (a draw of the
    same Gaussian).  Returns (rows float32 on device, labels int32, centres
    float32 on device); rows are ordered by cluster."""
    import torch
    sizes = np.asarray(sizes, np.int64)
    sd = torch.from_numpy((np.arange(1, d + 1, dtype=np.float64) ** -0.25).astype(np.float32)).to(device)
    g = torch.Generator(device=device).manual_seed(int(seed) * 16 + S_MEANS)
    cent = torch.randn((len(sizes), d), device=device, generator=g) * sd
    lab = torch.from_numpy(np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)).to(device)
    n = int(sizes.sum())
    x = torch.empty((n, d), dtype=torch.float32, device=device)
    g2 = torch.Generator(device=device).manual_seed(int(seed) * 16 + S_BASE)
    for lo in range(0, n, chunk):
        m = min(chunk, n - lo)
        x[lo:lo + m] = cent[lab[lo:lo + m].long()] + noise * torch.randn((m, d), device=device, generator=g2) * sd
    return x, lab, cent


def power_law_sizes(nlist: int, lo: int, hi: int, alpha: float, seed: int = SEED) -> np.ndarray:
    """nlist sizes from a Pareto law of exponent alpha truncated to [lo, hi]."""
    g = rng(seed, S_AUX, 7)
    u = g.random(nlist)
    return np.clip(np.floor(lo * (1.0 - u) ** (-1.0 / alpha)), lo, hi).astype(np.int64)
