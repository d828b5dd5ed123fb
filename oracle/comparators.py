"""Quantisers the paper compares against in its space-accuracy experiment
(Sec. 5.1, algorithms (2)-(4); results in Sec. 5.2.1), for a CPU-only
accuracy comparison on synthetic data.  TEST INFRASTRUCTURE ONLY, like the
rest of ``oracle/``: plain numpy, FP64, no code shared with the GPU library.

Every function returns estimated squared distances (nq x n) between raw
query rows and quantised data rows, after both were centred on the data's
global centroid (the paper's pre-processing for this experiment).

* SQ: one global range [v_l, v_r] over every coordinate of every data
  vector, split uniformly into 2^B - 1 segments; each coordinate rounds to
  its nearest boundary (B-bit unsigned integer); the distance is computed
  from the reconstructed vector.
* LVQ: the same with the range [v_l, v_r] of each vector on its own.
* RaBitQ (pad): the vector padded with zeros to B*D dimensions and
  quantised with the 1-bit RaBitQ codebook of that space (the B = 1 case of
  the extended method, here with the oracle's own quantiser).
* RaBitQ (ext): the extended method with B bits (the oracle's quantiser and
  factor-form estimator with a float query).
"""
from __future__ import annotations

import numpy as np

from . import quantize


def _uniform_sq(X, vl, vr, B):
    """Round every coordinate of X to the nearest of 2^B levels of [vl, vr]
    (vl, vr broadcast against X) and return the reconstruction."""
    L = (1 << B) - 1
    span = np.where(vr > vl, vr - vl, 1.0)
    k = np.clip(np.rint((X - vl) / span * L), 0, L)
    return vl + k * span / L


def _sqdist(Q, Xh):
    return (Q * Q).sum(1)[:, None] + (Xh * Xh).sum(1)[None, :] - 2.0 * Q @ Xh.T


def sq_estimate(X, Q, B):
    """SQ with one global range (Sec. 5.1, algorithm (3))."""
    Xh = _uniform_sq(X, X.min(), X.max(), B)
    return _sqdist(Q, Xh)


def lvq_estimate(X, Q, B):
    """LVQ: a range per vector (Sec. 5.1, algorithm (4))."""
    Xh = _uniform_sq(X, X.min(1, keepdims=True), X.max(1, keepdims=True), B)
    return _sqdist(Q, Xh)


def _factor_estimate(Xr, Qr, B):
    """Extended-RaBitQ estimate with a float query in the rotated space:
    ||r||^2 + ||s||^2 + f_rescale <y_bar, s'> (Eq. eq:dis to ip with Eq. eq
    3.3: represent, factor form)."""
    codes, fa, fr, _ = quantize(Xr, B, norm2=(Xr * Xr).sum(1))
    Y = codes.astype(np.float64) - ((1 << B) - 1) / 2.0
    return (Qr * Qr).sum(1)[:, None] + fa[None, :] + fr[None, :] * (Qr @ Y.T)


def ext_estimate(X, Q, B, P):
    """RaBitQ (ext) with B bits; P: the D x D rotation."""
    return _factor_estimate(X @ P, Q @ P, B)


def pad_estimate(X, Q, B, P_pad):
    """RaBitQ (pad): zero-pad to B*D dimensions, 1-bit RaBitQ there (Sec. 3.1);
    P_pad: the (B*D) x (B*D) rotation."""
    n, D = X.shape
    Xp = np.zeros((n, P_pad.shape[0]))
    Xp[:, :D] = X
    Qp = np.zeros((Q.shape[0], P_pad.shape[0]))
    Qp[:, :D] = Q
    return _factor_estimate(Xp @ P_pad, Qp @ P_pad, 1)


def relative_errors(est, true):
    """(average, maximum) relative error of estimated squared distances (Sec. 5.1 metrics)."""
    rel = np.abs(est - true) / true
    return float(rel.mean()), float(rel.max())
