"""Pins of the oracle's projection to d < D dimensions before quantising
(App. C), CPU only.  The estimate of ||o_r - q_r||^2 is ||r||^2 + ||s||^2 -
(2D/d) <P_d r, P_d s> with the projected inner product estimated by the
extended codes.  Pins: d = D reduces to the plain encoding exactly; over
random rotations the estimate is unbiased (Johnson-Lindenstrauss for the
projection, Lemma 2.1 for the codes); the error grows as d shrinks."""
import math

import numpy as np

import oracle
from paper_2409_09913_amd import synth


def test_full_dimension_is_the_plain_encoding():
    g = np.random.default_rng(41)
    D, n, B = 64, 200, 4
    x = g.standard_normal((n, D))
    cent = g.standard_normal((3, D))
    asg = g.integers(0, 3, n).astype(np.int32)
    P = synth.haar_orthogonal(D, seed=42)
    c1, fa1, fr1, _, _ = oracle.encode(x, cent, asg, P, B)
    c2, fa2, fr2 = oracle.encode_proj(x, cent, asg, P, B, D)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(fa2, fa1, rtol=1e-12)
    np.testing.assert_allclose(fr2, fr1, rtol=1e-12)


def _est(x, c, q, P, B, dc):
    codes, fa, fr = oracle.encode_proj(x[None, :], c[None, :], np.zeros(1, np.int32), P, B, dc)
    s = (q - c) @ P
    y = codes[0].astype(np.float64) - ((1 << B) - 1) / 2.0
    return fa[0] + s @ s + fr[0] * (y @ s[:dc])


def test_projection_unbiased_over_rotations():
    D, dc, B, M = 64, 16, 3, 2000
    g = np.random.default_rng(43)
    x, c = g.standard_normal(D), 0.2 * g.standard_normal(D)
    q = x + 0.8 * g.standard_normal(D)
    est = np.array([_est(x, c, q, synth.haar_orthogonal(D, seed=9000 + m), B, dc) for m in range(M)])
    true = float(((x - q) ** 2).sum())
    assert abs(est.mean() - true) < 4 * est.std() / math.sqrt(M)


def test_projection_error_grows_as_d_shrinks():
    D, B = 128, 4
    g = np.random.default_rng(44)
    err = {}
    for dc in (16, 32, 64, 128):
        e = []
        for m in range(150):
            x, q = g.standard_normal(D), g.standard_normal(D)
            c = np.zeros(D)
            e.append(abs(_est(x, c, q, synth.haar_orthogonal(D, seed=500 + m), B, dc) - ((x - q) ** 2).sum()))
        err[dc] = np.mean(e)
    assert err[16] > err[32] > err[64] > err[128], err
