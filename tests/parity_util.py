"""Comparison helpers shared by the GPU parity tests (numpy only).

FP32 estimates are compared with the tolerance of reading C-15: 1e-4
relative to the magnitude of the terms that form them (an estimate is a
difference of large terms and can be near zero or negative).  Top-k id sets
must agree except for ids at the k-th value (near-ties).
"""
import numpy as np


def term_scale(codes, fa, fr, crot, qrot, off, ids_o, q_ids, probes, B):
    """Per query: the largest |f_add| + ||s||^2 + |f_rescale <y,s'>| over its candidates."""
    out = np.zeros(qrot.shape[0])
    yb = codes.astype(np.float64) - ((1 << B) - 1) / 2.0
    for iq in range(qrot.shape[0]):
        m = 0.0
        for l in probes[iq]:
            if l < 0:
                continue
            s = qrot[iq].astype(np.float64) - crot[l].astype(np.float64)
            lo, hi = off[l], off[l + 1]
            if hi > lo:
                t = np.abs(fa[lo:hi]) + s @ s + np.abs(fr[lo:hi] * (yb[lo:hi] @ s))
                m = max(m, float(t.max()))
        out[iq] = m
    return out


def compare_topk(gi, ge, oi, oe, scale, rel=1e-4):
    for q in range(gi.shape[0]):
        tol = rel * scale[q] + 1e-30
        valid_o = oi[q] >= 0
        valid_g = gi[q] >= 0
        np.testing.assert_array_equal(valid_g, valid_o)
        assert np.all(np.abs(ge[q][valid_g] - oe[q][valid_o]) <= tol), (q, ge[q], oe[q])
        sg, so = set(gi[q][valid_g].tolist()), set(oi[q][valid_o].tolist())
        if sg != so:
            kth = oe[q][valid_o][-1]
            for i in sg ^ so:
                # an id that is in one list only must sit at the boundary (near-tie)
                pos = np.nonzero(gi[q] == i)[0]
                val = ge[q][pos[0]] if pos.size else oe[q][np.nonzero(oi[q] == i)[0][0]]
                assert abs(val - kth) <= 2 * tol, (q, i, val, kth)
