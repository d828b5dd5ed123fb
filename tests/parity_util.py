"""Comparison helpers shared by the GPU parity tests (numpy only).

FP32 estimates are compared with the tolerance of reading C-15: 1e-4
relative to the magnitude of the terms that form each candidate's own
estimate, f_add + ||s||^2 + |f_rescale <y_bar, s'>| (an estimate is a
difference of large terms and can be near zero or negative).  Top-k id sets
must agree except for ids at the boundary (near-ties of the k-th value).
"""
import numpy as np


class CandTerms:
    """Per-candidate term magnitude of reading C-15 for (query, member id)."""

    def __init__(self, off, ids, codes, fa, fr, crot, qrot, probes, B, metric="l2"):
        self.off = np.asarray(off, np.int64)
        self.pos = np.empty(int(np.max(ids)) + 1 if len(ids) else 0, np.int64)
        self.pos[np.asarray(ids, np.int64)] = np.arange(len(ids))
        self.codes, self.fa, self.fr = codes, fa, fr
        self.crot, self.qrot, self.probes = crot, qrot, probes
        self.half = ((1 << B) - 1) / 2.0
        self.metric = metric

    def __call__(self, iq, mid):
        """f_add + ||s||^2 + |f_rescale <y_bar, s'>| of member `mid` for query iq."""
        p = int(self.pos[mid])
        l = int(np.searchsorted(self.off, p, side="right") - 1)
        assert l in set(int(v) for v in self.probes[iq]), (iq, mid, l)
        yb = self.codes[p].astype(np.float64) - self.half
        if self.metric != "l2":
            # negated inner product -<c', q'> + (f_rescale / 2) <y_bar, q'>: its two terms
            q = self.qrot[iq].astype(np.float64)
            return abs(float(self.crot[l].astype(np.float64) @ q)) + abs(0.5 * float(self.fr[p]) * float(yb @ q))
        s = self.qrot[iq].astype(np.float64) - self.crot[l].astype(np.float64)
        # codes narrower than s (a projection): they meet its first coordinates
        return abs(float(self.fa[p])) + float(s @ s) + abs(float(self.fr[p]) * float(yb @ s[:yb.shape[0]]))


def compare_topk(gi, ge, oi, oe, terms, rel=1e-4):
    """gi/ge: the GPU's top-k ids and FP32 estimates; oi/oe: the oracle's.
    Each id in both lists: |gpu - oracle| <= rel * its own terms.  An id in
    one list only must be a boundary near-tie of the oracle's k-th value.
    The GPU's list is ascending by (estimate, id)."""
    for q in range(gi.shape[0]):
        valid_o = oi[q] >= 0
        valid_g = gi[q] >= 0
        np.testing.assert_array_equal(valid_g, valid_o, err_msg=f"query {q}: candidate counts differ")
        g_ids, g_e = gi[q][valid_g], ge[q][valid_g].astype(np.float64)
        o_ids, o_e = oi[q][valid_o], oe[q][valid_o]
        # ascending by (estimate, id)
        for t in range(1, len(g_ids)):
            assert (g_e[t - 1] < g_e[t]) or (g_e[t - 1] == g_e[t] and g_ids[t - 1] < g_ids[t]), (q, t)
        gmap = dict(zip(g_ids.tolist(), g_e.tolist()))
        omap = dict(zip(o_ids.tolist(), o_e.tolist()))
        for i in set(gmap) & set(omap):
            tol = rel * terms(q, i)
            assert abs(gmap[i] - omap[i]) <= tol, (q, i, gmap[i], omap[i], tol)
        diff = set(gmap) ^ set(omap)
        if diff:
            kth_id, kth = int(o_ids[-1]), float(o_e[-1])
            t_kth = rel * terms(q, kth_id)
            for i in diff:
                val = gmap[i] if i in gmap else omap[i]
                tol = rel * terms(q, i) + t_kth
                assert abs(val - kth) <= tol, (q, i, val, kth, tol)


def both_paths(ix, run):
    """Runs `run()` (returning numpy (ids, estimates or distances)) once on the
    scan's pair-grouped pipeline and once on its small-batch path, asserts the
    two results are bit-identical, restores the index's threshold and returns
    the pipeline's result."""
    keep = ix.small_batch()
    try:
        ix.set_small_batch(0)
        a_i, a_e = run()
        ix.set_small_batch(1024)
        b_i, b_e = run()
    finally:
        ix.set_small_batch(keep)
    np.testing.assert_array_equal(a_i, b_i, err_msg="small-batch path: ids differ from the pipeline's")
    np.testing.assert_array_equal(np.asarray(a_e).view(np.uint32), np.asarray(b_e).view(np.uint32),
                                  err_msg="small-batch path: values differ from the pipeline's")
    return a_i, a_e
