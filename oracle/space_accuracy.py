"""Space-accuracy comparison of Sec. 5.2.1 on synthetic data (CPU only):
average and maximum relative error of estimated squared distances of
RaBitQ (ext), RaBitQ (pad), SQ and LVQ at B = 1..8 bits per dimension.

Data: a 16-component Gaussian mixture (means N(0, I), sigma 0.3), centred on
its global centroid as in the paper's pre-processing; queries are fresh
draws of the same mixture.  Bits per dimension include each method's
per-vector floats (two for RaBitQ (ext), RaBitQ (pad) and LVQ).

    python -m oracle.space_accuracy [--d 256] [--n 5000] [--nq 50]
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import comparators as cmp          # noqa: E402
from paper_2409_09913_amd import synth          # noqa: E402


def table(d=256, n=5000, nq=50, bits=range(1, 9), seed=240909913):
    X = synth.gmm(n, d, 16, 0.3, seed=seed, stream=synth.S_BASE).astype(np.float64)
    Q = synth.gmm(nq, d, 16, 0.3, seed=seed, stream=synth.S_QUERY).astype(np.float64)
    c = X.mean(0)
    X, Q = X - c, Q - c
    true = (Q * Q).sum(1)[:, None] + (X * X).sum(1)[None, :] - 2.0 * Q @ X.T
    P = synth.haar_orthogonal(d, seed=seed)
    rows = []
    for B in bits:
        ext = cmp.relative_errors(cmp.ext_estimate(X, Q, B, P), true)
        pad = cmp.relative_errors(cmp.pad_estimate(X, Q, B, synth.haar_orthogonal(B * d, seed=seed + B)), true)
        sq = cmp.relative_errors(cmp.sq_estimate(X, Q, B), true)
        lvq = cmp.relative_errors(cmp.lvq_estimate(X, Q, B), true)
        rows.append(dict(B=B, bits_per_dim=dict(ext=B + 64 / d, pad=B + 64 / d, sq=B, lvq=B + 64 / d),
                         ext=ext, pad=pad, sq=sq, lvq=lvq))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--d", type=int, default=256)
    ap.add_argument("--n", type=int, default=5000)
    ap.add_argument("--nq", type=int, default=50)
    a = ap.parse_args()
    print("| B | RaBitQ (ext) avg / max | RaBitQ (pad) avg / max | SQ avg / max | LVQ avg / max | LVQ / ext (avg) |")
    print("|---|---|---|---|---|---|")
    for r in table(a.d, a.n, a.nq):
        f = lambda t: "%.2e / %.2e" % t
        print("| %d | %s | %s | %s | %s | %.1f |" % (r["B"], f(r["ext"]), f(r["pad"]), f(r["sq"]), f(r["lvq"]),
                                                   r["lvq"][0] / r["ext"][0]))


if __name__ == "__main__":
    main()
