"""Space-accuracy comparison of Sec. 5.2.1 on synthetic data (CPU only):
RaBitQ (ext) against SQ, LVQ and RaBitQ (pad) (Sec. 5.1, algorithms (2)-(4),
in oracle/comparators.py).  The checks are the paper's findings: at every B
the extended method's average relative error is below LVQ's, which is below
SQ's; at B = 1 and 2 SQ and LVQ are worse by an order of magnitude or more;
RaBitQ (pad) is close at B = 1 but decays like 1/sqrt(B), while the
extended method's error decays exponentially in B."""
import numpy as np

from oracle import space_accuracy


def test_space_accuracy_findings():
    rows = {r["B"]: r for r in space_accuracy.table(d=256, n=2000, nq=20)}
    for B, r in rows.items():
        assert r["ext"][0] < r["lvq"][0] < r["sq"][0], (B, r)
    for B in (1, 2):
        assert rows[B]["lvq"][0] > 10 * rows[B]["ext"][0]
        assert rows[B]["sq"][0] > 10 * rows[B]["ext"][0]
    assert rows[1]["pad"][0] < 1.5 * rows[1]["ext"][0]
    # (pad): O(1/sqrt(B D)); (ext): about 2^-B
    assert rows[8]["pad"][0] / rows[1]["pad"][0] > 0.8 / np.sqrt(8)
    assert rows[8]["ext"][0] / rows[1]["ext"][0] < 4 * 2.0 ** -7
    for B in range(2, 9):
        assert 1.5 < rows[B - 1]["ext"][0] / rows[B]["ext"][0] < 2.6
