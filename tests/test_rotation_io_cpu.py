"""Host-side pieces of the library, on the CPU (no device work):

* erq_sample_rotation, the random orthogonal matrix of Sec. 3.2.1: it is
  orthogonal, deterministic in the seed, and Haar distributed.  The Haar
  checks use moments that any other sampler would miss: for a Haar
  orthogonal n x n matrix Q (n >= 2) the trace has mean 0 and variance 1
  (Diaconis and Shahshahani), det Q = +1 with probability 1/2, and an entry
  has E[Q_ij^2] = 1/n and E[Q_ij^4] = 3/(n(n+2)) (a coordinate of a uniform
  unit vector).  Leaving out the sign fix of the QR factor breaks the trace
  and determinant moments.
* erq_index_load rejects files that are not index files, of another version,
  or whose size does not match their header, before touching a device.
"""
import ctypes as C
import os
import struct

import numpy as np
import pytest

from paper_2409_09913_amd import erq


@pytest.mark.parametrize("dp", [64, 128, 768])
def test_sampled_rotation_is_orthogonal_and_deterministic(dp):
    P = erq.sample_rotation(dp, 7)
    E = P.astype(np.float64).T @ P.astype(np.float64) - np.eye(dp)
    assert np.abs(E).max() <= 2e-6
    assert np.array_equal(P, erq.sample_rotation(dp, 7))
    assert not np.array_equal(P, erq.sample_rotation(dp, 8))


def test_sampled_rotation_is_haar():
    M = 3000
    tr, det = np.empty(M), np.empty(M)
    q11 = np.empty(M)
    for s in range(M):
        Q = erq.sample_rotation(64, 5000 + s).astype(np.float64)
        tr[s] = np.trace(Q)
        det[s] = np.sign(np.linalg.det(Q))
        q11[s] = Q[3, 5]
    nn = 64
    assert abs(tr.mean()) <= 4.0 / np.sqrt(M)
    assert abs(tr.var() - 1.0) <= 0.15
    assert abs((det > 0).mean() - 0.5) <= 4 * 0.5 / np.sqrt(M)
    assert abs((q11 ** 2).mean() - 1.0 / nn) <= 4 * np.sqrt(2.0) / nn / np.sqrt(M)
    m4 = 3.0 / (nn * (nn + 2))
    assert abs((q11 ** 4).mean() - m4) <= 0.25 * m4


def _lib():
    return erq.load()


def test_load_rejects_bad_files(tmp_path):
    lib = _lib()
    h = C.c_void_p()
    assert lib.erq_index_load(os.fsencode(str(tmp_path / "missing.idx")), None, C.byref(h)) == erq.ERQ_EINVAL
    p = tmp_path / "junk.idx"
    p.write_bytes(b"not an index file at all" * 10)
    assert lib.erq_index_load(os.fsencode(str(p)), None, C.byref(h)) == erq.ERQ_EINVAL
    # a well-formed header of version 1 whose arrays are missing: size mismatch
    # (version, dp, bits, has_raw, metric, code dimension), (nlist, n, tiles), schedule, seed
    # ..., schedule, seed, (two-stage flag, eps0), (query planes, small-batch threshold)
    hdr = b"ERQIDX\0\0" + struct.pack("<Iiiiii", 2, 64, 4, 0, 0, 64) + struct.pack("<qqq", 2, 10, 2) + \
        struct.pack("<iiii", 0, 0, 0, 0) + struct.pack("<Q", 0) + struct.pack("<if", 0, 0.0) + struct.pack("<ii", 1, 32)
    p2 = tmp_path / "short.idx"
    p2.write_bytes(hdr)
    assert lib.erq_index_load(os.fsencode(str(p2)), None, C.byref(h)) == erq.ERQ_EINVAL
    assert b"size" in lib.erq_last_error()
    for tail in (struct.pack("<if", 2, 0.0), struct.pack("<if", 1, -1.0)):   # bad two-stage flag, eps0
        pb = tmp_path / "ts.idx"
        pb.write_bytes(hdr[:80] + tail + hdr[88:])
        assert lib.erq_index_load(os.fsencode(str(pb)), None, C.byref(h)) == erq.ERQ_EINVAL
        assert b"bad header" in lib.erq_last_error()
    for planes in (0, 3, 2):            # bad query planes; 2 with B = 4
        pb = tmp_path / "qp.idx"
        pb.write_bytes(hdr[:88] + struct.pack("<ii", planes, 32))
        assert lib.erq_index_load(os.fsencode(str(pb)), None, C.byref(h)) == erq.ERQ_EINVAL
        assert b"bad header" in lib.erq_last_error()
    for dc in (0, 32, 96, 128):        # code dimension not a multiple of 64 in [64, dp]
        pb = tmp_path / f"dc{dc}.idx"
        pb.write_bytes(hdr[:28] + struct.pack("<i", dc) + hdr[32:])
        assert lib.erq_index_load(os.fsencode(str(pb)), None, C.byref(h)) == erq.ERQ_EINVAL
        assert b"bad header" in lib.erq_last_error()
    p3 = tmp_path / "v9.idx"
    p3.write_bytes(b"ERQIDX\0\0" + struct.pack("<Iiiiii", 9, 64, 4, 0, 0, 64) + hdr[32:])
    assert lib.erq_index_load(os.fsencode(str(p3)), None, C.byref(h)) == erq.ERQ_EUNSUPPORTED
