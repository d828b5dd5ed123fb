"""Host-side checks of the C ABI: the library loads, exports every symbol
that include/erq.h declares, and rejects bad arguments before any device work
(no compute call is made here; there is no GPU in this environment)."""
import ctypes as C
import os
import re

import pytest

from paper_2409_09913_amd import erq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "erq.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(erq_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("erq_rotate", "erq_quantize", "erq_coarse_probe", "erq_index_build", "erq_index_import",
                 "erq_scan", "erq_rerank", "erq_search", "erq_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = erq.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(erq.SIGNATURES), "binding and header disagree"
    assert lib.erq_version() == 200


def test_argument_validation_without_device_work():
    lib = erq.load()
    nul = None
    # dp not a multiple of 64
    assert lib.erq_rotate(nul, 0, 65, nul, 0, nul, nul) == erq.ERQ_ESHAPE
    assert b"multiple of 64" in lib.erq_last_error()
    # bits out of range
    assert lib.erq_quantize(nul, 0, 64, 9, nul, nul, nul, nul, nul, nul) == erq.ERQ_EUNSUPPORTED
    # dp above the quantiser's LDS window
    assert lib.erq_quantize(nul, 0, 4096, 4, nul, nul, nul, nul, nul, nul) == erq.ERQ_EUNSUPPORTED
    # bad precision
    assert lib.erq_rotate(nul, 0, 64, nul, 3, nul, nul) == erq.ERQ_EUNSUPPORTED
    # nprobe larger than nlist
    assert lib.erq_coarse_probe(nul, 0, nul, 4, 64, 5, 0, nul, nul, nul, 0, nul) == erq.ERQ_EUNSUPPORTED
    # null index
    assert lib.erq_scan(nul, nul, 0, nul, 1, 1, nul, nul, nul, 0, nul) == erq.ERQ_EINVAL
    assert lib.erq_rerank(nul, nul, 0, nul, 1, 1, nul, nul, nul) == erq.ERQ_EINVAL
    h = C.c_void_p()
    assert lib.erq_index_create(64, 0, 4, nul, 0, 0, nul, C.byref(h)) == erq.ERQ_EUNSUPPORTED
    assert lib.erq_index_create(64, 4, 0, nul, 0, 0, nul, C.byref(h)) == erq.ERQ_EINVAL
    assert lib.erq_index_create(64, 4, 4, nul, 0, 7, nul, C.byref(h)) == erq.ERQ_EINVAL
    # the no-allocation search checks its arguments like erq_search
    assert lib.erq_search_static(nul, nul, 1, 4, 10, 0, nul, nul, nul, nul, nul, nul) == erq.ERQ_EINVAL
    assert lib.erq_sample_rotation(65, 1, nul) == erq.ERQ_ESHAPE
    sz = C.c_size_t()
    assert lib.erq_probe_workspace_size(10, 0, 64, 1, C.byref(sz)) == erq.ERQ_EINVAL
    assert lib.erq_probe_workspace_size(10, 16, 100, 4, C.byref(sz)) == erq.ERQ_EINVAL   # dp not a multiple of 64
    assert lib.erq_probe_workspace_size(10, 16, 64, 4, C.byref(sz)) == erq.ERQ_OK and sz.value >= 10 * 16 * 4 + 26 * 64 * 4
    assert lib.erq_index_destroy(nul) == erq.ERQ_OK
