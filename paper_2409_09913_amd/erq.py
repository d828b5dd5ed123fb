"""Thin ctypes binding of liberq.so (include/erq.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors must be contiguous CUDA(HIP) tensors of the stated dtype;
work is enqueued on torch's current stream.  If liberq.so is missing the
first call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liberq.so")

ERQ_OK, ERQ_EINVAL, ERQ_ESHAPE, ERQ_ENOMEM, ERQ_EUNSUPPORTED, ERQ_EDEVICE = range(6)
METRICS = {"l2": 0, "ip": 1, "cosine": 2}

# name -> (restype, argtypes) for every symbol of include/erq.h
_p, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
SIGNATURES = {
    "erq_last_error": (C.c_char_p, []),
    "erq_version": (C.c_int, []),
    "erq_rotate": (C.c_int, [_p, _i64, _i32, _p, _i32, _p, _p]),
    "erq_quantize": (C.c_int, [_p, _i64, _i32, _i32, _p, _p, _p, _p, _p, _p]),
    "erq_probe_workspace_size": (C.c_int, [_i64, _i64, _i32, _i32, C.POINTER(_sz)]),
    "erq_coarse_probe": (C.c_int, [_p, _i64, _p, _i64, _i32, _i32, _i32, _p, _p, _p, _sz, _p]),
    "erq_sample_rotation": (C.c_int, [_i32, C.c_uint64, _p]),
    "erq_index_create": (C.c_int, [_i32, _i32, _i64, _p, C.c_uint64, _i32, _p, C.POINTER(_p)]),
    "erq_index_destroy": (C.c_int, [_p]),
    "erq_index_set_projection": (C.c_int, [_p, _i32, _p]),
    "erq_index_set_two_stage": (C.c_int, [_p, C.c_float]),
    "erq_index_set_query_planes": (C.c_int, [_p, _i32]),
    "erq_index_set_small_batch": (C.c_int, [_p, _i32]),
    "erq_index_small_batch": (C.c_int, [_p, C.POINTER(_i32)]),
    "erq_index_code_dim": (C.c_int, [_p, C.POINTER(_i32)]),
    "erq_index_get_rotation": (C.c_int, [_p, _p, _p]),
    "erq_index_save": (C.c_int, [_p, C.c_char_p, _p]),
    "erq_index_load": (C.c_int, [C.c_char_p, _p, C.POINTER(_p)]),
    "erq_index_import": (C.c_int, [_p, _i64, _p, _p, _p, _p, _p, _p, _p, _p]),
    "erq_kmeans": (C.c_int, [_p, _i64, _i32, _i64, _i32, C.c_uint64, _p, _p, _p]),
    "erq_index_build": (C.c_int, [_p, _p, _i64, _p, _p, _i32, _i32, _p]),
    "erq_index_set_raw": (C.c_int, [_p, _p, _i64, _p]),
    "erq_index_info": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32),
                                 C.POINTER(_i64), C.POINTER(_i64)]),
    "erq_index_export": (C.c_int, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "erq_scan_workspace_size": (C.c_int, [_p, _i64, _i32, _i32, C.POINTER(_sz)]),
    "erq_scan": (C.c_int, [_p, _p, _i64, _p, _i32, _i32, _p, _p, _p, _sz, _p]),
    "erq_rerank": (C.c_int, [_p, _p, _i64, _p, _i32, _i32, _p, _p, _p]),
    "erq_search_workspace_size": (C.c_int, [_p, _i64, _i32, _i32, _i32, C.POINTER(_sz)]),
    "erq_search": (C.c_int, [_p, _p, _i64, _i32, _i32, _i32, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "erq_search_static": (C.c_int, [_p, _p, _i64, _i32, _i32, _i32, _p, _p, _p, _p, _p, _p]),
    "erq_static_scratch_bytes": (C.c_int, [C.POINTER(_sz)]),
    "erq_index_set_tune": (C.c_int, [_p, _i32, _i32, _i32, _i32]),
    "erq_index_get_tune": (C.c_int, [_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]),
    "erq_index_tune": (C.c_int, [_p, _p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p, _sz, _p,
                                 C.POINTER(_i32), C.POINTER(C.c_double)]),
    "erq_profile_enable": (C.c_int, [_i32]),
    "erq_profile_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(_i64), _i32]),
}

_lib = None


class ErqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"erq status {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Loads liberq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run `python -m paper_2409_09913_amd.build` "
                               "(there is no CPU fallback)")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != ERQ_OK:
        raise ErqError(rc, load().erq_last_error().decode())


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _ws(nbytes: int, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------
def rotate(x, P, precision: int = 0, out=None):
    """Rows of x times P (= P^T applied to each row): precision 0 FP32 matrix
    cores, 1 BF16 inputs, 2 the BF16 hi/lo three-product form of erq_search."""
    n, dp = x.shape
    if out is None:
        out = torch.empty_like(x)
    _check(load().erq_rotate(_ptr(x, torch.float32, "x"), n, dp, _ptr(P, torch.float32, "P"),
                             precision, _ptr(out, torch.float32, "out"), _stream()))
    return out


def quantize(rrot, bits: int, norm2=None):
    """Algorithm 1 on rotated rows; returns (codes uint8, f_add, f_rescale, cos_oo)."""
    n, dp = rrot.shape
    dev = rrot.device
    codes = torch.empty((n, dp), dtype=torch.uint8, device=dev)
    fa = torch.empty(n, dtype=torch.float32, device=dev)
    fr = torch.empty(n, dtype=torch.float32, device=dev)
    co = torch.empty(n, dtype=torch.float32, device=dev)
    _check(load().erq_quantize(_ptr(rrot, torch.float32, "rrot"), n, dp, bits,
                               _ptr(norm2, torch.float32, "norm2"), _ptr(codes, torch.uint8),
                               _ptr(fa), _ptr(fr), _ptr(co), _stream()))
    return codes, fa, fr, co


def coarse_probe(q, centroids, nprobe: int, with_dist: bool = False, metric: str = "l2"):
    nq, dp = q.shape
    nl = centroids.shape[0]
    sz = C.c_size_t()
    _check(load().erq_probe_workspace_size(nq, nl, q.shape[1], nprobe, C.byref(sz)))
    ws = _ws(sz.value, q.device)
    probes = torch.empty((nq, nprobe), dtype=torch.int32, device=q.device)
    pd = torch.empty((nq, nprobe), dtype=torch.float32, device=q.device) if with_dist else None
    _check(load().erq_coarse_probe(_ptr(q, torch.float32, "q"), nq, _ptr(centroids, torch.float32, "centroids"),
                                   nl, dp, nprobe, METRICS[metric], _ptr(probes), _ptr(pd), _ptr(ws), ws.numel(),
                                   _stream()))
    return (probes, pd) if with_dist else probes


def sample_rotation(dp: int, seed: int):
    """The library's Haar rotation for (dp, seed) as a host numpy array (no device work)."""
    import numpy as np
    out = np.empty((dp, dp), np.float32)
    _check(load().erq_sample_rotation(dp, seed, out.ctypes.data_as(C.c_void_p)))
    return out


def kmeans(x, nlist: int, iters: int = 10, seed: int = 240909913):
    """Lloyd k-means of the rows of x in the library (erq_kmeans); returns
    (centroids nlist x dp float32, assign int32) on x's device."""
    n, dp = x.shape
    cent = torch.empty((nlist, dp), dtype=torch.float32, device=x.device)
    asg = torch.empty(n, dtype=torch.int32, device=x.device)
    _check(load().erq_kmeans(_ptr(x, torch.float32, "x"), n, dp, nlist, iters, seed, _ptr(cent), _ptr(asg),
                             _stream()))
    return cent, asg


class Index:
    """Owner of an erq_index handle (lists, packed codes, factors, P, centroids).
    P: the dp x dp rotation (device tensor), or None to have the library
    sample it from `seed`."""

    def __init__(self, dp: int, bits: int, nlist: int, P=None, seed: int = 0, metric: str = "l2", _handle=None):
        self.dp, self.bits, self.nlist, self.metric = dp, bits, nlist, metric
        self.device = P.device if P is not None else torch.device("cuda", torch.cuda.current_device())
        if _handle is not None:
            self.h = _handle
            return
        h = C.c_void_p()
        _check(load().erq_index_create(dp, bits, nlist, _ptr(P, torch.float32, "P"), seed, METRICS[metric], _stream(),
                                       C.byref(h)))
        self.h = h

    @classmethod
    def load_file(cls, path: str):
        """An index read from a file of save()."""
        h = C.c_void_p()
        _check(load().erq_index_load(os.fsencode(path), _stream(), C.byref(h)))
        n, dp, b, nl, cb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(load().erq_index_info(h, C.byref(n), C.byref(dp), C.byref(b), C.byref(nl), C.byref(cb)))
        return cls(dp.value, b.value, nl.value, _handle=h)

    def set_projection(self, dc: int):
        """Codes of dc < dp dimensions (App. C random projection); only on an
        empty index."""
        _check(load().erq_index_set_projection(self.h, dc, _stream()))

    def set_two_stage(self, eps0: float):
        """MSB-first two-stage scan (Sec. 4.2) with the Lemma 2.1 bound at eps0;
        on an empty index it makes the build store the 1-bit data, on a
        built one it sets eps0 (0 = the one-stage scan)."""
        _check(load().erq_index_set_two_stage(self.h, float(eps0)))

    def set_query_planes(self, planes: int):
        """1: one int8 query plane; 2: a second plane of the rounding remainder
        (B >= 5), 254 times smaller query error at twice the matrix-core work."""
        _check(load().erq_index_set_query_planes(self.h, planes))

    def set_small_batch(self, max_queries: int):
        """Batches of at most max_queries queries take the scan's small-batch
        path (0 = never; default 128)."""
        _check(load().erq_index_set_small_batch(self.h, max_queries))

    def small_batch(self) -> int:
        """The current small-batch threshold."""
        v = C.c_int32()
        _check(load().erq_index_small_batch(self.h, C.byref(v)))
        return v.value

    def code_dim(self) -> int:
        dc = C.c_int32()
        _check(load().erq_index_code_dim(self.h, C.byref(dc)))
        return dc.value

    def save(self, path: str):
        _check(load().erq_index_save(self.h, os.fsencode(path), _stream()))

    def rotation(self):
        P = torch.empty((self.dp, self.dp), dtype=torch.float32, device=self.device)
        _check(load().erq_index_get_rotation(self.h, _ptr(P), _stream()))
        return P

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().erq_index_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def import_(self, list_off, ids, codes, f_add, f_rescale, centroids, centroids_rot=None):
        n = ids.shape[0]
        _check(load().erq_index_import(self.h, n, _ptr(list_off, torch.int64, "list_off"), _ptr(ids, torch.int64, "ids"),
                                       _ptr(codes, torch.uint8, "codes"), _ptr(f_add, torch.float32, "f_add"),
                                       _ptr(f_rescale, torch.float32, "f_rescale"),
                                       _ptr(centroids, torch.float32, "centroids"),
                                       _ptr(centroids_rot, torch.float32, "centroids_rot"), _stream()))

    def build(self, x, centroids=None, assign=None, precision: int = 0, keep_raw: bool = False):
        """Index phase on the device; centroids None: the library's k-means."""
        _check(load().erq_index_build(self.h, _ptr(x, torch.float32, "x"), x.shape[0],
                                      _ptr(centroids, torch.float32, "centroids"),
                                      _ptr(assign, torch.int32, "assign"), precision, int(keep_raw), _stream()))

    def set_raw(self, x):
        _check(load().erq_index_set_raw(self.h, _ptr(x, torch.float32, "x"), x.shape[0], _stream()))

    def info(self):
        n, dp, b, nl, cb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(load().erq_index_info(self.h, C.byref(n), C.byref(dp), C.byref(b), C.byref(nl), C.byref(cb)))
        return dict(n=n.value, dp=dp.value, bits=b.value, nlist=nl.value, code_bytes=cb.value)

    def export(self):
        inf = self.info()
        n, dp, nl = inf["n"], inf["dp"], inf["nlist"]
        dev = self.device
        off = torch.empty(nl + 1, dtype=torch.int64, device=dev)
        ids = torch.empty(n, dtype=torch.int64, device=dev)
        codes = torch.empty((n, self.code_dim()), dtype=torch.uint8, device=dev)
        fa = torch.empty(n, dtype=torch.float32, device=dev)
        fr = torch.empty(n, dtype=torch.float32, device=dev)
        cr = torch.empty((nl, dp), dtype=torch.float32, device=dev)
        _check(load().erq_index_export(self.h, _ptr(off), _ptr(ids), _ptr(codes), _ptr(fa), _ptr(fr), _ptr(cr),
                                       _stream()))
        return off, ids, codes, fa, fr, cr

    def scan_workspace_size(self, nq, nprobe, kk):
        sz = C.c_size_t()
        _check(load().erq_scan_workspace_size(self.h, nq, nprobe, kk, C.byref(sz)))
        return sz.value

    def scan(self, qrot, probes, kk: int, ws=None):
        nq = qrot.shape[0]
        nprobe = probes.shape[1]
        if ws is None:
            ws = _ws(self.scan_workspace_size(nq, nprobe, kk), qrot.device)
        ids = torch.empty((nq, kk), dtype=torch.int64, device=qrot.device)
        est = torch.empty((nq, kk), dtype=torch.float32, device=qrot.device)
        _check(load().erq_scan(self.h, _ptr(qrot, torch.float32, "qrot"), nq, _ptr(probes, torch.int32, "probes"),
                               nprobe, kk, _ptr(ids), _ptr(est), _ptr(ws), ws.numel(), _stream()))
        return ids, est

    def rerank(self, q, cand, k: int):
        nq, kc = cand.shape
        ids = torch.empty((nq, k), dtype=torch.int64, device=q.device)
        d = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        _check(load().erq_rerank(self.h, _ptr(q, torch.float32, "q"), nq, _ptr(cand, torch.int64, "cand"), kc, k,
                                 _ptr(ids), _ptr(d), _stream()))
        return ids, d

    def search_workspace_size(self, nq, nprobe, k, rerank_k=0):
        sz = C.c_size_t()
        _check(load().erq_search_workspace_size(self.h, nq, nprobe, k, rerank_k, C.byref(sz)))
        return sz.value

    def search(self, q, nprobe: int, k: int, rerank_k: int = 0, ws=None, out=None,
               nprobe_q=None, k_q=None, rerank_q=None):
        """k-NN of the rows of q.  nprobe, k, rerank_k are the batch's largest
        values; nprobe_q, k_q, rerank_q (int32 device tensors of nq, optional)
        give each query its own (see erq_search)."""
        nq = q.shape[0]
        if ws is None:
            ws = _ws(self.search_workspace_size(nq, nprobe, k, rerank_k), q.device)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int64, device=q.device),
                   torch.empty((nq, k), dtype=torch.float32, device=q.device))
        ids, d = out
        _check(load().erq_search(self.h, _ptr(q, torch.float32, "q"), nq, nprobe, k, rerank_k,
                                 _ptr(nprobe_q, torch.int32, "nprobe_q"), _ptr(k_q, torch.int32, "k_q"),
                                 _ptr(rerank_q, torch.int32, "rerank_q"), _ptr(ids), _ptr(d),
                                 _ptr(ws), ws.numel(), _stream()))
        return ids, d


    def search_static(self, q, nprobe: int, k: int, rerank_k: int = 0, out=None, nprobe_q=None, k_q=None,
                      rerank_q=None):
        """erq_search on the library's static device scratch (no workspace, no
        allocation in the library; the outputs are allocated here unless given)."""
        nq = q.shape[0]
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int64, device=q.device),
                   torch.empty((nq, k), dtype=torch.float32, device=q.device))
        ids, d = out
        _check(load().erq_search_static(self.h, _ptr(q, torch.float32, "q"), nq, nprobe, k, rerank_k,
                                        _ptr(nprobe_q, torch.int32, "nprobe_q"), _ptr(k_q, torch.int32, "k_q"),
                                        _ptr(rerank_q, torch.int32, "rerank_q"), _ptr(ids), _ptr(d), _stream()))
        return ids, d

    def set_tune(self, nqt: int = 0, pd: int = 0, round1: int = 0, round2: int = 0):
        """Scan schedule (0 = built-in rule for that knob)."""
        _check(load().erq_index_set_tune(self.h, nqt, pd, round1, round2))

    def get_tune(self):
        a, b, c, d = _i32(), _i32(), _i32(), _i32()
        _check(load().erq_index_get_tune(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"nqt": a.value, "pd": b.value, "round1": c.value, "round2": d.value}

    def tune(self, q, nprobe: int, k: int, rerank_k: int = 0, reps: int = 2, ws=None, out=None):
        """Times every valid scan schedule on these queries and keeps the fastest;
        returns {"nqt", "pd", "round1", "round2", "ms"}."""
        nq = q.shape[0]
        if ws is None:
            ws = _ws(self.search_workspace_size(nq, nprobe, k, rerank_k), q.device)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int64, device=q.device),
                   torch.empty((nq, k), dtype=torch.float32, device=q.device))
        ch = (_i32 * 4)()
        ms = C.c_double()
        _check(load().erq_index_tune(self.h, _ptr(q, torch.float32, "q"), nq, nprobe, k, rerank_k, reps,
                                     _ptr(out[0]), _ptr(out[1]), _ptr(ws), ws.numel(), _stream(), ch, C.byref(ms)))
        return {"nqt": ch[0], "pd": ch[1], "round1": ch[2], "round2": ch[3], "ms": ms.value}


def static_scratch_bytes() -> int:
    """Size of the library's static device scratch used by erq_search_static."""
    sz = C.c_size_t()
    _check(load().erq_static_scratch_bytes(C.byref(sz)))
    return sz.value


def profile_enable(on=True):
    """Bracket the library's kernels with HIP events on their launch stream
    (2: also count the pairs re-scanned in pass C, synchronising per scan)."""
    _check(load().erq_profile_enable(int(on)))


def profile_read(kernel: str, reset: bool = False):
    """(total milliseconds, launches) recorded for one kernel since the last reset."""
    ms, n = C.c_double(), C.c_int64()
    _check(load().erq_profile_read(kernel.encode(), C.byref(ms), C.byref(n), int(reset)))
    return ms.value, n.value
