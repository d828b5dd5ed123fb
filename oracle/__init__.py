"""CPU oracle of Extended RaBitQ (arXiv 2409.09913).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The product path
(``paper_2409_09913_amd``) never imports this package, and this package never
imports the product path; the two share no code.

The arithmetic lives in ``erq_oracle.c`` (plain scalar C, FP64); this module
only marshals numpy arrays.  Every function cites the passage it follows in
the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "erq_oracle.c")
_LIB = os.path.join(_HERE, "liberq_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP across items)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        p = C.c_void_p
        i64, i32 = C.c_int64, C.c_int
        lib.orc_rotate.argtypes = [p, i64, i32, p, p]
        lib.orc_quantize_one.argtypes = [p, i32, i32, p, p, p, p]
        lib.orc_quantize_one.restype = i32
        lib.orc_objective.argtypes = [p, i32, i32, p]
        lib.orc_objective.restype = C.c_double
        lib.orc_quantize.argtypes = [p, i64, i32, i32, p, p, p, p, p]
        lib.orc_quantize.restype = i32
        lib.orc_encode.argtypes = [p, i64, i32, p, p, p, i32, p, p, p, p, p]
        lib.orc_encode.restype = i32
        lib.orc_query_quant.argtypes = [p, i32, p, p, p]
        lib.orc_query_quant2.argtypes = [p, i32, p, p, p, p, p]
        lib.orc_est_paper.argtypes = [p, i32, i32, p, C.c_double, C.c_double]
        lib.orc_est_paper.restype = C.c_double
        lib.orc_probe.argtypes = [p, i64, p, i64, i32, i32, p, p]
        lib.orc_search.argtypes = [p, p, p, p, p, p, p, i64, i32, i32,
                                   p, i64, p, i32, i32, i32, p, p]
        lib.orc_search.restype = i32
        lib.orc_search_ld.argtypes = [p, p, p, p, p, p, p, i64, i32, i32, i32,
                                      p, i64, p, i32, i32, i32, p, p]
        lib.orc_search_ld.restype = i32
        lib.orc_encode_proj.argtypes = [p, i64, i32, i32, p, p, p, i32, p, p, p]
        lib.orc_encode_proj.restype = i32
        lib.orc_rerank.argtypes = [p, i32, p, i64, p, i32, i32, p, p]
        lib.orc_search_ip.argtypes = [p, p, p, p, p, p, p, i64, i32, i32,
                                      p, i64, p, i32, i32, i32, p, p]
        lib.orc_search_ip.restype = i32
        lib.orc_probe_ip.argtypes = [p, i64, p, i64, i32, i32, p, p]
        lib.orc_rerank_ip.argtypes = [p, i32, p, i64, p, i32, i32, p, p]
        lib.orc_knn_ip.argtypes = [p, i64, i32, p, i64, i32, p, p]
        lib.orc_knn.argtypes = [p, i64, i32, p, i64, i32, p, p]
        d = C.c_double
        lib.orc_search_two_stage.argtypes = [p, p, p, p, p, p, p, i64, i32, i32,
                                             p, i64, p, i32, i32, d, p, p, p]
        lib.orc_search_two_stage.restype = i32
        lib.orc_msb_bounds.argtypes = [p, p, i64, p, p, p, p, i64, i32, i32,
                                       p, i64, p, i32, p, i32, d, p, p]
        lib.orc_msb_bounds.restype = i32
        lib.orc_num_threads.restype = i32
        lib.orc_set_threads.argtypes = [i32]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    _load().orc_set_threads(int(n))


def rotate(x, P):
    """x (n x dp) times P in FP64: the rows of P^T x (Sec. 3.4)."""
    x = _c(x, np.float64)
    P = _c(P, np.float64)
    n, dp = x.shape
    out = np.empty((n, dp), np.float64)
    _load().orc_rotate(_p(x), n, dp, _p(P), _p(out))
    return out


def quantize_one(o, B):
    """Algorithm 1 on one rotated vector. Returns (code, <y,o'>, ||y||^2, events)."""
    o = _c(o, np.float64)
    dp = o.shape[0]
    code = np.empty(dp, np.uint8)
    ip, ny, ne = C.c_double(), C.c_double(), C.c_int64()
    rc = _load().orc_quantize_one(_p(o), dp, B, _p(code), C.byref(ip), C.byref(ny), C.byref(ne))
    if rc != 0:
        raise ValueError("bad arguments to quantize_one")
    return code, ip.value, ny.value, ne.value


def objective(o, B, code):
    """<y/||y||, o'> for a stored code y_u (Eq. eq 3.2: optimization)."""
    o = _c(o, np.float64)
    code = _c(code, np.uint8)
    return float(_load().orc_objective(_p(o), o.shape[0], B, _p(code)))


def quantize(rrot, B, norm2=None):
    """Batched Algorithm 1 + factors. Returns codes, f_add, f_rescale, cos_oo (FP64)."""
    rrot = _c(rrot, np.float64)
    n, dp = rrot.shape
    codes = np.empty((n, dp), np.uint8)
    fa = np.empty(n, np.float64)
    fr = np.empty(n, np.float64)
    co = np.empty(n, np.float64)
    nr = None if norm2 is None else _c(norm2, np.float64)
    rc = _load().orc_quantize(_p(rrot), n, dp, B, None if nr is None else _p(nr),
                              _p(codes), _p(fa), _p(fr), _p(co))
    if rc != 0:
        raise ValueError("bad arguments to quantize")
    return codes, fa, fr, co


def encode(x, cent, assign, P, B):
    """Index phase (Sec. 3.4 + IVF centring): codes, f_add, f_rescale, cos_oo, r'."""
    x = _c(x, np.float64)
    cent = _c(cent, np.float64)
    assign = _c(assign, np.int32)
    P = _c(P, np.float64)
    n, dp = x.shape
    codes = np.empty((n, dp), np.uint8)
    fa = np.empty(n, np.float64)
    fr = np.empty(n, np.float64)
    co = np.empty(n, np.float64)
    rr = np.empty((n, dp), np.float64)
    rc = _load().orc_encode(_p(x), n, dp, _p(cent), _p(assign), _p(P), B,
                            _p(codes), _p(fa), _p(fr), _p(co), _p(rr))
    if rc != 0:
        raise ValueError("bad arguments to encode")
    return codes, fa, fr, co, rr


def query_quant(s):
    """int8 quantisation of one FP32 rotated residual; returns (s_int, delta, sum)."""
    s = _c(s, np.float32)
    sq = np.empty(s.shape[0], np.int8)
    d, t = C.c_float(), C.c_int32()
    _load().orc_query_quant(_p(s), s.shape[0], _p(sq), C.byref(d), C.byref(t))
    return sq, d.value, t.value


def query_quant2(s):
    """The two int8 planes of one FP32 rotated query (erq_oracle.c,
    orc_query_quant2); returns (q_hi, q_lo, delta, sum q_hi, sum q_lo)."""
    s = _c(s, np.float32)
    sh = np.empty(s.shape[0], np.int8)
    sl = np.empty(s.shape[0], np.int8)
    d, th, tl = C.c_float(), C.c_int32(), C.c_int32()
    _load().orc_query_quant2(_p(s), s.shape[0], _p(sh), _p(sl), C.byref(d), C.byref(th), C.byref(tl))
    return sh, sl, d.value, th.value, tl.value


def est_paper(code, B, s, norm_r2, cos_oo):
    """Paper-form estimate of the squared distance with a float query (FP64)."""
    code = _c(code, np.uint8)
    s = _c(s, np.float64)
    return float(_load().orc_est_paper(_p(code), code.shape[0], B, _p(s),
                                       float(norm_r2), float(cos_oo)))


def probe(q, cent, nprobe):
    """nprobe nearest centroids per query (FP64), ties by centroid id."""
    q = _c(q, np.float32)
    cent = _c(cent, np.float32)
    nq, dp = q.shape
    nc = cent.shape[0]
    pr = np.empty((nq, nprobe), np.int32)
    pd = np.empty((nq, nprobe), np.float64)
    _load().orc_probe(_p(q), nq, _p(cent), nc, dp, nprobe, _p(pr), _p(pd))
    return pr, pd


def encode_proj(x, cent, assign, P, B, dc):
    """Index phase with a random projection to dc < dp dimensions (App. C):
    codes (n x dc), f_add = ||r||^2, f_rescale = -(2 dp/dc) ||r'_d||^2/<y, r'_d>."""
    x = _c(x, np.float64)
    cent = _c(cent, np.float64)
    assign = _c(assign, np.int32)
    P = _c(P, np.float64)
    n, dp = x.shape
    codes = np.empty((n, dc), np.uint8)
    fa = np.empty(n, np.float64)
    fr = np.empty(n, np.float64)
    rc = _load().orc_encode_proj(_p(x), n, dp, dc, _p(cent), _p(assign), _p(P), B, _p(codes), _p(fa), _p(fr))
    if rc != 0:
        raise ValueError("bad arguments to encode_proj")
    return codes, fa, fr


def search(list_off, ids, codes, f_add, f_rescale, crot, qrot, probes, B, kk,
           cos_oo=None, est_mode=0):
    """IVF scan + top-kk by (est, id); est_mode 0 = int8 query (factor form),
    1 = float query (paper form, needs cos_oo), 2 = float query (factor form),
    3 = int8 query in two planes (query_quant2).
    With codes narrower than qrot / crot (the projection of App. C) the codes
    use the first coordinates and ||s||^2 all of them."""
    list_off = _c(list_off, np.int64)
    ids = _c(ids, np.int64)
    codes = _c(codes, np.uint8)
    fa = _c(f_add, np.float32)
    fr = _c(f_rescale, np.float32)
    crot = _c(crot, np.float32)
    qrot = _c(qrot, np.float32)
    probes = _c(probes, np.int32)
    co = _c(cos_oo if cos_oo is not None else np.ones(ids.shape[0]), np.float64)
    nq, ld = qrot.shape
    dp = codes.shape[1] if codes.ndim == 2 and codes.shape[0] else ld
    nprobe = probes.shape[1]
    oi = np.empty((nq, kk), np.int64)
    od = np.empty((nq, kk), np.float64)
    rc = _load().orc_search_ld(_p(list_off), _p(ids), _p(codes), _p(fa), _p(fr), _p(co),
                               _p(crot), crot.shape[0], dp, ld, B, _p(qrot), nq, _p(probes),
                               nprobe, kk, est_mode, _p(oi), _p(od))
    if rc != 0:
        raise ValueError("bad arguments to search")
    return oi, od


def rerank(x, q, cand, k):
    """Exact FP64 re-rank of candidate ids; returns (ids, squared dists)."""
    x = _c(x, np.float32)
    q = _c(q, np.float32)
    cand = _c(cand, np.int64)
    nq = q.shape[0]
    oi = np.empty((nq, k), np.int64)
    od = np.empty((nq, k), np.float64)
    _load().orc_rerank(_p(x), x.shape[1], _p(q), nq, _p(cand), cand.shape[1], k, _p(oi), _p(od))
    return oi, od


def knn(x, q, k):
    """Exact k-NN by FP64 brute force."""
    x = _c(x, np.float32)
    q = _c(q, np.float32)
    oi = np.empty((q.shape[0], k), np.int64)
    od = np.empty((q.shape[0], k), np.float64)
    _load().orc_knn(_p(x), x.shape[0], x.shape[1], _p(q), q.shape[0], k, _p(oi), _p(od))
    return oi, od


# --------------------------------------------------------------------------
# Inner-product metric: values are negated inner products, ascending.
# --------------------------------------------------------------------------
def search_two_stage(list_off, ids, codes, f_add, f_rescale, l1, crot, qrot, probes, B, kk, eps0):
    """MSB-first two-stage IVF scan of Sec. 4.2 (erq_oracle.c, orc_search_two_stage):
    the 1-bit estimate of the most significant bits with its Lemma 2.1 lower
    bound prunes a candidate when it exceeds the kk-th best full estimate so
    far; the rest get the full int8 estimate of search(est_mode=0), completed
    by Eq. 4.2.  l1: ||r'||_1 per member (list order).  Returns (ids, est,
    number of full estimates per query)."""
    list_off = _c(list_off, np.int64)
    ids = _c(ids, np.int64)
    codes = _c(codes, np.uint8)
    fa = _c(f_add, np.float32)
    fr = _c(f_rescale, np.float32)
    l1 = _c(l1, np.float64)
    crot = _c(crot, np.float32)
    qrot = _c(qrot, np.float32)
    probes = _c(probes, np.int32)
    nq, dp = qrot.shape
    nprobe = probes.shape[1]
    oi = np.empty((nq, kk), np.int64)
    od = np.empty((nq, kk), np.float64)
    nf = np.empty(nq, np.int64)
    rc = _load().orc_search_two_stage(_p(list_off), _p(ids), _p(codes), _p(fa), _p(fr), _p(l1), _p(crot),
                                      crot.shape[0], dp, B, _p(qrot), nq, _p(probes), nprobe, kk, float(eps0),
                                      _p(oi), _p(od), _p(nf))
    if rc != 0:
        raise ValueError("bad arguments to search_two_stage")
    return oi, od, nf


def msb_bounds(list_off, ids, codes, f_add, l1, crot, qrot, probes, B, cand, eps0):
    """(est1, lb) of the 1-bit stage for candidate ids cand[nq x m] (Sec. 4.2,
    Lemma 2.1; erq_oracle.c, orc_msb_bounds); +inf for ids < 0."""
    list_off = _c(list_off, np.int64)
    ids = _c(ids, np.int64)
    codes = _c(codes, np.uint8)
    fa = _c(f_add, np.float32)
    l1 = _c(l1, np.float64)
    crot = _c(crot, np.float32)
    qrot = _c(qrot, np.float32)
    probes = _c(probes, np.int32)
    cand = _c(cand, np.int64)
    nq, dp = qrot.shape
    m = cand.shape[1]
    e1 = np.empty((nq, m), np.float64)
    lb = np.empty((nq, m), np.float64)
    rc = _load().orc_msb_bounds(_p(list_off), _p(ids), ids.shape[0], _p(codes), _p(fa), _p(l1), _p(crot),
                                crot.shape[0], dp, B, _p(qrot), nq, _p(probes), probes.shape[1], _p(cand), m,
                                float(eps0), _p(e1), _p(lb))
    if rc != 0:
        raise ValueError("bad arguments to msb_bounds")
    return e1, lb


def search_ip(list_off, ids, codes, f_add, f_rescale, crot, qrot, probes, B, kk, cos_oo=None, est_mode=0):
    """IVF scan by largest estimated inner product (erq_oracle.c, orc_search_ip)."""
    list_off = _c(list_off, np.int64)
    ids = _c(ids, np.int64)
    codes = _c(codes, np.uint8)
    fa = _c(f_add, np.float32)
    fr = _c(f_rescale, np.float32)
    crot = _c(crot, np.float32)
    qrot = _c(qrot, np.float32)
    probes = _c(probes, np.int32)
    co = _c(cos_oo if cos_oo is not None else np.ones(ids.shape[0]), np.float64)
    nq, dp = qrot.shape
    nprobe = probes.shape[1]
    oi = np.empty((nq, kk), np.int64)
    od = np.empty((nq, kk), np.float64)
    rc = _load().orc_search_ip(_p(list_off), _p(ids), _p(codes), _p(fa), _p(fr), _p(co),
                               _p(crot), crot.shape[0], dp, B, _p(qrot), nq, _p(probes),
                               nprobe, kk, est_mode, _p(oi), _p(od))
    if rc != 0:
        raise ValueError("bad arguments to search_ip")
    return oi, od


def probe_ip(q, cent, nprobe):
    """nprobe centroids of largest inner product (FP64), ties by id."""
    q = _c(q, np.float32)
    cent = _c(cent, np.float32)
    nq, dp = q.shape
    pr = np.empty((nq, nprobe), np.int32)
    pd = np.empty((nq, nprobe), np.float64)
    _load().orc_probe_ip(_p(q), nq, _p(cent), cent.shape[0], dp, nprobe, _p(pr), _p(pd))
    return pr, pd


def rerank_ip(x, q, cand, k):
    x = _c(x, np.float32)
    q = _c(q, np.float32)
    cand = _c(cand, np.int64)
    nq = q.shape[0]
    oi = np.empty((nq, k), np.int64)
    od = np.empty((nq, k), np.float64)
    _load().orc_rerank_ip(_p(x), x.shape[1], _p(q), nq, _p(cand), cand.shape[1], k, _p(oi), _p(od))
    return oi, od


def knn_ip(x, q, k):
    x = _c(x, np.float32)
    q = _c(q, np.float32)
    oi = np.empty((q.shape[0], k), np.int64)
    od = np.empty((q.shape[0], k), np.float64)
    _load().orc_knn_ip(_p(x), x.shape[0], x.shape[1], _p(q), q.shape[0], k, _p(oi), _p(od))
    return oi, od
