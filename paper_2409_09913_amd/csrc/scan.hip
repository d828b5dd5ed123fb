// IVF scan of Extended RaBitQ codes on the int8 matrix cores (Sec. 3.3,
// Sec. 4.1).  Every rotated query q' is quantised to int8 once
// (symmetric, delta = max|q'|/127, q_int = rint(q' / delta)).  For a probed
// list with rotated centroid c' the residual is s' = q' - c', and by
// linearity <y_bar, s'> = <y_bar, q'> - <y_bar, c'>, where the list term is
// folded into the member's factor g_add = f_add - f_rescale <y_bar, c'>.  The
// estimated squared distance of a member is then
//     est = g_add + ||s'||^2 + f_rescale * delta/2 * (2 <y_u, q_int> - (2^B - 1) sum q_int)
// (Eq. eq:dis to ip with Eq. eq 3.3: represent), with <y_u, q_int>
// accumulated exactly in int32 by v_mfma_i32_32x32x32_i8.  The kk smallest
// (est, id) per query are returned.  One query batch runs as:
//
//  1. pair build: (query, probe) pairs grouped by list (count, scan,
//     scatter) for a range of probe ranks; work items are (list, tile of its
//     queries[, chunk of kVch members]), longest list first.
//  2. first bound: every estimate of the first kDenseV members of the kDenseR
//     nearest probed lists is written to fixed slots of the query's
//     candidate buffer; tau_q is the kk-th best of them (radix select).  Any
//     subset of a query's candidates gives a valid bound: every member of the
//     final top-kk has est <= tau_q.  The buffer keeps those estimates at
//     or under tau_q, and the first round skips the members they cover.
//  3. pass B (the scan) in rounds of probe rank, [0, round1) and the rest
//     (cut further when kk * nprobe is large against a candidate buffer):
//     64 vectors x 32 or 64 queries per wave step.  Estimates above tau_q are
//     dropped with one compare; the rest are staged in a per-query LDS
//     buffer (spilling straight to global memory when it is full) and
//     appended to the query's candidate buffer in HBM.  A query whose buffer
//     overflowed in a round gets back the count it had before the round,
//     tau_q drops to the kk-th best of its kCapQ stored candidates, and the
//     round's pairs of those queries are scanned again.  After a round tau_q
//     drops to the kk-th best candidate so far.
//  4. select: per query, the exact kk smallest (est, id) of its candidates.
//  5. fallback: a query whose buffer still overflowed is scanned again in
//     full by one workgroup that keeps its exact top-kk in LDS.
#include <algorithm>
#include <type_traits>

#include "erq_common.h"

namespace erq {

namespace {

constexpr int kThreads = 256;
constexpr int kQT = 32;        // queries per MFMA column tile
constexpr int kCapB = 32;      // per-query survivor buffer of a pass-B item (LDS)
constexpr int kDenseR = 4;     // first bound: nearest probes per query ...
constexpr int kDenseV = 256;   // ... and members per list (all estimates kept)
constexpr int kRound1 = 4;     // pass B: the rounds up to probe rank kRound1 (the first is [0, kDenseR))
constexpr int kCapQ = 4096;    // candidate buffer per query (HBM)
constexpr int kVch = 1024;     // pass-B members per item (long lists are split)
constexpr int kSmallS = 64;    // small-batch path: at most this many workgroups per query

__device__ inline unsigned f2key(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key2f(unsigned k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
__device__ inline bool lt(float e0, int i0, float e1, int i1) { return e0 < e1 || (e0 == e1 && i0 < i1); }

struct PartsC { int n; int w[3]; int pos[3]; };
template <int BITS>
__device__ constexpr PartsC parts_c() {
    if (BITS == 1) return PartsC{1, {1, 0, 0}, {0, 0, 0}};
    if (BITS == 2) return PartsC{1, {2, 0, 0}, {0, 0, 0}};
    if (BITS == 3) return PartsC{2, {2, 1, 0}, {0, 2, 0}};
    if (BITS == 4) return PartsC{1, {4, 0, 0}, {0, 0, 0}};
    if (BITS == 5) return PartsC{2, {4, 1, 0}, {0, 4, 0}};
    if (BITS == 6) return PartsC{2, {4, 2, 0}, {0, 4, 0}};
    if (BITS == 7) return PartsC{3, {4, 2, 1}, {0, 4, 6}};
    return PartsC{1, {8, 0, 0}, {0, 0, 0}};
}

template <int W>
__device__ inline void load_part(const uint8_t* p, uint32_t* X) {
    if (W == 8) {
        uint4 a = *(const uint4*)p, b = *(const uint4*)(p + 16);
        X[0] = a.x; X[1] = a.y; X[2] = a.z; X[3] = a.w; X[4] = b.x; X[5] = b.y; X[6] = b.z; X[7] = b.w;
    } else if (W == 4) {
        uint4 a = *(const uint4*)p;
        X[0] = a.x; X[1] = a.y; X[2] = a.z; X[3] = a.w;
    } else if (W == 2) {
        uint2 a = *(const uint2*)p;
        X[0] = a.x; X[1] = a.y;
    } else {
        X[0] = *(const uint32_t*)p;
    }
}

template <int W, int POS>
__device__ inline void unpack_part(const uint32_t* X, uint32_t* U) {
    constexpr int per = 8 / W;
    constexpr uint32_t mask = 0x01010101u * ((1u << W) - 1u);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint32_t v = (W == 8) ? X[c] : ((X[c / per] >> ((c % per) * W)) & mask);
        U[c] |= (POS == 0) ? v : (v << POS);
    }
}

// codes of one K-block (64 dims) for this lane -> two int8x16 A fragments
template <int BITS>
__device__ inline void load_codes(const uint8_t* kb, int lane, v4i& a0, v4i& a1) {
    constexpr PartsC P = parts_c<BITS>();
    uint32_t U[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t X[8];
    load_part<P.w[0]>(kb + lane * 4 * P.w[0], X);
    unpack_part<P.w[0], P.pos[0]>(X, U);
    if constexpr (P.n > 1) {
        load_part<P.w[1]>(kb + P.w[0] * 256 + lane * 4 * P.w[1], X);
        unpack_part<P.w[1], P.pos[1]>(X, U);
    }
    if constexpr (P.n > 2) {
        load_part<P.w[2]>(kb + (P.w[0] + P.w[1]) * 256 + lane * 4 * P.w[2], X);
        unpack_part<P.w[2], P.pos[2]>(X, U);
    }
    a0 = v4i{(int)U[0], (int)U[1], (int)U[2], (int)U[3]};
    a1 = v4i{(int)U[4], (int)U[5], (int)U[6], (int)U[7]};
}

// raw packed words of one K-block (64 dims) of a tile for this lane: BITS dwords
template <int BITS>
__device__ inline void load_raw(const uint8_t* kbp, int lane, uint32_t* d) {
    constexpr PartsC P = parts_c<BITS>();
    load_part<P.w[0]>(kbp + lane * 4 * P.w[0], d);
    if constexpr (P.n > 1) load_part<P.w[1]>(kbp + P.w[0] * 256 + lane * 4 * P.w[1], d + P.w[0]);
    if constexpr (P.n > 2)
        load_part<P.w[2]>(kbp + (P.w[0] + P.w[1]) * 256 + lane * 4 * P.w[2], d + P.w[0] + P.w[1]);
}

template <int BITS>
__device__ inline void unpack_raw(const uint32_t* d, v4i& a0, v4i& a1) {
    constexpr PartsC P = parts_c<BITS>();
    uint32_t U[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unpack_part<P.w[0], P.pos[0]>(d, U);
    if constexpr (P.n > 1) unpack_part<P.w[1], P.pos[1]>(d + P.w[0], U);
    if constexpr (P.n > 2) unpack_part<P.w[2], P.pos[2]>(d + P.w[0] + P.w[1], U);
    a0 = v4i{(int)U[0], (int)U[1], (int)U[2], (int)U[3]};
    a1 = v4i{(int)U[4], (int)U[5], (int)U[6], (int)U[7]};
}

__device__ inline int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Estimator epilogue of one (member, query) pair, evaluated in this order by
// every scan kernel, so that a pair's estimate is bit-identical whichever
// kernel computes it: e = f_rescale * (h2 * IP + hc) + g_add and
// est = e + ||s||^2, where f = (g_add, f_rescale) and the column constants
// are h2 = 2 * delta/2 and hc = delta/2 * corr * sum(q_int) (epi_consts).
template <int BITS>
__device__ inline void epi_consts(float hd, int ss, float& h2, float& hc) {
    constexpr int corr = 2 * (BITS == 8 ? 128 : 0) - ((1 << BITS) - 1);
    h2 = 2.0f * hd;
    hc = hd * (float)(corr * ss);
}
__device__ inline float epi_e(float2 f, int acc, float h2, float hc) {
    return __fmaf_rn(f.y, __fmaf_rn(h2, (float)acc, hc), f.x);
}
// Two query planes: IP = <y, q_hi> + <y, q_lo> / 254, so
// e = f_rescale * (h2 * IP_hi + (h2l * IP_lo + hc)) + g_add with h2l = h2 / 254
// and hc = delta/2 * corr * (sum q_hi + sum q_lo / 254).
template <int BITS>
__device__ inline void epi_consts2(float hd, int ss, int ssl, float& h2, float& h2l, float& hc) {
    constexpr int corr = 2 * (BITS == 8 ? 128 : 0) - ((1 << BITS) - 1);
    h2 = 2.0f * hd;
    h2l = __fdiv_rn(h2, 254.0f);
    hc = __fmaf_rn(__fdiv_rn(hd, 254.0f), (float)(corr * ssl), hd * (float)(corr * ss));
}
__device__ inline float epi_e2(float2 f, int ah, int al, float h2, float h2l, float hc) {
    return __fmaf_rn(f.y, __fmaf_rn(h2, (float)ah, __fmaf_rn(h2l, (float)al, hc)), f.x);
}

// Item of a pair table grouped by list: largest rank r with item_off[r] <= item.
__device__ inline void decode_item(int item, const int32_t* item_off, const int32_t* list_order, int nlist,
                                   int* l, int* t) {
    int lo = 0, hi = nlist;
    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (item_off[mid] <= item) lo = mid; else hi = mid; }
    while (lo + 1 < nlist && item_off[lo + 1] <= item) ++lo;
    *l = list_order[lo];
    *t = item - item_off[lo];
}

// Queries of a scan, prepared once per batch: q' quantised to int8 (qint,
// nq x dp), delta/2 (qhd) and the sum of the int8 values (qss) per query,
// and ||s||^2 = ||q' - c'||^2 per (query, probe) pair (sdist).
// With two query planes (large B) the low plane q_lo and its sums follow:
// q' ~= delta * (q_int + q_lo / 254).
struct QArgs {
    const int8_t* qint;
    const float* qhd;
    const int32_t* qss;
    const float* sdist;
    float s2_floor;          // 0 for L2 (a squared distance rounded below 0 is clamped), -inf otherwise
    const int8_t* qlo;       // nq x dp, or null (one plane)
    const int32_t* qss_lo;
};

// Prologue shared by the scan kernels, in two steps with a barrier between
// them.  Step 1 (threads < mq): per-query scalars of the item's pairs into
// s_* (query id, slot, ||s||^2, delta/2, sum of q_int, bound).  Step 2 (all
// threads): the int8 query rows into LDS, row-major with a row stride of
// dp + 16 bytes (query qi at qs + qi*qstride), rows past mq zero; every
// thread issues all of its 16-byte loads (up to kRowLoads) before it stores
// any, so a batch costs one memory latency.  The 16-byte pad spreads the
// B-fragment reads of the 32 columns over all LDS banks.
__device__ inline void load_query_scalars(float* s_s2, float* s_hd, int* s_ss, int* s_slot, int* s_q,
                                          unsigned* s_tau, const unsigned* __restrict__ tau_key, const QArgs& qa,
                                          const int32_t* __restrict__ pq, const int32_t* __restrict__ pslot,
                                          int mq, int tid)
{
    if (tid < mq) {
        const int q = pq[tid], slot = pslot[tid];
        s_s2[tid] = fmaxf(qa.sdist[slot], qa.s2_floor);   // L2: the probe's expanded form may round below 0
        s_hd[tid] = qa.qhd[q];
        s_ss[tid] = qa.qss[q];
        s_slot[tid] = slot;
        s_q[tid] = q;
        if (s_tau) s_tau[tid] = tau_key[q];
    }
}

constexpr int kRowLoads = 12;

// With LO (NQT = 2), rows [kQT, 2 kQT) hold the low planes of the queries of
// rows [0, kQT).
template <int NQT, bool LO = false>
__device__ inline void load_query_rows(int8_t* qs, int qstride, const int* s_q, const int8_t* __restrict__ qint,
                                       int dp, int mq, int tid, const int8_t* __restrict__ qlo = nullptr)
{
    constexpr int QPI = kQT * NQT;
    const int nch = dp >> 4;                       // 16-byte chunks per row
    const float rnch = 1.0f / (float)nch;          // u / nch below is exact: u < 2^16, gap >= 0.5/nch
    const int units = QPI * nch;
    for (int base = 0; base < units; base += kRowLoads * kThreads) {
        uint4 w[kRowLoads];
#pragma unroll
        for (int k = 0; k < kRowLoads; ++k) {
            const int u = base + k * kThreads + tid;
            const int qi = (int)(((float)u + 0.5f) * rnch);
            const int c = u - qi * nch;
            w[k] = make_uint4(0, 0, 0, 0);
            if constexpr (LO) {
                const int qq = qi < kQT ? qi : qi - kQT;
                if (u < units && qq < mq)
                    w[k] = *(const uint4*)((qi < kQT ? qint : qlo) + (int64_t)s_q[qq] * dp + 16 * c);
            } else {
                if (u < units && qi < mq) w[k] = *(const uint4*)(qint + (int64_t)s_q[qi] * dp + 16 * c);
            }
        }
#pragma unroll
        for (int k = 0; k < kRowLoads; ++k) {
            const int u = base + k * kThreads + tid;
            const int qi = (int)(((float)u + 0.5f) * rnch);
            const int c = u - qi * nch;
            if (u < units) *(uint4*)(qs + qi * qstride + 16 * c) = w[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Pass B: items of 32*NQT queries; each wave step is 64 vectors (two code
// tiles) x 32*NQT queries, so every unpacked code fragment feeds 2*NQT MFMAs
// and every query fragment 2.  Estimates above the query's bound are dropped
// with one compare; survivors go to the query's candidate buffer in HBM
// (staged in LDS; straight to HBM once the LDS stage is full).
// ---------------------------------------------------------------------------
template <int BITS, int NQT, int PD, bool DENSE, bool LO>
__global__ __launch_bounds__(kThreads, 2) void scanB_kernel(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ tile_off,
    const int64_t* __restrict__ list_off, const float2* __restrict__ fac,
    const int64_t* __restrict__ ids, int dp, QArgs qa, const int32_t* __restrict__ pair_off,
    const int32_t* __restrict__ pair_q, const int32_t* __restrict__ pair_slot,
    const int32_t* __restrict__ item_off, const int4* __restrict__ desc, int nlist,
    int kk, unsigned* __restrict__ tau_key, int32_t* __restrict__ gcnt,
    float* __restrict__ gbuf_e, int32_t* __restrict__ gbuf_i, int32_t* __restrict__ work,
    int vch, int nprobe)
{
    constexpr bool dense = DENSE;
    // LO (two query planes, NQT = 2): the item holds up to kQT queries; query
    // tile 0 is their high planes, tile 1 their low planes, and the epilogue
    // combines the two accumulators of a column into one estimate.
    static_assert(!LO || NQT == 2, "two query planes use the two query tiles");
    // DENSE (first bound): only the first kDenseV members of each list,
    // no bound test, every estimate written to slot rank*kDenseV + member of
    // the query's buffer (rank = probe rank of the pair, < kDenseR)
    constexpr int QPI = kQT * NQT;
    extern __shared__ __align__(16) char smem[];
    __shared__ float s_s2[QPI], s_hd[QPI];
    __shared__ int s_ss[QPI], s_slot[QPI], s_q[QPI], s_cnt[QPI], s_base[QPI];
    __shared__ float s_be[QPI][kCapB];
    __shared__ int s_bi[QPI][kCapB];
    __shared__ unsigned s_tau[QPI];
    __shared__ float2 s_fac[kVch + 64];      // + NaN padding up to the group end
    __shared__ int s_id[kVch + 64];          // ids of the item's members (no global load in the epilogue)
    __shared__ int s_item[5];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar
    const int n_items = item_off[nlist];
    // Items are taken from a shared counter until it passes n_items; the id of
    // the next item is fetched while the current one is scanned.
    if (tid == 0) s_item[4] = atomicAdd(work, 1);
    __syncthreads();
    for (;;) {
    const int item = s_item[4];
    if (item >= n_items) break;
    if (tid == 0) {
        const int4 d = desc[item];
        s_item[0] = d.x; s_item[1] = d.y; s_item[2] = d.z; s_item[3] = d.w;
    }
    if (tid < QPI) s_cnt[tid] = 0;
    __syncthreads();
    if (tid == 0) s_item[4] = atomicAdd(work, 1);  // read again only after the item's last barrier
    const int l = s_item[0], p0 = s_item[1], mq = s_item[2], v0 = s_item[3];
    int8_t* qs = (int8_t*)smem;
    const int qstride = dp + 16;
    load_query_scalars(s_s2, s_hd, s_ss, s_slot, s_q, s_tau, tau_key, qa, pair_q + p0, pair_slot + p0, mq, tid);
    {   // factors and ids of the item's members, all loads of a thread in
        // flight at once; past the end NaN, which never passes
        constexpr int KF = (kVch + 64 + kThreads - 1) / kThreads;
        const int64_t fb = list_off[l] + v0;
        const int nf = min((int)(list_off[l + 1] - list_off[l]) - v0, dense ? kDenseV : kVch);
        const int nfp = (nf + 63) & ~63;
        float2 fv[KF];
        int iv[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int t = tid + k * kThreads;
            const bool in = t < nf;
            fv[k] = in ? fac[fb + t] : make_float2(__builtin_nanf(""), 0.0f);
            iv[k] = in ? (int)ids[fb + t] : -1;
        }
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int t = tid + k * kThreads;
            if (t < nfp) { s_fac[t] = fv[k]; s_id[t] = iv[k]; }
        }
    }
    __syncthreads();
    load_query_rows<NQT, LO>(qs, qstride, s_q, qa.qint, dp, mq, tid, qa.qlo);
    __syncthreads();

    const int nkb = dp / 64;
    // B fragment of lane (h = lane/32, j = lane%32) for query tile qt: query
    // qt*32 + j, bytes 16h.. of each 32-dim block
    const int8_t* qrow = qs + (lane & 31) * qstride + 16 * (lane >> 5);
    const int64_t tile_bytes = (int64_t)4 * dp * BITS;
    // members [v0, v0 + nl) of list l (v0 is a multiple of 64: whole tile pairs)
    const int nl = min((int)(list_off[l + 1] - list_off[l]) - v0, dense ? kDenseV : kVch);
    const int ntile = (nl + 31) >> 5;
    const int64_t tbase = tile_off[l] + (v0 >> 5);
    const int j = lane & 31;
    // Columns without a query (qi >= mq) have no LDS terms: they take zeros
    // and are excluded from the pass test by qok, not by their estimate.
    float qs2[NQT], qhd[NQT], qtau[NQT];
    int qss[NQT];
    bool qok[NQT];
#pragma unroll
    for (int qt = 0; qt < NQT; ++qt) {
        const int qi = LO ? j : qt * kQT + j;         // LO: both tiles are query j
        qok[qt] = qi < mq;
        qs2[qt] = qok[qt] ? s_s2[qi] : 0.0f;
        qhd[qt] = qok[qt] ? s_hd[qi] : 0.0f;
        qss[qt] = qok[qt] ? s_ss[qi] : 0;
        qtau[qt] = qok[qt] ? key2f(s_tau[qi]) : 0.0f;
    }
    // Epilogue constants per column: est = (g + fr * (H2 * acc + HC)) + s2 with
    // H2 = 2 delta/2 and HC = delta/2 * corr * sum(q_int); the bound test
    // compares the part before + s2 with AQ = tau - s2 rounded up by a margin
    // above the rounding of both subtractions, so it never drops a candidate
    // whose final estimate is <= tau.  Columns without a query take AQ = -inf.
    float cH2[NQT], cHC[NQT], cAQ[NQT], cH2L = 0.0f;
#pragma unroll
    for (int qt = 0; qt < NQT; ++qt) {
        epi_consts<BITS>(qhd[qt], qss[qt], cH2[qt], cHC[qt]);
        const float aq = qtau[qt] - qs2[qt];
        cAQ[qt] = qok[qt] ? aq + (fabsf(qtau[qt]) + fabsf(qs2[qt])) * 0x1p-20f : -__builtin_huge_valf();
    }
    if constexpr (LO)
        epi_consts2<BITS>(qhd[0], qss[0], qok[0] ? qa.qss_lo[s_q[j]] : 0, cH2[0], cH2L, cHC[0]);

    // Wave wid takes the tiles [ta, tb) of the item (a contiguous quarter,
    // so the waves differ by at most one tile) and walks them in groups of
    // two tiles as one sequence of K-steps (group, kb); a group with one tile
    // (the last of an odd range) skips the second tile's unpacking and
    // MFMAs behind a wave-uniform branch.
    // The packed codes of step s + PD are loaded while step s runs: a ring
    // of PD slots of raw words in registers, unrolled by PD so that each slot
    // is consumed and refilled in place (no copy of a register whose load is
    // in flight).  PD divides nkb, so a group always ends with the last slot.
    // Past the end the last step is loaded again, so no load is conditional.
    const int ta = (wid * ntile) >> 2, tb = ((wid + 1) * ntile) >> 2;
    const int ngw = (tb - ta + 1) >> 1;
    const int total = ngw * nkb;
    if (total > 0) {
        uint32_t ring[PD][2 * BITS];
        // next step to load: group tile t0 at p0 (second tile p0 + d1, or p0
        // itself for a single-tile group), K-block offset koff
        int t0 = ta, pleft = total;
        const uint8_t* p0 = codes + (tbase + t0) * tile_bytes;
        int64_t d1 = (t0 + 1 < tb) ? tile_bytes : 0;
        int64_t koff = 0;
        auto load_step = [&](uint32_t* d) {
            load_raw<BITS>(p0 + koff, lane, d);
            load_raw<BITS>(p0 + d1 + koff, lane, d + BITS);
            if (pleft > 1) {
                --pleft;
                koff += 256 * BITS;
                if (koff == tile_bytes) {
                    koff = 0;
                    t0 += 2;
                    p0 += 2 * tile_bytes;
                    d1 = (t0 + 1 < tb) ? tile_bytes : 0;
                }
            }
        };
#pragma unroll
        for (int p = 0; p < PD; ++p) load_step(ring[p]);
        // query fragments of K-block kb (they do not depend on the group):
        // those of the next K-block are read from LDS while this one's MFMAs run
        auto read_b = [&](int kb, v4i (&b)[NQT][2]) {
#pragma unroll
            for (int qt = 0; qt < NQT; ++qt) {
                b[qt][0] = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb);
                b[qt][1] = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb + 32);
            }
        };
        v4i bq[NQT][2];
        read_b(0, bq);
        v16i acc[2][NQT];
        // code x query products of a K-block; the first bound takes the
        // transposed product (rows queries, columns members) so that its
        // per-(query, member) stores run along members, 128 contiguous bytes
        // per half-wave
        auto mm = [](const v4i& a, const v4i& b, const v16i& c) -> v16i {
            if constexpr (DENSE) return __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c, 0, 0, 0);
            else return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
        };
        // the nkb K-steps of one group, for a group of two tiles or of one
        // (the width is a compile-time constant of each loop body)
        auto run_group = [&](auto two_c) {
            constexpr bool TWO = decltype(two_c)::value;
#pragma unroll
            for (int a = 0; a < (TWO ? 2 : 1); ++a)
#pragma unroll
                for (int qt = 0; qt < NQT; ++qt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[a][qt][r] = 0;
            for (int kb0 = 0; kb0 < nkb; kb0 += PD) {
#pragma unroll
                for (int p = 0; p < PD; ++p) {
                    v4i a00, a01, a10, a11;
                    unpack_raw<BITS>(ring[p], a00, a01);
                    if constexpr (TWO) unpack_raw<BITS>(ring[p] + BITS, a10, a11);
                    load_step(ring[p]);
                    const int kb = kb0 + p;
                    v4i bn[NQT][2];
                    read_b(kb + 1 < nkb ? kb + 1 : 0, bn);
#pragma unroll
                    for (int qt = 0; qt < NQT; ++qt) {
                        acc[0][qt] = mm(a00, bq[qt][0], acc[0][qt]);
                        if constexpr (TWO) acc[1][qt] = mm(a10, bq[qt][0], acc[1][qt]);
                    }
#pragma unroll
                    for (int qt = 0; qt < NQT; ++qt) {
                        acc[0][qt] = mm(a01, bq[qt][1], acc[0][qt]);
                        if constexpr (TWO) acc[1][qt] = mm(a11, bq[qt][1], acc[1][qt]);
                    }
#pragma unroll
                    for (int qt = 0; qt < NQT; ++qt) { bq[qt][0] = bn[qt][0]; bq[qt][1] = bn[qt][1]; }
                }
            }
        };
        for (int gi = 0; gi < ngw; ++gi) {
            const int gt0 = ta + 2 * gi;                // first tile of the group
            if (gt0 + 1 < tb) run_group(std::true_type{});
            else run_group(std::false_type{});
            // epilogue of group g: estimates, bound test, survivors to the stage.
            // The tile's 16 factor pairs are read from LDS before any is used,
            // and nothing here touches global memory except the rare overflow
            // of the stage, so the code loads in flight for the next group are
            // not waited for.
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int tt = gt0 + a;
                if (tt >= tb) break;
                if constexpr (DENSE) {
                    // first bound, transposed tile: this lane's member is
                    // tt*32 + j, row r of query tile qt is query
                    // qt*32 + out_row(lane, r); every estimate is kept, in the
                    // same arithmetic as the bounded scan's
                    const int v = tt * 32 + j;
                    const float2 f = s_fac[v];
                    const int id = s_id[v];
                    if (v < nl) {
#pragma unroll
                        for (int qt = 0; qt < (LO ? 1 : NQT); ++qt) {
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                const int qi = qt * kQT + out_row(lane, r);
                                if (qi >= mq) continue;
                                float h2, hc, e;
                                if constexpr (LO) {
                                    float h2l;
                                    epi_consts2<BITS>(s_hd[qi], s_ss[qi], qa.qss_lo[s_q[qi]], h2, h2l, hc);
                                    e = epi_e2(f, acc[a][0][r], acc[a][1][r], h2, h2l, hc);
                                } else {
                                    epi_consts<BITS>(s_hd[qi], s_ss[qi], h2, hc);
                                    e = epi_e(f, acc[a][qt][r], h2, hc);
                                }
                                const int q = s_q[qi];
                                const int64_t sl = (int64_t)q * kCapQ + (int64_t)(s_slot[qi] - q * nprobe) * kDenseV;
                                gbuf_e[sl + v] = e + s_s2[qi];
                                gbuf_i[sl + v] = id;
                            }
                        }
                    }
                    continue;
                }
                float2 fr[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) fr[r] = s_fac[tt * 32 + out_row(lane, r)];   // NaN past the end
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int v = tt * 32 + out_row(lane, r);
                    const float2 f = fr[r];
                    float e[NQT];
                    bool pass[NQT], anyp = false;
                    if constexpr (LO) {                     // one estimate from the two planes
                        e[0] = epi_e2(f, acc[a][0][r], acc[a][1][r], cH2[0], cH2L, cHC[0]);
                        pass[0] = e[0] <= cAQ[0];
                        pass[1] = false;
                        e[1] = 0.0f;
                        anyp = pass[0];
                    } else {
#pragma unroll
                        for (int qt = 0; qt < NQT; ++qt) {
                            e[qt] = epi_e(f, acc[a][qt][r], cH2[qt], cHC[qt]);
                            pass[qt] = e[qt] <= cAQ[qt];
                            anyp = anyp || pass[qt];
                        }
                    }
                    if (!__any(anyp)) continue;
#pragma unroll
                    for (int qt = 0; qt < (LO ? 1 : NQT); ++qt) {
                        if (!pass[qt]) continue;
                        const float est = e[qt] + qs2[qt];
                        const int qi = qt * kQT + j;
                        const int id = s_id[v];
                        const int pos = atomicAdd(&s_cnt[qi], 1);
                        if (pos < kCapB) {
                            s_be[qi][pos] = est; s_bi[qi][pos] = id;
                        } else {                            // stage full: straight to HBM
                            const int q = s_q[qi];
                            const int gp = atomicAdd(&gcnt[q], 1);
                            if (gp < kCapQ) {
                                gbuf_e[(int64_t)q * kCapQ + gp] = est;
                                gbuf_i[(int64_t)q * kCapQ + gp] = id;
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // flush the LDS stage to the query's candidate buffer
    const int qi = tid >> 2, sub = tid & 3;
    if (qi < mq && sub == 0) {
        const int m = min(s_cnt[qi], kCapB);
        s_base[qi] = (m > 0) ? atomicAdd(&gcnt[s_q[qi]], m) : 0;
    }
    __syncthreads();
    if (qi < mq) {
        const int q = s_q[qi];
        const int m = min(s_cnt[qi], kCapB);
        const int base = s_base[qi];
        for (int e = sub; e < m; e += 4) {
            if (base + e < kCapQ) {
                gbuf_e[(int64_t)q * kCapQ + base + e] = s_be[qi][e];
                gbuf_i[(int64_t)q * kCapQ + base + e] = s_bi[qi][e];
            }
        }
    }
    __syncthreads();                               // LDS of this item is free; s_item[4] is the next id
    }
}


// ---------------------------------------------------------------------------
// Two-stage pass B (Sec. 4.2, most significant bits first).  For a group of
// two code tiles, every (member, query) pair first gets the 1-bit estimate
// of the most significant bit planes (RaBitQ's code of the same residual),
//     est1 = g1 + f1 * delta/2 * (2 <x_b, q_int> - sum q_int) + ||s||^2,
// g1 = f_add - f1 <x, c'> (x = x_b - 1/2, f1 = -4 f_add / ||r'||_1), and its
// Lemma 2.1 lower bound est1 - eps0 ||s|| e1 (e1 = 2 ||r|| sqrt(1 - c^2) / c
// / sqrt(D - 1), c = ||r'||_1 / (sqrt(D) ||r||), per member).  Pairs whose
// bound is above the query's bound are dropped; when no pair of the group is
// left, the group's full codes are never read.  Otherwise the full product
// <y_u, q_int> of the group is taken from the full codes (on the matrix cores
// it costs the same as the product of the remaining bits alone), and the
// pairs kept by the first stage get the one-stage estimate and bound test.
// ---------------------------------------------------------------------------
constexpr int kVch2 = 384;     // members per item (the LDS also holds their 1-bit factors)

template <int BITS, int NQT>
__global__ __launch_bounds__(kThreads, 2) void scan2_kernel(
    const uint8_t* __restrict__ codes, const uint8_t* __restrict__ msb, const int64_t* __restrict__ tile_off,
    const int64_t* __restrict__ list_off, const float2* __restrict__ fac, const float4* __restrict__ fac1,
    const int64_t* __restrict__ ids, int dp, QArgs qa, const int32_t* __restrict__ pair_q,
    const int32_t* __restrict__ pair_slot, const int32_t* __restrict__ item_off, const int4* __restrict__ desc,
    int nlist, unsigned* __restrict__ tau_key, int32_t* __restrict__ gcnt, float* __restrict__ gbuf_e,
    int32_t* __restrict__ gbuf_i, int32_t* __restrict__ work, float eps0, int32_t* __restrict__ gstat)
{
    // gstat (or null): [0] groups scanned, [1] groups whose full codes were not read
    constexpr int QPI = kQT * NQT;
    constexpr int KC = 4;                          // K-blocks whose words are loaded together
    extern __shared__ __align__(16) char smem[];
    __shared__ float s_s2[QPI], s_hd[QPI];
    __shared__ int s_ss[QPI], s_slot[QPI], s_q[QPI], s_cnt[QPI], s_base[QPI];
    __shared__ float s_be[QPI][kCapB];
    __shared__ int s_bi[QPI][kCapB];
    __shared__ unsigned s_tau[QPI];
    __shared__ float2 s_fac[kVch2 + 64];
    __shared__ float4 s_f1[kVch2 + 64];
    __shared__ int s_id[kVch2 + 64];
    __shared__ int s_item[5];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_items = item_off[nlist];
    if (tid == 0) s_item[4] = atomicAdd(work, 1);
    __syncthreads();
    for (;;) {
    const int item = s_item[4];
    if (item >= n_items) break;
    if (tid == 0) {
        const int4 d = desc[item];
        s_item[0] = d.x; s_item[1] = d.y; s_item[2] = d.z; s_item[3] = d.w;
    }
    if (tid < QPI) s_cnt[tid] = 0;
    __syncthreads();
    if (tid == 0) s_item[4] = atomicAdd(work, 1);  // read again only after the item's last barrier
    const int l = s_item[0], p0 = s_item[1], mq = s_item[2], v0 = s_item[3];
    int8_t* qs = (int8_t*)smem;
    const int qstride = dp + 16;
    load_query_scalars(s_s2, s_hd, s_ss, s_slot, s_q, s_tau, tau_key, qa, pair_q + p0, pair_slot + p0, mq, tid);
    {   // factors (both stages) and ids of the item's members; past the end NaN, which never passes
        constexpr int KF = (kVch2 + 64 + kThreads - 1) / kThreads;
        const int64_t fb = list_off[l] + v0;
        const int nf = min((int)(list_off[l + 1] - list_off[l]) - v0, kVch2);
        const int nfp = (nf + 63) & ~63;
        float2 fv[KF];
        float4 gv[KF];
        int iv[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int t = tid + k * kThreads;
            const bool in = t < nf;
            fv[k] = in ? fac[fb + t] : make_float2(__builtin_nanf(""), 0.0f);
            gv[k] = in ? fac1[fb + t] : make_float4(__builtin_nanf(""), 0.0f, 0.0f, 0.0f);
            iv[k] = in ? (int)ids[fb + t] : -1;
        }
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int t = tid + k * kThreads;
            if (t < nfp) { s_fac[t] = fv[k]; s_f1[t] = gv[k]; s_id[t] = iv[k]; }
        }
    }
    __syncthreads();
    load_query_rows<NQT>(qs, qstride, s_q, qa.qint, dp, mq, tid);
    __syncthreads();

    const int nkb = dp / 64;
    const int8_t* qrow = qs + (lane & 31) * qstride + 16 * (lane >> 5);
    const int64_t tile_bytes = (int64_t)4 * dp * BITS, tile1 = (int64_t)4 * dp;
    const int nl = min((int)(list_off[l + 1] - list_off[l]) - v0, kVch2);
    const int ntile = (nl + 31) >> 5;
    const int64_t tbase = tile_off[l] + (v0 >> 5);
    const int j = lane & 31;
    // column constants as in scanB_kernel, for both code widths, and the
    // bound's per-column factor eps0 * ||s||
    float qs2[NQT], cH2[NQT], cHC[NQT], cH21[NQT], cHC1[NQT], cAQ[NQT], cEN[NQT];
#pragma unroll
    for (int qt = 0; qt < NQT; ++qt) {
        const int qi = qt * kQT + j;
        const bool ok = qi < mq;
        qs2[qt] = ok ? s_s2[qi] : 0.0f;
        const float hd = ok ? s_hd[qi] : 0.0f, tau = ok ? key2f(s_tau[qi]) : 0.0f;
        const int ss = ok ? s_ss[qi] : 0;
        epi_consts<BITS>(hd, ss, cH2[qt], cHC[qt]);
        epi_consts<1>(hd, ss, cH21[qt], cHC1[qt]);
        const float aq = tau - qs2[qt];
        cAQ[qt] = ok ? aq + (fabsf(tau) + fabsf(qs2[qt])) * 0x1p-20f : -__builtin_huge_valf();
        cEN[qt] = eps0 * sqrtf(fmaxf(qs2[qt], 0.0f));
    }
    const int ta = (wid * ntile) >> 2, tb = ((wid + 1) * ntile) >> 2;
    for (int gt0 = ta; gt0 < tb; gt0 += 2) {
        // a single-tile group (the last of an odd range) reads its tile twice
        // and ignores the copy
        const int64_t o0 = tbase + gt0, o1 = (gt0 + 1 < tb) ? o0 + 1 : o0;
        v16i acc[2][NQT];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int qt = 0; qt < NQT; ++qt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][qt][r] = 0;
        // stage 1: the most significant bit planes
        for (int kb0 = 0; kb0 < nkb; kb0 += KC) {
            uint32_t w[KC][2];
#pragma unroll
            for (int p = 0; p < KC; ++p) {
                const int kb = min(kb0 + p, nkb - 1);
                w[p][0] = *(const uint32_t*)(msb + o0 * tile1 + kb * 256 + lane * 4);
                w[p][1] = *(const uint32_t*)(msb + o1 * tile1 + kb * 256 + lane * 4);
            }
#pragma unroll
            for (int p = 0; p < KC; ++p) {
                const int kb = kb0 + p;
                if (kb >= nkb) break;                   // wave-uniform
                v4i a00, a01, a10, a11;
                unpack_raw<1>(w[p], a00, a01);
                unpack_raw<1>(w[p] + 1, a10, a11);
#pragma unroll
                for (int qt = 0; qt < NQT; ++qt) {
                    const v4i b0 = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb);
                    const v4i b1 = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb + 32);
                    acc[0][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a00, b0, acc[0][qt], 0, 0, 0);
                    acc[1][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a10, b0, acc[1][qt], 0, 0, 0);
                    acc[0][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a01, b1, acc[0][qt], 0, 0, 0);
                    acc[1][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a11, b1, acc[1][qt], 0, 0, 0);
                }
            }
        }
        // lower-bound test: bit a*16 + r of pm[qt] for every kept pair
        uint32_t pm[NQT];
#pragma unroll
        for (int qt = 0; qt < NQT; ++qt) pm[qt] = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int tt = gt0 + a;
            if (tt >= tb) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float4 g = s_f1[tt * 32 + out_row(lane, r)];
#pragma unroll
                for (int qt = 0; qt < NQT; ++qt) {
                    const float e1 = epi_e(make_float2(g.x, g.y), acc[a][qt][r], cH21[qt], cHC1[qt]);
                    if (__fmaf_rn(-cEN[qt], g.z, e1) <= cAQ[qt]) pm[qt] |= 1u << (a * 16 + r);
                }
            }
        }
        bool anyq = false;
#pragma unroll
        for (int qt = 0; qt < NQT; ++qt) anyq = anyq || pm[qt] != 0;
        const bool skip = !__any(anyq);                 // wave-uniform
        if (gstat && lane == 0) {                       // counted only while profiling
            atomicAdd(&gstat[0], 1);
            if (skip) atomicAdd(&gstat[1], 1);
        }
        if (skip) continue;                             // the group's full codes are not read
        // stage 2: the full codes
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int qt = 0; qt < NQT; ++qt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][qt][r] = 0;
        for (int kb0 = 0; kb0 < nkb; kb0 += KC) {
            uint32_t w[KC][2 * BITS];
#pragma unroll
            for (int p = 0; p < KC; ++p) {
                const int kb = min(kb0 + p, nkb - 1);
                load_raw<BITS>(codes + o0 * tile_bytes + (int64_t)kb * 256 * BITS, lane, w[p]);
                load_raw<BITS>(codes + o1 * tile_bytes + (int64_t)kb * 256 * BITS, lane, w[p] + BITS);
            }
#pragma unroll
            for (int p = 0; p < KC; ++p) {
                const int kb = kb0 + p;
                if (kb >= nkb) break;
                v4i a00, a01, a10, a11;
                unpack_raw<BITS>(w[p], a00, a01);
                unpack_raw<BITS>(w[p] + BITS, a10, a11);
#pragma unroll
                for (int qt = 0; qt < NQT; ++qt) {
                    const v4i b0 = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb);
                    const v4i b1 = *(const v4i*)(qrow + qt * kQT * qstride + 64 * kb + 32);
                    acc[0][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a00, b0, acc[0][qt], 0, 0, 0);
                    acc[1][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a10, b0, acc[1][qt], 0, 0, 0);
                    acc[0][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a01, b1, acc[0][qt], 0, 0, 0);
                    acc[1][qt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a11, b1, acc[1][qt], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int tt = gt0 + a;
            if (tt >= tb) break;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int v = tt * 32 + out_row(lane, r);
                const uint32_t bit = 1u << (a * 16 + r);
#pragma unroll
                for (int qt = 0; qt < NQT; ++qt) {
                    if (!(pm[qt] & bit)) continue;
                    const float e = epi_e(s_fac[v], acc[a][qt][r], cH2[qt], cHC[qt]);
                    if (!(e <= cAQ[qt])) continue;
                    const float est = e + qs2[qt];
                    const int qi = qt * kQT + j;
                    const int id = s_id[v];
                    const int pos = atomicAdd(&s_cnt[qi], 1);
                    if (pos < kCapB) {
                        s_be[qi][pos] = est; s_bi[qi][pos] = id;
                    } else {                            // stage full: straight to HBM
                        const int q = s_q[qi];
                        const int gp = atomicAdd(&gcnt[q], 1);
                        if (gp < kCapQ) {
                            gbuf_e[(int64_t)q * kCapQ + gp] = est;
                            gbuf_i[(int64_t)q * kCapQ + gp] = id;
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // flush the LDS stage to the query's candidate buffer
    const int qi = tid >> 2, sub = tid & 3;
    if (qi < mq && sub == 0) {
        const int m = min(s_cnt[qi], kCapB);
        s_base[qi] = (m > 0) ? atomicAdd(&gcnt[s_q[qi]], m) : 0;
    }
    __syncthreads();
    if (qi < mq) {
        const int q = s_q[qi];
        const int m = min(s_cnt[qi], kCapB);
        const int base = s_base[qi];
        for (int e = sub; e < m; e += 4) {
            if (base + e < kCapQ) {
                gbuf_e[(int64_t)q * kCapQ + base + e] = s_be[qi][e];
                gbuf_i[(int64_t)q * kCapQ + base + e] = s_bi[qi][e];
            }
        }
    }
    __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Per query, over its candidate buffer (count c): radix select of the key of
// the kk-th smallest estimate (4 passes of 8 bits).  One wave per query (4
// per block); each pass re-reads the buffer (lane l: entries l, l + 64, ...,
// just written, so from L2) into a wave-private LDS histogram; no block
// barrier.  For kk <= 64 a shorter route usually applies: a bound from the
// lanes' minima picks at most 64 candidates that contain the top-kk, and one
// bitonic sort of (key, id) across the wave ranks them.
//   mode 0: lowers the query's bound to it (the kk-th best candidate so far).
//   mode 1: writes the exact top-kk ascending by (est, id): every candidate
//           with a smaller key, and of those whose key equals the kk-th the
//           ones with the smallest ids (a second radix select, over ids,
//           when they are more than needed); at most kk entries are then
//           ranked by (est, id).  A buffer that overflowed raises the
//           query's flag for the fallback.
//   mode 2: after a round; a buffer that overflowed raises the flag, gets back
//           the count gprev it had before the round, and the bound drops to
//           the kk-th best of its kCapQ stored candidates (all of them real
//           estimates of distinct members, so still a valid bound).
// ---------------------------------------------------------------------------
constexpr int kSelQ = 4;               // queries (waves) per block
constexpr int kSelB = 8;               // entries per lane loaded together (512 per wave)

// LDS written by some lanes of a wave and read by others: wait for the
// wave's LDS operations and keep the compiler from moving accesses across
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Rank kr (1-based) among the values val(t) (t < c) with (v & mask) ==
// prefix: the next 8-bit digit at `shift` and the rank within that digit.
// Lane l reads entries l, l + 64, ...; hist: the wave's 256 bins.
template <class F>
__device__ __attribute__((always_inline)) inline void wave_digit(const unsigned (&v0)[kSelB], F val, int c, int lane,
                                                                  unsigned prefix, unsigned mask, int shift,
                                                                  unsigned* hist, unsigned& kr, unsigned& digit)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[lane * 4 + b] = 0;
    wave_lds_sync();
    unsigned run_d = 0xFFFFFFFFu, run_n = 0;
    // the first 64 * kSelB entries come from registers (v0), the rest in
    // batches with kSelB loads in flight
    for (int base = 0; base < c; base += 64 * kSelB) {
        unsigned v[kSelB];
#pragma unroll
        for (int k = 0; k < kSelB; ++k) {
            const int t = base + lane + 64 * k;
            v[k] = (base == 0) ? v0[k] : ((t < c) ? val(t) : 0u);
        }
#pragma unroll
        for (int k = 0; k < kSelB; ++k) {
            const int t = base + lane + 64 * k;
            if (t < c && (v[k] & mask) == prefix) {
                const unsigned dg = (v[k] >> shift) & 0xFF;
                if (dg != run_d) {
                    if (run_n) atomicAdd(&hist[run_d], run_n);
                    run_d = dg; run_n = 0;
                }
                ++run_n;
            }
        }
    }
    if (run_n) atomicAdd(&hist[run_d], run_n);
    wave_lds_sync();
    unsigned h[4], s = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) { h[b] = hist[lane * 4 + b]; s += h[b]; }
    unsigned incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    unsigned run = incl - s, my_d = 0, my_kr = 0;
    bool found = false;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (!found && run < kr && kr <= run + h[b]) { found = true; my_d = lane * 4 + b; my_kr = kr - run; }
        run += h[b];
    }
    const int src = __ffsll((unsigned long long)__ballot(found)) - 1;
    digit = __shfl(my_d, src);
    kr = __shfl(my_kr, src);
    wave_lds_sync();                        // the bins are read before the next pass clears them
}

// Ascending bitonic sort of one 64-bit value per lane across the wave
// (lane r ends with the r-th smallest)
__device__ inline unsigned long long wave_sort_u64(unsigned long long v, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned plo = (unsigned)__shfl_xor((int)(unsigned)v, j);
            const unsigned phi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), j);
            const unsigned long long p = ((unsigned long long)phi << 32) | plo;
            const bool take_min = ((lane & j) == 0) == ((lane & k) == 0);
            v = take_min ? (p < v ? p : v) : (p > v ? p : v);
        }
    return v;
}

// LDS slots per wave for the selected entries of mode 1: a power of two >= kk
// (and >= 64), so that a bitonic sort can run over them
__host__ __device__ inline int sel_slots(int kk) {
    int s = 64;
    while (s < kk) s <<= 1;
    return s;
}

// Ascending bitonic sort by (est, id) of the m entries (se, si) of one wave
// in LDS, padded with (+inf, INT_MAX) up to the next power of two (at most
// sel_slots(kk) entries); lanes move pairs t, t + 64, ... of each step.
__device__ inline void wave_bitonic(float* se, int* si, int m, int lane) {
    int S = 1;
    while (S < m) S <<= 1;
    for (int t = m + lane; t < S; t += 64) { se[t] = __builtin_huge_valf(); si[t] = 0x7FFFFFFF; }
    wave_lds_sync();
    for (int kb = 2; kb <= S; kb <<= 1)
        for (int j = kb >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < S / 2; t += 64) {
                const int i = 2 * t - (t & (j - 1)), p = i + j;
                const bool up = (i & kb) == 0;
                const float e0 = se[i], e1 = se[p];
                const int i0 = si[i], i1 = si[p];
                if (lt(e0, i0, e1, i1) != up) { se[i] = e1; se[p] = e0; si[i] = i1; si[p] = i0; }
            }
            wave_lds_sync();
        }
}

// post (mode 0 only), applied on entry after the count is read: 1 empties the
// buffer (count and count-before-round 0), 2 records the count as the
// count before the next round (after dropping, from a buffer more than a
// quarter full, the entries above the new bound), 3 (after the first bound)
// keeps the entries at or under the new bound and drops the padding, and
// records what is left as the count before the first round
template <int MODE>
__global__ __launch_bounds__(256) void buf_select_kernel(int32_t* __restrict__ gcnt,
                                                         int32_t* __restrict__ gprev,
                                                         float* __restrict__ gbuf_e,
                                                         int32_t* __restrict__ gbuf_i, int64_t nq, int kk,
                                                         int post, unsigned* __restrict__ tau_key,
                                                         int32_t* __restrict__ ovf, int64_t* __restrict__ out_ids,
                                                         float* __restrict__ out_est, int32_t* __restrict__ any_over)
{
    constexpr int mode = MODE;
    __shared__ unsigned hist[kSelQ][256];
    // mode 1: the selected entries of each wave, kS = pow2 >= max(kk, 64) slots
    extern __shared__ __align__(16) char sel_smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kS = sel_slots(kk);
    float* s_e = (float*)sel_smem + w * kS;
    int* s_i = (int*)(sel_smem + sizeof(float) * kSelQ * kS) + w * kS;
    const int64_t q = (int64_t)blockIdx.x * kSelQ + w;
    if (q >= nq) return;                                // the whole wave
    const int craw = gcnt[q];
    const bool over = craw > kCapQ;
    if (mode == 0 && (post == 1 || post == 2) && lane == 0) {
        if (post == 1) { gcnt[q] = 0; gprev[q] = 0; }
        else gprev[q] = craw;
    }
    if (mode != 0 && over && lane == 0) atomicOr(any_over, 1);   // gate of the rescans / fallback
    if (mode == 1 && over) {
        if (lane == 0) ovf[q] = 1;
        return;
    }
    if (mode != 0 && !over) {
        if (lane == 0) ovf[q] = 0;
        if (mode == 2) return;
    }
    if (mode == 0 && post != 3 && (over || craw < kk)) return;   // no (new) bound from this buffer
    const int c = over ? kCapQ : craw;
    const float* be = gbuf_e + q * kCapQ;
    const int* bi = gbuf_i + q * kCapQ;
    auto key_at = [&](int t) -> unsigned { return f2key(be[t]); };
    unsigned key0[kSelB];                                // keys of entries lane + 64 k (k < kSelB)
#pragma unroll
    for (int k = 0; k < kSelB; ++k) {
        const int t = lane + 64 * k;
        key0[k] = (t < c) ? key_at(t) : 0u;
    }
    unsigned kth = 0xFFFFFFFFu, need_eq = 0;
    // kk <= 64 and every key in registers: the kk-th smallest of the lanes'
    // minima is at or above the kk-th smallest key (the kk lanes at or below
    // it each hold a distinct key no larger), so the keys at or under it
    // contain the top-kk; when they are at most 64, one sort across the wave
    // of (key, id) ranks them directly.  Otherwise the radix select below.
    bool fast = false;
    if (kk <= 64 && c >= kk) {
        // keys of batch `base` (the first from registers, the rest re-read
        // from the buffer, just written, so from L2); past c all ones
        auto batch = [&](int base, unsigned (&v)[kSelB]) {
#pragma unroll
            for (int k = 0; k < kSelB; ++k) {
                const int t = base + lane + 64 * k;
                v[k] = (base == 0) ? (t < c ? key0[k] : 0xFFFFFFFFu) : (t < c ? key_at(t) : 0xFFFFFFFFu);
            }
        };
        unsigned mn = 0xFFFFFFFFu;
        for (int base = 0; base < c; base += 64 * kSelB) {
            unsigned v[kSelB];
            batch(base, v);
#pragma unroll
            for (int k = 0; k < kSelB; ++k) mn = min(mn, v[k]);
        }
        const unsigned long long ms = wave_sort_u64(((unsigned long long)mn << 32) | (unsigned)lane, lane);
        const unsigned T = (unsigned)__shfl((int)(unsigned)(ms >> 32), kk - 1);
        unsigned m = 0;
        for (int base = 0; base < c; base += 64 * kSelB) {
            unsigned v[kSelB];
            batch(base, v);
#pragma unroll
            for (int k = 0; k < kSelB; ++k) m += (unsigned)__popcll(__ballot(base + lane + 64 * k < c && v[k] <= T));
        }
        if (m <= 64) {
            fast = true;
            unsigned* ck = hist[w];                      // keys of the candidates [0, 64), positions [64, 128)
            const unsigned long long below = (1ull << lane) - 1ull;
            unsigned run = 0;
            for (int base = 0; base < c; base += 64 * kSelB) {
                unsigned v[kSelB];
                batch(base, v);
#pragma unroll
                for (int k = 0; k < kSelB; ++k) {
                    const bool p = base + lane + 64 * k < c && v[k] <= T;
                    const unsigned long long bal = __ballot(p);
                    if (p) {
                        const unsigned pos = run + (unsigned)__popcll(bal & below);
                        ck[pos] = v[k];
                        ck[64 + pos] = (unsigned)(base + lane + 64 * k);
                    }
                    run += (unsigned)__popcll(bal);
                }
            }
            wave_lds_sync();
            unsigned long long cv = ~0ull;               // past the candidates: above every (key, id)
            if (lane < (int)m)
                cv = ((unsigned long long)ck[lane] << 32) | (mode == 1 ? (unsigned)bi[ck[64 + lane]] : (unsigned)lane);
            wave_lds_sync();
            cv = wave_sort_u64(cv, lane);
            kth = (unsigned)__shfl((int)(unsigned)(cv >> 32), kk - 1);
            if (mode == 1) {                             // the top-kk by (est, id), in order
                if (lane < kk) {
                    out_ids[q * kk + lane] = (int)(unsigned)cv;
                    out_est[q * kk + lane] = key2f((unsigned)(cv >> 32));
                }
                return;
            }
        }
    }
    if (!fast && c >= kk) {
        unsigned prefix = 0, mask = 0, kr = (unsigned)kk;
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 24 - 8 * pass;
            unsigned dg;
            wave_digit(key0, key_at, c, lane, prefix, mask, shift, hist[w], kr, dg);
            prefix |= dg << shift;
            mask |= 0xFFu << shift;
        }
        kth = prefix;
        need_eq = kr;                                    // entries equal to kth that belong to the top-kk
    }
    if (mode == 0) {
        if (lane == 0) atomicMin(&tau_key[q], kth);
        if (post == 3 || (post == 2 && c > kCapQ / 4)) {
            // between rounds: entries above the new bound can never reach the
            // top-kk, so the buffer keeps only those at or below it (in place,
            // in buffer order: every entry moves to a position at or before
            // its own, and a chunk is read whole before any of it is written).
            // The first bound's padding (+inf, no member) is dropped too.
            constexpr unsigned kInfKey = 0xFF800000u;    // f2key(+inf)
            float* wbe = gbuf_e + q * kCapQ;
            int32_t* wbi = gbuf_i + q * kCapQ;
            const unsigned long long below = (1ull << lane) - 1ull;
            unsigned run = 0;
            for (int base = 0; base < c; base += 64 * kSelB) {
                bool kv[kSelB];
                float ev[kSelB];
                int iv[kSelB];
#pragma unroll
                for (int k = 0; k < kSelB; ++k) {
                    const int t = base + lane + 64 * k;
                    const unsigned kt = t >= c ? 0xFFFFFFFFu : (base == 0 ? key0[k] : key_at(t));
                    kv[k] = kt <= kth && kt < kInfKey;
                    ev[k] = kv[k] ? wbe[t] : 0.0f;
                    iv[k] = kv[k] ? wbi[t] : 0;
                }
#pragma unroll
                for (int k = 0; k < kSelB; ++k) {
                    const unsigned long long bal = __ballot(kv[k]);
                    if (kv[k]) {
                        const unsigned p = run + (unsigned)__popcll(bal & below);
                        wbe[p] = ev[k];
                        wbi[p] = iv[k];
                    }
                    run += (unsigned)__popcll(bal);
                }
            }
            if (lane == 0) { gcnt[q] = (int)run; gprev[q] = (int)run; }
        }
        return;
    }
    if (mode == 2) {                                     // over: kCapQ >= kk entries were ranked
        if (lane == 0) {
            atomicMin(&tau_key[q], kth);
            gcnt[q] = gprev[q];
            ovf[q] = 1;
        }
        return;
    }
    // mode 1: the selected entries.  c < kk: all of them.  Else every key
    // below kth, and of the keys equal to kth the need_eq smallest ids.
    unsigned idth = 0xFFFFFFFFu;                         // ids <= idth are taken among the equal keys
    if (c >= kk) {
        unsigned neq = 0;
        for (int base = 0; base < c; base += 64 * kSelB) {
            unsigned v[kSelB];
#pragma unroll
            for (int k = 0; k < kSelB; ++k) {
                const int t = base + lane + 64 * k;
                v[k] = (base == 0) ? key0[k] : ((t < c) ? key_at(t) : 0u);
            }
#pragma unroll
            for (int k = 0; k < kSelB; ++k) neq += (base + lane + 64 * k < c && v[k] == kth) ? 1u : 0u;
        }
        for (int o = 32; o > 0; o >>= 1) neq += __shfl_xor(neq, o);
        if (neq > need_eq) {                             // ties at the boundary: smallest ids win
            // entries outside the tie read as 0xFFFFFFFF, above any id taken
            auto id_at = [&](int t) -> unsigned { return key_at(t) == kth ? (unsigned)bi[t] : 0xFFFFFFFFu; };
            unsigned id0[kSelB];
#pragma unroll
            for (int k = 0; k < kSelB; ++k) {
                const int t = lane + 64 * k;
                id0[k] = (t < c && key0[k] == kth) ? (unsigned)bi[t] : 0xFFFFFFFFu;
            }
            unsigned prefix = 0, mask = 0, kr = need_eq;
            for (int pass = 0; pass < 4; ++pass) {
                const int shift = 24 - 8 * pass;
                unsigned dg;
                wave_digit(id0, id_at, c, lane, prefix, mask, shift, hist[w], kr, dg);
                prefix |= dg << shift;
                mask |= 0xFFu << shift;
            }
            idth = prefix;
        }
    }
    // compaction of the selected entries (at most kk, in lane order)
    auto sel_key = [&](int t, unsigned k) -> bool {
        if (c < kk) return true;
        return k < kth || (k == kth && (idth == 0xFFFFFFFFu || (unsigned)bi[t] <= idth));
    };
    auto selected = [&](int base, int k) -> bool {
        const int t = base + lane + 64 * k;
        return sel_key(t, base == 0 ? key0[k] : key_at(t));
    };
    unsigned cnt = 0;
    for (int base = 0; base < c; base += 64 * kSelB) {
        bool v[kSelB];
#pragma unroll
        for (int k = 0; k < kSelB; ++k) {
            const int t = base + lane + 64 * k;
            v[k] = (t < c) && selected(base, k);
        }
#pragma unroll
        for (int k = 0; k < kSelB; ++k) cnt += v[k] ? 1u : 0u;
    }
    unsigned pos = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(pos, o);
        if (lane >= o) pos += y;
    }
    const unsigned m_all = __shfl(pos, 63);
    pos -= cnt;                                          // exclusive prefix
    for (int base = 0; base < c && __any(cnt > 0); base += 64 * kSelB) {
        bool v[kSelB];
#pragma unroll
        for (int k = 0; k < kSelB; ++k) {
            const int t = base + lane + 64 * k;
            v[k] = cnt > 0 && (t < c) && selected(base, k);
        }
#pragma unroll
        for (int k = 0; k < kSelB; ++k) {
            if (v[k]) {
                const int t = base + lane + 64 * k;
                if (pos < (unsigned)kk) {
                    s_e[pos] = be[t];
                    s_i[pos] = bi[t];
                }
                ++pos;
                --cnt;
            }
        }
    }
    wave_lds_sync();
    const int m = (int)min(m_all, (unsigned)kk);
    if (m <= 64) {
        // rank of entry `lane` by (est, id) among the m selected; equal pairs by position
        if (lane < m) {
            const float e = s_e[lane];
            const int id = s_i[lane];
            int r = 0;
            for (int j = 0; j < m; ++j) {
                const float ej = s_e[j];
                const int ij = s_i[j];
                r += (lt(ej, ij, e, id) || (j < lane && ej == e && ij == id)) ? 1 : 0;
            }
            out_ids[q * kk + r] = id;
            out_est[q * kk + r] = e;
        }
    } else {
        wave_bitonic(s_e, s_i, m, lane);
        for (int t = lane; t < m; t += 64) {
            out_ids[q * kk + t] = s_i[t];
            out_est[q * kk + t] = s_e[t];
        }
    }
    for (int t = m + lane; t < kk; t += 64) {
        out_ids[q * kk + t] = -1;
        out_est[q * kk + t] = __builtin_huge_valf();
    }
}

// ---------------------------------------------------------------------------
// Exact fallback for the queries whose candidate buffer still overflowed
// after their rounds were rescanned: one workgroup per flagged query scans
// every member of its probed lists and keeps the exact kk smallest (est, id)
// in LDS as 64-bit keys (order-preserving image of the estimate, then the
// id).  Keys below the current threshold T are appended; when fewer than
// 4 * 32 free slots remain, a radix select keeps the kk smallest and T drops
// to the largest kept key, so each compaction frees kCapE - kk slots and the
// scan always advances.  Estimates use the pass-B arithmetic (epi_e), so a
// query gets the same result on this path as on the bounded one.
// ---------------------------------------------------------------------------
constexpr int kCapE = 4096;      // candidate keys per flagged query (LDS)
constexpr int kPerE = kCapE / 256;

// inclusive prefix sum over the 256 threads of a block; s_w: 4 slots
__device__ inline unsigned block_scan256(unsigned v, unsigned* s_w) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    unsigned base = 0;
    for (int w = 0; w < wid; ++w) base += s_w[w];
    __syncthreads();                             // s_w is free for the next call
    return base + x;
}

// Radix select (8 passes of 8 bits) of the kr-th smallest (1-based, kr <= c)
// of keys[0, c), block-wide.  Returns it; *need is how many of the keys equal
// to it belong to the kr smallest.
__device__ __attribute__((always_inline)) inline unsigned long long block_select64(
    const unsigned long long* keys, int c, unsigned kr, unsigned* hist, unsigned* s_w, unsigned* s_bc, unsigned& need)
{
    const int tid = threadIdx.x;
    unsigned long long prefix = 0, mask = 0;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        hist[tid] = 0;
        __syncthreads();
        unsigned run_d = 0xFFFFFFFFu, run_n = 0;
        for (int t = tid; t < c; t += 256) {
            const unsigned long long k = keys[t];
            if ((k & mask) == prefix) {
                const unsigned dg = (unsigned)(k >> shift) & 0xFFu;
                if (dg != run_d) {
                    if (run_n) atomicAdd(&hist[run_d], run_n);
                    run_d = dg; run_n = 0;
                }
                ++run_n;
            }
        }
        if (run_n) atomicAdd(&hist[run_d], run_n);
        __syncthreads();
        const unsigned v = hist[tid];
        const unsigned incl = block_scan256(v, s_w);
        const unsigned excl = incl - v;
        if (excl < kr && kr <= incl) { s_bc[0] = (unsigned)tid; s_bc[1] = kr - excl; }
        __syncthreads();
        prefix |= (unsigned long long)s_bc[0] << shift;
        mask |= 0xFFull << shift;
        kr = s_bc[1];
        __syncthreads();                         // s_bc and hist are read before the next pass
    }
    need = kr;
    return prefix;
}

// Keeps the kk smallest of keys[0, c) (c > kk, c <= kCapE) in keys[0, kk):
// the keys below the kk-th, then as many keys equal to it as belong to the kk
// smallest (first ones in index order).  Returns the kk-th smallest key.
// Every thread reads its contiguous chunk into registers before any writes.
__device__ __attribute__((always_inline)) inline unsigned long long block_keep(
    unsigned long long* keys, int c, int kk, unsigned* hist, unsigned* s_w, unsigned* s_bc)
{
    unsigned need;
    const unsigned long long kth = block_select64(keys, c, (unsigned)kk, hist, s_w, s_bc, need);
    const int per = (c + 255) / 256;             // <= kPerE
    const int b0 = min(c, (int)threadIdx.x * per), b1 = min(c, b0 + per);
    unsigned long long v[kPerE];
    unsigned nl = 0, ne = 0;
#pragma unroll
    for (int u = 0; u < kPerE; ++u) {
        const int t = b0 + u;
        v[u] = (t < b1) ? keys[t] : ~0ull;
        nl += (t < b1 && v[u] < kth) ? 1u : 0u;
        ne += (t < b1 && v[u] == kth) ? 1u : 0u;
    }
    unsigned pl = block_scan256(nl, s_w) - nl;   // barriers inside: every chunk has been read
    unsigned pe = block_scan256(ne, s_w) - ne;
    const unsigned nless = (unsigned)kk - need;
#pragma unroll
    for (int u = 0; u < kPerE; ++u) {
        const int t = b0 + u;
        if (t < b1) {
            if (v[u] < kth) keys[pl++] = v[u];
            else if (v[u] == kth) {
                if (pe < need) keys[nless + pe] = v[u];
                ++pe;
            }
        }
    }
    __syncthreads();
    return kth;
}

// Exact top-kk of one query over its probed lists by one workgroup, the
// query replicated over the 32 MFMA columns (LO: columns 16..31 its low
// plane).  Two uses:
//  * fallback (slices == 0): the flagged queries (ovf) of a scan whose
//    candidate buffer still overflowed; writes the sorted result;
//  * small batches (slices = S > 0, ovf and gate null): workgroup (q, s)
//    takes the s-th of S equal parts of query q's member tiles (over all its
//    probed lists, in probe order) and appends its top-kk
//    (unsorted) to the query's candidate buffer, whose count starts at 0
//    (at most S kk <= kCapQ entries, all distinct members), for the final
//    select; a search of a few queries then runs in a handful of launches.
// Grid-stride over (query, slice).  Dynamic LDS: kCapE keys, the tile prefix
// over the probes (nprobe + 1 ints, rounded up to 16 bytes) and the query's
// int8 rows (dp bytes per plane).  redo counts the probed pairs of the
// fallback's queries (diagnostics).
template <int BITS, bool LO>
__global__ __launch_bounds__(256) void exact_kernel(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ tile_off, const int64_t* __restrict__ list_off,
    const float2* __restrict__ fac, const int64_t* __restrict__ ids, int dp, QArgs qa,
    const int32_t* __restrict__ probes, int64_t nq, int nprobe, int nlist, int kk,
    const int32_t* __restrict__ ovf, const int32_t* __restrict__ gate, int32_t* __restrict__ redo,
    int64_t* __restrict__ out_ids, float* __restrict__ out_est, int slices, int32_t* __restrict__ gcnt,
    float* __restrict__ gbuf_e, int32_t* __restrict__ gbuf_i)
{
    if (gate && *gate == 0) return;
    const int S = slices > 0 ? slices : 1;
    extern __shared__ __align__(16) char smem[];
    unsigned long long* keys = (unsigned long long*)smem;
    int* tpref = (int*)(smem + sizeof(unsigned long long) * kCapE);
    int8_t* qs = (int8_t*)(tpref + ((nprobe + 4) & ~3));
    __shared__ unsigned hist[256], s_w[4], s_bc[2];
    __shared__ int s_cnt;
    __shared__ unsigned long long s_T;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nkb = dp / 64;
    const int64_t tile_bytes = (int64_t)4 * dp * BITS;
    // every MFMA column is the query itself; LO: columns 16..31 its low plane (LDS row 2)
    const int8_t* qrow = qs + 16 * (lane >> 5) + ((LO && (lane & 31) >= 16) ? dp : 0);
    for (int64_t w = blockIdx.x; w < nq * S; w += gridDim.x) {
        const int64_t q = w / S;
        const int sl = (int)(w - q * S);
        if (ovf && !ovf[q]) continue;            // the same for the whole block
        __syncthreads();                         // LDS of the previous query is free
        for (int c = tid; c < dp / 16; c += 256) *(uint4*)(qs + 16 * c) = *(const uint4*)(qa.qint + q * dp + 16 * c);
        if constexpr (LO)
            for (int c = tid; c < dp / 16; c += 256)
                *(uint4*)(qs + dp + 16 * c) = *(const uint4*)(qa.qlo + q * dp + 16 * c);
        // member tiles per probe (thread t: probes 4t .. 4t+3), exclusive prefix
        unsigned nt[4], sum = 0, npair = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = 4 * tid + u;
            unsigned n = 0;
            if (p < nprobe) {
                const int l = probes[q * nprobe + p];
                if (l >= 0 && l < nlist) {
                    n = (unsigned)((list_off[l + 1] - list_off[l] + 31) >> 5);
                    ++npair;
                }
            }
            nt[u] = n;
            sum += n;
        }
        const unsigned incl = block_scan256(sum, s_w);
        unsigned run = incl - sum;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = 4 * tid + u;
            if (p < nprobe) tpref[p] = (int)run;
            run += nt[u];
        }
        if (tid == 255) tpref[nprobe] = (int)incl;
        if (tid == 0) { s_cnt = 0; s_T = ~0ull; }
        if (redo && npair) atomicAdd(redo, (int)npair);
        __syncthreads();
        // the slice's share of the query's tiles (all probes, in probe order): an
        // even split, whatever the list lengths
        const int64_t all = tpref[nprobe];
        const int g0 = (int)(all * sl / S), total = (int)(all * (sl + 1) / S);
        float h2, hc, h2l = 0.0f;
        if constexpr (LO) epi_consts2<BITS>(qa.qhd[q], qa.qss[q], qa.qss_lo[q], h2, h2l, hc);
        else epi_consts<BITS>(qa.qhd[q], qa.qss[q], h2, hc);
        for (int base = g0; base < total; base += 4) {
            const int g = base + wid;
            const unsigned long long T = s_T;
            if (g < total) {
                int lo = 0, hi = nprobe;             // tpref[lo] <= g < tpref[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (tpref[mid] <= g) lo = mid; else hi = mid;
                }
                const int tt = g - tpref[lo];
                const int l = probes[q * nprobe + lo];
                const float s2 = fmaxf(qa.sdist[q * nprobe + lo], qa.s2_floor);
                const int64_t lb = list_off[l];
                const int nl = (int)(list_off[l + 1] - lb);
                const uint8_t* tp = codes + (tile_off[l] + tt) * tile_bytes;
                v16i acc;
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] = 0;
                // the packed words of KC K-blocks are loaded together, then used
                constexpr int KC = 8;
                for (int kb0 = 0; kb0 < nkb; kb0 += KC) {
                    uint32_t wd[KC][BITS];
#pragma unroll
                    for (int p = 0; p < KC; ++p)
                        load_raw<BITS>(tp + (int64_t)min(kb0 + p, nkb - 1) * 256 * BITS, lane, wd[p]);
#pragma unroll
                    for (int p = 0; p < KC; ++p) {
                        const int kb = kb0 + p;
                        if (kb >= nkb) break;            // wave-uniform
                        v4i a0, a1;
                        unpack_raw<BITS>(wd[p], a0, a1);
                        const v4i b0 = *(const v4i*)(qrow + 64 * kb);
                        const v4i b1 = *(const v4i*)(qrow + 64 * kb + 32);
                        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc, 0, 0, 0);
                    }
                }
                // lane (h, j < 16) takes output row out_row(lane, j): the 32
                // lanes cover the tile's 32 members once
                const int j = lane & 31;
                int a = acc[0];
#pragma unroll
                for (int r = 1; r < 16; ++r) a = (r == (j & 15)) ? acc[r] : a;
                // LO: lane j + 16 holds the low plane's product of the same row
                const int alo = LO ? __shfl_down(a, 16) : 0;
                if (j < 16) {
                    const int v = tt * 32 + out_row(lane, j);
                    if (v < nl) {
                        const float est = (LO ? epi_e2(fac[lb + v], a, alo, h2, h2l, hc)
                                              : epi_e(fac[lb + v], a, h2, hc)) + s2;
                        const unsigned long long key =
                            ((unsigned long long)f2key(est) << 32) | (unsigned)(int)ids[lb + v];
                        if (key < T) keys[atomicAdd(&s_cnt, 1)] = key;
                    }
                }
            }
            __syncthreads();
            if (s_cnt > kCapE - 4 * 32) {        // room for the next step's 128 candidates
                const unsigned long long kth = block_keep(keys, s_cnt, kk, hist, s_w, s_bc);
                if (tid == 0) { s_cnt = kk; s_T = kth; }
                __syncthreads();
            }
        }
        const int c = s_cnt;
        int m = c;
        if (c > kk) {
            block_keep(keys, c, kk, hist, s_w, s_bc);
            m = kk;
        }
        if (slices > 0) {                        // this slice's top-kk appended to the query's buffer
            __syncthreads();                     // every thread has read the count
            if (tid == 0) s_cnt = m > 0 ? atomicAdd(&gcnt[q], m) : 0;
            __syncthreads();
            const int base = s_cnt;
            for (int t = tid; t < m; t += 256) {
                const unsigned long long k = keys[t];
                gbuf_e[q * kCapQ + base + t] = key2f((unsigned)(k >> 32));
                gbuf_i[q * kCapQ + base + t] = (int32_t)(unsigned)(k & 0xFFFFFFFFull);
            }
            continue;
        }
        // ascending bitonic sort of keys[0, m), padded to a power of two (<= kk rounded up)
        int S = 1;
        while (S < m) S <<= 1;
        for (int t = m + tid; t < S; t += 256) keys[t] = ~0ull;
        __syncthreads();
        for (int kb = 2; kb <= S; kb <<= 1)
            for (int jj = kb >> 1; jj > 0; jj >>= 1) {
                for (int t = tid; t < S / 2; t += 256) {
                    const int i = 2 * t - (t & (jj - 1)), p = i + jj;
                    const bool up = (i & kb) == 0;
                    const unsigned long long k0 = keys[i], k1 = keys[p];
                    if ((k0 < k1) != up) { keys[i] = k1; keys[p] = k0; }
                }
                __syncthreads();
            }
        for (int t = tid; t < kk; t += 256) {
            if (t < m) {
                const unsigned long long k = keys[t];
                out_ids[q * kk + t] = (int64_t)(int)(unsigned)(k & 0xFFFFFFFFull);
                out_est[q * kk + t] = key2f((unsigned)(k >> 32));
            } else {
                out_ids[q * kk + t] = -1;
                out_est[q * kk + t] = __builtin_huge_valf();
            }
        }
    }
}

// q' -> int8 once per query (symmetric: inv = 127/max|q'|, round half to
// even, clamp to +-127), delta/2 and the sum of the int8 values; one wave per query
// (the first dp coordinates of each row of qrot, rows ld apart)
// qlo (or null): the low plane, q_lo = rint((q' * inv - q_int) * 254), and its sums
__global__ __launch_bounds__(256) void qprep_kernel(const float* __restrict__ qrot, int64_t nq, int dp, int ld,
                                                    int8_t* __restrict__ qint, float* __restrict__ qhd,
                                                    int32_t* __restrict__ qss, int8_t* __restrict__ qlo,
                                                    int32_t* __restrict__ qss_lo)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    const float* qv = qrot + q * ld;
    // rows of whole 256-float blocks, 16-byte aligned: four consecutive
    // coordinates per lane and access (same arithmetic per coordinate)
    const bool vec = (dp & 255) == 0 && (((uintptr_t)qv) & 15) == 0;
    float amax = 0.0f;
    if (vec) {
        for (int i = 4 * lane; i < dp; i += 256) {
            const float4 v = *(const float4*)(qv + i);
            amax = fmaxf(fmaxf(amax, fmaxf(fabsf(v.x), fabsf(v.y))), fmaxf(fabsf(v.z), fabsf(v.w)));
        }
    } else {
        for (int i = lane; i < dp; i += 64) amax = fmaxf(amax, fabsf(qv[i]));
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    const float inv = (amax > 0.0f) ? __fdiv_rn(127.0f, amax) : 0.0f;
    int ssum = 0, slo = 0;
    if (vec) {
        for (int i = 4 * lane; i < dp; i += 256) {
            const float4 v = *(const float4*)(qv + i);
            const float x[4] = {v.x, v.y, v.z, v.w};
            uint32_t hi = 0, lo = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float t = x[c] * inv;
                const int a = max(-127, min(127, (int)rintf(t)));
                hi |= (uint32_t)(uint8_t)(int8_t)a << (8 * c);
                ssum += a;
                if (qlo) {
                    const int b = max(-127, min(127, (int)rintf((t - (float)a) * 254.0f)));
                    lo |= (uint32_t)(uint8_t)(int8_t)b << (8 * c);
                    slo += b;
                }
            }
            *(uint32_t*)(qint + q * dp + i) = hi;
            if (qlo) *(uint32_t*)(qlo + q * dp + i) = lo;
        }
    } else
    for (int i = lane; i < dp; i += 64) {
        const float t = qv[i] * inv;
        int v = (int)rintf(t);
        v = max(-127, min(127, v));
        qint[q * dp + i] = (int8_t)v;
        ssum += v;
        if (qlo) {
            int w = (int)rintf((t - (float)v) * 254.0f);
            w = max(-127, min(127, w));
            qlo[q * dp + i] = (int8_t)w;
            slo += w;
        }
    }
    for (int o = 32; o > 0; o >>= 1) { ssum += __shfl_xor(ssum, o); slo += __shfl_xor(slo, o); }
    if (lane == 0) {
        qhd[q] = 0.5f * ((amax > 0.0f) ? __fdiv_rn(amax, 127.0f) : 0.0f);
        qss[q] = ssum;
        if (qss_lo) qss_lo[q] = slo;
    }
}

// The per-pair term of every (query, probe) pair in FP32, one wave per pair
// (used when the caller has no probe distances): ||q' - c'||^2 for L2,
// -<q', c'> for the inner-product metrics (IP)
// (over all dp coordinates of the rotated query and centroid, whatever the
// code dimension)
template <bool IP>
__global__ __launch_bounds__(256) void pair_s2_kernel(const float* __restrict__ qrot,
                                                      const float* __restrict__ cent_rot,
                                                      const int32_t* __restrict__ probes, int64_t np, int nprobe,
                                                      int nlist, int dp, float* __restrict__ sdist)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= np) return;
    const int l = probes[i];
    float s = 0.0f;
    if (l >= 0 && l < nlist) {
        const float* qv = qrot + (i / nprobe) * dp;
        const float* cv = cent_rot + (int64_t)l * dp;
        if constexpr (IP) {
            for (int d = lane; d < dp; d += 64) s -= qv[d] * cv[d];
        } else {
            for (int d = lane; d < dp; d += 64) { const float t = qv[d] - cv[d]; s += t * t; }
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) sdist[i] = s;
}

// Scan factors of every member: (g_add, f_rescale) with
// g_add = f_add - f_rescale * <y_bar, c'>, y_bar = y_u - (2^B-1)/2 and c' the
// rotated centroid of the member's list, <y_bar, c'> accumulated in FP64.
// Then est = g_add + ||s||^2 + f_rescale * <y_bar, q'> for s' = q' - c'.
// codes_u: n x dp unpacked y_u in list order; one wave per member.
// Inner-product metrics: (0, f_rescale / 2), so that the same epilogue gives
// -<c, q> + (f_rescale / 2) <y_bar, q'> with the per-pair term -<c', q'>.
__global__ __launch_bounds__(256) void scan_fac_kernel(const uint8_t* __restrict__ codes_u,
                                                       const int64_t* __restrict__ list_off, int nlist,
                                                       const float* __restrict__ cent_rot,
                                                       const float2* __restrict__ fac, int64_t n, int dp, int ld,
                                                       int bits, int ip, float2* __restrict__ sfac)
{
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    if (ip) {
        if (lane == 0) sfac[v] = make_float2(0.0f, 0.5f * fac[v].y);
        return;
    }
    int lo = 0, hi = nlist;                        // list of member v: last l with list_off[l] <= v
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (list_off[mid] <= v) lo = mid; else hi = mid; }
    const uint8_t* y = codes_u + v * dp;
    const float* c = cent_rot + (int64_t)lo * ld;      // the codes cover its first dp coordinates
    const double half = 0.5 * (double)((1 << bits) - 1);
    double acc = 0.0;
    for (int d = lane; d < dp; d += 64) acc += ((double)y[d] - half) * (double)c[d];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const float2 f = fac[v];
        sfac[v] = make_float2((float)((double)f.x - (double)f.y * acc), f.y);
    }
}

// 1-bit factors of the two-stage scan per member (list order), from the
// most significant bits x_b of y_u and l1 = ||r'||_1:
// (g1, f1, e1, 0) with f1 = -4 f_add / l1, g1 = f_add - f1 <x, c'> (x = x_b -
// 1/2, FP64 accumulate) and e1 = 2 ||r|| sqrt(1 - c^2) / c / sqrt(D - 1),
// c = l1 / (sqrt(D) ||r||); a member at its centroid gets (0, 0, 0, 0), whose
// 1-bit estimate ||s||^2 is exact.  One wave per member.
__global__ __launch_bounds__(256) void scan1_fac_kernel(const uint8_t* __restrict__ codes_u,
                                                        const int64_t* __restrict__ list_off, int nlist,
                                                        const float* __restrict__ cent_rot, int ld,
                                                        const float2* __restrict__ fac, const float* __restrict__ l1,
                                                        int64_t n, int dp, int bits, float4* __restrict__ fac1)
{
    const int lane = threadIdx.x & 63;
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (v >= n) return;
    int lo = 0, hi = nlist;
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (list_off[mid] <= v) lo = mid; else hi = mid; }
    const uint8_t* y = codes_u + v * dp;
    const float* c = cent_rot + (int64_t)lo * ld;
    double acc = 0.0;
    for (int d = lane; d < dp; d += 64) acc += ((double)(y[d] >> (bits - 1)) - 0.5) * (double)c[d];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const double fa = (double)fac[v].x, s1 = (double)l1[v];
        float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (fa > 0.0 && s1 > 0.0) {
            const double f1 = -4.0 * fa / s1, nr = sqrt(fa);
            const double cc = fmin(s1 / (sqrt((double)dp) * nr), 1.0);
            const double e1 = 2.0 * nr * sqrt(fmax(1.0 - cc * cc, 0.0)) / cc / sqrt((double)dp - 1.0);
            out = make_float4((float)(fa - f1 * acc), (float)f1, (float)e1, 0.0f);
        }
        fac1[v] = out;
    }
}

// before the first bound: slots [0, kDenseR*kDenseV) of every query's buffer
// hold +inf, the count covers them, and the bound is +inf
__global__ void fill_dense_kernel(float* __restrict__ gbuf_e, int64_t nq, int32_t* __restrict__ gcnt,
                                  unsigned* __restrict__ tau_key, int32_t* __restrict__ redo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 4 slots per thread
    constexpr int W = kDenseR * kDenseV;
    if (i < 3) redo[i] = 0;                        // counters: fallback pairs, two-stage groups, skipped groups
    if (4 * i >= nq * W) return;
    const int64_t q = (4 * i) / W, o = 4 * i - q * W;
    const float inf = __builtin_huge_valf();
    *(float4*)(gbuf_e + q * kCapQ + o) = make_float4(inf, inf, inf, inf);
    if (o == 0) { gcnt[q] = W; tau_key[q] = 0xFFFFFFFFu; }
}


// ---------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// pairs with probe rank in [rlo, rhi) (and, with qmask, of flagged queries only)
__device__ inline bool pair_sel(const int32_t* probes, int64_t i, int nprobe, int nlist, int rlo, int rhi,
                                const int32_t* qmask, int* l_out, int64_t* q_out) {
    const int l = probes[i];
    if (l < 0 || l >= nlist) return false;
    const int64_t q = i / nprobe;
    const int p = (int)(i - q * nprobe);
    if (p < rlo || p >= rhi) return false;
    if (qmask && !qmask[q]) return false;
    *l_out = l; *q_out = q;
    return true;
}

__global__ void pair_count_kernel(const int32_t* __restrict__ probes, int64_t np, int nprobe, int nlist,
                                  int rlo, int rhi, const int32_t* __restrict__ qmask, int32_t* __restrict__ cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int l; int64_t q;
    if (pair_sel(probes, i, nprobe, nlist, rlo, rhi, qmask, &l, &q)) atomicAdd(&cnt[l], 1);
}

__global__ void pair_scatter_kernel(const int32_t* __restrict__ probes, int64_t np, int nprobe, int nlist,
                                    int rlo, int rhi, const int32_t* __restrict__ qmask,
                                    const int32_t* __restrict__ off, int32_t* __restrict__ fill,
                                    int32_t* __restrict__ pq, int32_t* __restrict__ pslot)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int l; int64_t q;
    if (!pair_sel(probes, i, nprobe, nlist, rlo, rhi, qmask, &l, &q)) return;
    const int pos = off[l] + atomicAdd(&fill[l], 1);
    pq[pos] = (int32_t)q;
    pslot[pos] = (int32_t)i;
}

// Items of list l: ceil(cnt/qpi) query tiles, times ceil((n_l - vs)/vch)
// member chunks when vch > 0 (none when n_l <= vs; members [0, vs) are
// skipped, already scanned); with vch == 0 one item per query tile, empty
// lists included (their pairs still get an output row).
__device__ inline int items_of(const int32_t* cnt, const int64_t* list_off, int l, int qpi, int vch, int vs) {
    const int tiles = (cnt[l] + qpi - 1) / qpi;
    if (vch <= 0) return tiles;
    const int nv = (int)(list_off[l + 1] - list_off[l]) - vs;
    return nv > 0 ? tiles * ((nv + vch - 1) / vch) : 0;
}

// Counting sort of the selected pairs by list without global atomics, for
// nlist <= kHistMax: block b of kPairBlocks takes a contiguous range of pairs,
// counts them per list in LDS (cnt2[b][l]); a per-list exclusive prefix over
// the blocks gives every block its first slot in each list; each block then
// places its pairs with LDS atomics.
constexpr int kPairBlocks = 128;
constexpr int kHistMax = 16384;

// gate (all the kernels of a pair build and of a scan launch): when non-null
// and zero, the launch has nothing to do and returns at once
__global__ __launch_bounds__(1024) void pair_hist_kernel(const int32_t* __restrict__ probes, int64_t np, int nprobe,
                                                         int nlist, int rlo, int rhi,
                                                         const int32_t* __restrict__ qmask,
                                                         int32_t* __restrict__ cnt2, const int32_t* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int hist[kHistMax];
    const int b = blockIdx.x;
    for (int l = threadIdx.x; l < nlist; l += blockDim.x) hist[l] = 0;
    __syncthreads();
    const int64_t chunk = (np + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = b * chunk, i1 = min(np, i0 + chunk);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        int l; int64_t q;
        if (pair_sel(probes, i, nprobe, nlist, rlo, rhi, qmask, &l, &q)) atomicAdd(&hist[l], 1);
    }
    __syncthreads();
    for (int l = threadIdx.x; l < nlist; l += blockDim.x) cnt2[(int64_t)b * nlist + l] = hist[l];
}

// per list: exclusive prefix of cnt2 over the blocks (in place) and the total.
// 64 lists per workgroup; thread (list, quarter) loads its quarter of the
// blocks at once, quarter sums are combined in LDS
__global__ __launch_bounds__(256) void pair_colsum_kernel(int32_t* __restrict__ cnt2, int nlist,
                                                          int32_t* __restrict__ cnt, const int32_t* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    constexpr int BQ = kPairBlocks / 4;
    __shared__ int part[4][64];
    const int lq = threadIdx.x & 63, bq = threadIdx.x >> 6;
    const int l = blockIdx.x * 64 + lq;
    int v[BQ];
    int sum = 0;
#pragma unroll
    for (int t = 0; t < BQ; ++t) {
        v[t] = (l < nlist) ? cnt2[(int64_t)(bq * BQ + t) * nlist + l] : 0;
        sum += v[t];
    }
    part[bq][lq] = sum;
    __syncthreads();
    int run = 0;
    for (int w = 0; w < bq; ++w) run += part[w][lq];
    if (l >= nlist) return;
#pragma unroll
    for (int t = 0; t < BQ; ++t) {
        cnt2[(int64_t)(bq * BQ + t) * nlist + l] = run;
        run += v[t];
    }
    if (bq == 3) cnt[l] = run;
}

__global__ __launch_bounds__(1024) void pair_place_kernel(const int32_t* __restrict__ probes, int64_t np, int nprobe,
                                                          int nlist, int rlo, int rhi,
                                                          const int32_t* __restrict__ qmask,
                                                          const int32_t* __restrict__ cnt2,
                                                          const int32_t* __restrict__ off,
                                                          int32_t* __restrict__ pq, int32_t* __restrict__ pslot,
                                                          const int32_t* __restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int base[kHistMax];
    const int b = blockIdx.x;
    for (int l = threadIdx.x; l < nlist; l += blockDim.x) base[l] = off[l] + cnt2[(int64_t)b * nlist + l];
    __syncthreads();
    const int64_t chunk = (np + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = b * chunk, i1 = min(np, i0 + chunk);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        int l; int64_t q;
        if (!pair_sel(probes, i, nprobe, nlist, rlo, rhi, qmask, &l, &q)) continue;
        const int pos = atomicAdd(&base[l], 1);
        pq[pos] = (int32_t)q;
        pslot[pos] = (int32_t)i;
    }
}

__device__ inline void list_scan(const int32_t* __restrict__ cnt, int nlist, const int32_t* __restrict__ list_order,
                                 const int64_t* __restrict__ list_off, int qpi, int vch, int vs,
                                 int32_t* __restrict__ pair_off, int32_t* __restrict__ item_off);

// single workgroup: pair_off (by list id) and item_off (by rank of list_order).
// Thread 0 also zeroes the work counter of the scan launch that follows and,
// when given, two flags (zf0, zf1), so that they need no launches of their own.
__global__ __launch_bounds__(1024) void pair_scan_kernel(const int32_t* __restrict__ cnt, int nlist,
                                                         const int32_t* __restrict__ list_order,
                                                         const int64_t* __restrict__ list_off, int qpi, int vch,
                                                         int vs, int32_t* __restrict__ pair_off,
                                                         int32_t* __restrict__ item_off,
                                                         const int32_t* __restrict__ gate, int32_t* __restrict__ work,
                                                         int32_t* __restrict__ zf0, int32_t* __restrict__ zf1)
{
    if (threadIdx.x == 0) {
        *work = 0;
        if (zf0) *zf0 = 0;
        if (zf1) *zf1 = 0;
    }
    // a gated-off build publishes zero items, so the scan after it is empty
    if (gate && *gate == 0) {
        if (threadIdx.x == 0) { item_off[nlist] = 0; pair_off[nlist] = 0; }
        return;
    }
    list_scan(cnt, nlist, list_order, list_off, qpi, vch, vs, pair_off, item_off);
}

// One workgroup of 1024: exclusive prefix of the pair counts (pair_off, by
// list id) and of the item counts (item_off, by rank of list_order).
__device__ inline void list_scan(const int32_t* __restrict__ cnt, int nlist, const int32_t* __restrict__ list_order,
                                 const int64_t* __restrict__ list_off, int qpi, int vch, int vs,
                                 int32_t* __restrict__ pair_off, int32_t* __restrict__ item_off)
{
    __shared__ int part_a[1024], part_b[1024];
    const int tid = threadIdx.x;
    const int chunk = (nlist + 1023) / 1024;
    const int beg = tid * chunk, end = min(nlist, beg + chunk);
    int sa = 0, sb = 0;
    for (int i = beg; i < end; ++i) { sa += cnt[i]; sb += items_of(cnt, list_off, list_order[i], qpi, vch, vs); }
    part_a[tid] = sa; part_b[tid] = sb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int va = (tid >= o) ? part_a[tid - o] : 0;
        int vb = (tid >= o) ? part_b[tid - o] : 0;
        __syncthreads();
        part_a[tid] += va; part_b[tid] += vb;
        __syncthreads();
    }
    int ra = part_a[tid] - sa, rb = part_b[tid] - sb;
    for (int i = beg; i < end; ++i) {
        pair_off[i] = ra; ra += cnt[i];
        item_off[i] = rb; rb += items_of(cnt, list_off, list_order[i], qpi, vch, vs);
    }
    if (tid == 1023) { pair_off[nlist] = part_a[1023]; item_off[nlist] = part_b[1023]; }
}

// descriptor of every item, (list, first pair, queries, first member), so
// that a scan kernel reads one int4 per item; one thread per item
__device__ inline void item_desc_one(int64_t item, const int32_t* __restrict__ item_off,
                                     const int32_t* __restrict__ list_order, const int64_t* __restrict__ list_off,
                                     const int32_t* __restrict__ pair_off, int nlist, int qpi, int vch, int vs,
                                     int4* __restrict__ desc)
{
    int l, t;
    decode_item((int)item, item_off, list_order, nlist, &l, &t);
    const int nv = (int)(list_off[l + 1] - list_off[l]) - vs;
    const int nvc = (vch > 0) ? max(1, (nv + vch - 1) / vch) : 1;
    const int qtile = t / nvc, vc = t - qtile * nvc;
    const int p0 = pair_off[l] + qtile * qpi;
    desc[item] = make_int4(l, p0, min(qpi, pair_off[l + 1] - p0), vs + vc * vch);
}

__global__ void item_desc_kernel(const int32_t* __restrict__ item_off, const int32_t* __restrict__ list_order,
                                 const int64_t* __restrict__ list_off, const int32_t* __restrict__ pair_off,
                                 int nlist, int qpi, int vch, int vs, int64_t cap, int4* __restrict__ desc)
{
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // empty build: item_off[nlist] == 0
    if (item >= cap || item >= item_off[nlist]) return;
    item_desc_one(item, item_off, list_order, list_off, pair_off, nlist, qpi, vch, vs, desc);
}

// A gated pair build (the rescan of overflowed queries, the exact fallback)
// in one launch of one workgroup: nothing but the published empty build when
// the gate is off (the usual case); else the flagged queries are gathered into
// qlist (nq slots), and only their pairs of rank [rlo, rhi) are visited: count
// per list (global atomics), the list scan, placement and the item
// descriptors, in time proportional to the flagged pairs, not to all pairs.
// Their order within a list is free (every query's result is its exact top-kk
// whatever the grouping).  cnt: nlist counters.
__global__ __launch_bounds__(1024) void pair_build_gated_kernel(
    const int32_t* __restrict__ probes, int64_t nq, int nprobe, int nlist, int rlo, int rhi,
    const int32_t* __restrict__ qmask, const int32_t* __restrict__ list_order,
    const int64_t* __restrict__ list_off, int qpi, int vch, int vs, int32_t* __restrict__ cnt,
    int32_t* __restrict__ pair_off, int32_t* __restrict__ item_off, int32_t* __restrict__ pq,
    int32_t* __restrict__ pslot, int4* __restrict__ desc, int64_t cap, int32_t* __restrict__ work,
    const int32_t* __restrict__ gate, int32_t* __restrict__ qlist)
{
    __shared__ int nflag;
    const int tid = threadIdx.x;
    if (tid == 0) *work = 0;
    if (*gate == 0) {
        if (tid == 0) { item_off[nlist] = 0; pair_off[nlist] = 0; }
        return;
    }
    if (tid == 0) nflag = 0;
    for (int l = tid; l < nlist; l += 1024) cnt[l] = 0;
    __syncthreads();
    for (int64_t q = tid; q < nq; q += 1024)
        if (!qmask || qmask[q]) qlist[atomicAdd(&nflag, 1)] = (int32_t)q;
    __syncthreads();
    const int nr = rhi - rlo;
    const int64_t nsel = (int64_t)nflag * nr;     // flagged pairs, visited as (query of qlist, rank)
    for (int64_t j = tid; j < nsel; j += 1024) {
        const int64_t q = qlist[j / nr];
        const int l = probes[q * nprobe + rlo + (int)(j % nr)];
        if (l >= 0 && l < nlist) atomicAdd(&cnt[l], 1);
    }
    __syncthreads();
    list_scan(cnt, nlist, list_order, list_off, qpi, vch, vs, pair_off, item_off);
    __syncthreads();
    for (int l = tid; l < nlist; l += 1024) cnt[l] = 0;     // placement counters
    __syncthreads();
    for (int64_t j = tid; j < nsel; j += 1024) {
        const int64_t q = qlist[j / nr];
        const int64_t i = q * nprobe + rlo + (int)(j % nr);
        const int l = probes[i];
        if (l < 0 || l >= nlist) continue;
        const int pos = pair_off[l] + atomicAdd(&cnt[l], 1);
        pq[pos] = (int32_t)q;
        pslot[pos] = (int32_t)i;
    }
    const int64_t n_items = min<int64_t>(item_off[nlist], cap);
    for (int64_t item = tid; item < n_items; item += 1024)
        item_desc_one(item, item_off, list_order, list_off, pair_off, nlist, qpi, vch, vs, desc);
}

struct ScanArgs {
    QArgs qa;
    const int32_t *pair_off, *pair_q, *pair_slot, *item_off;
    const int4* desc;
    int64_t grid;
    int kk;
};

struct BArgs { unsigned* tau_key; int32_t* gcnt; float* gbuf_e; int32_t* gbuf_i; int32_t* work;
               int vch, dense, nprobe; int32_t* gstat; };

template <int BITS, int NQT, int PD, bool DENSE, bool LO>
hipError_t launchB_d(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    const void* kern = (const void*)scanB_kernel<BITS, NQT, PD, DENSE, LO>;
    const size_t sm = (size_t)(ix->dc + 16) * kQT * NQT;
    if (sm > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    // resident blocks only: the kernel takes items from a work counter
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, sm);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t grid = std::min<int64_t>(a.grid, (int64_t)std::max(per_cu, 1) * std::max(ncu, 1));
    hipLaunchKernelGGL((scanB_kernel<BITS, NQT, PD, DENSE, LO>), dim3((unsigned)grid), dim3(kThreads), sm, st,
                       ix->codes, ix->tile_off, ix->list_off, ix->sfac, ix->ids, ix->dc,
                       a.qa, a.pair_off, a.pair_q, a.pair_slot, a.item_off, a.desc, (int)ix->nlist,
                       a.kk, b.tau_key, b.gcnt, b.gbuf_e, b.gbuf_i, b.work, b.vch, b.nprobe);
    return hipGetLastError();
}

template <int BITS, int NQT, int PD, bool LO>
hipError_t launchB_t(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    if (b.dense) return launchB_d<BITS, NQT, PD, true, LO>(ix, a, b, st);
    return launchB_d<BITS, NQT, PD, false, LO>(ix, a, b, st);
}

template <int BITS, int NQT, bool LO = false>
hipError_t launchB_n(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    switch (scan_pd(ix)) {
        case 6:
            if constexpr (BITS <= 4) return launchB_t<BITS, NQT, 6, LO>(ix, a, b, st);
            break;
        case 4: return launchB_t<BITS, NQT, 4, LO>(ix, a, b, st);
        case 3: return launchB_t<BITS, NQT, 3, LO>(ix, a, b, st);
        case 2: return launchB_t<BITS, NQT, 2, LO>(ix, a, b, st);
        default: break;
    }
    return launchB_t<BITS, NQT, 1, LO>(ix, a, b, st);
}

template <int BITS>
hipError_t launchB_b(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    if (ix->qplanes == 2) {                         // two query planes: B >= 5 only
        if constexpr (BITS >= 5) return launchB_n<BITS, 2, true>(ix, a, b, st);
        return hipErrorInvalidValue;
    }
    // the first bound takes one query tile per item: its items hold the few
    // queries whose nearest lists coincide
    if (scan_nqt(ix) == 2 && !b.dense) return launchB_n<BITS, 2>(ix, a, b, st);
    return launchB_n<BITS, 1>(ix, a, b, st);
}

hipError_t launchB(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    switch (ix->bits) {
        case 1: return launchB_b<1>(ix, a, b, st);
        case 2: return launchB_b<2>(ix, a, b, st);
        case 3: return launchB_b<3>(ix, a, b, st);
        case 4: return launchB_b<4>(ix, a, b, st);
        case 5: return launchB_b<5>(ix, a, b, st);
        case 6: return launchB_b<6>(ix, a, b, st);
        case 7: return launchB_b<7>(ix, a, b, st);
        default: return launchB_b<8>(ix, a, b, st);
    }
}

template <int BITS, int NQT>
hipError_t launch2_n(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    const void* kern = (const void*)scan2_kernel<BITS, NQT>;
    const size_t sm = (size_t)(ix->dc + 16) * kQT * NQT;
    if (sm > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, sm);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t grid = std::min<int64_t>(a.grid, (int64_t)std::max(per_cu, 1) * std::max(ncu, 1));
    hipLaunchKernelGGL((scan2_kernel<BITS, NQT>), dim3((unsigned)grid), dim3(kThreads), sm, st,
                       ix->codes, ix->msb, ix->tile_off, ix->list_off, ix->sfac, ix->fac1, ix->ids, ix->dc,
                       a.qa, a.pair_q, a.pair_slot, a.item_off, a.desc, (int)ix->nlist,
                       b.tau_key, b.gcnt, b.gbuf_e, b.gbuf_i, b.work, ix->eps0, b.gstat);
    return hipGetLastError();
}

template <int BITS>
hipError_t launch2_b(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    if (scan_nqt(ix) == 2) return launch2_n<BITS, 2>(ix, a, b, st);
    return launch2_n<BITS, 1>(ix, a, b, st);
}

// two-stage pass B (B >= 2)
hipError_t launch2(const Index* ix, const ScanArgs& a, const BArgs& b, hipStream_t st)
{
    switch (ix->bits) {
        case 2: return launch2_b<2>(ix, a, b, st);
        case 3: return launch2_b<3>(ix, a, b, st);
        case 4: return launch2_b<4>(ix, a, b, st);
        case 5: return launch2_b<5>(ix, a, b, st);
        case 6: return launch2_b<6>(ix, a, b, st);
        case 7: return launch2_b<7>(ix, a, b, st);
        case 8: return launch2_b<8>(ix, a, b, st);
        default: return hipErrorInvalidValue;
    }
}

// slices (> 0) and the buffers: the small-batch mode of exact_kernel
struct ExactOut { int slices; int32_t* gcnt; float* gbuf_e; int32_t* gbuf_i; };

template <int BITS, bool LO>
hipError_t launch_exact_l(const Index* ix, const QArgs& qa, const int32_t* probes, int64_t nq, int nprobe, int kk,
                          const int32_t* ovf, const int32_t* gate, int32_t* redo, int64_t* oi, float* oe,
                          const ExactOut& xo, hipStream_t st)
{
    const size_t sm = sizeof(unsigned long long) * kCapE + sizeof(int) * ((nprobe + 4) & ~3) +
                      (size_t)ix->dc * (LO ? 2 : 1);
    const unsigned grid = (unsigned)std::min<int64_t>(nq * std::max(xo.slices, 1), 4096);
    hipLaunchKernelGGL((exact_kernel<BITS, LO>), dim3(grid), dim3(256), sm, st, ix->codes, ix->tile_off,
                       ix->list_off, ix->sfac, ix->ids, ix->dc, qa, probes, nq, nprobe, (int)ix->nlist, kk, ovf, gate,
                       redo, oi, oe, xo.slices, xo.gcnt, xo.gbuf_e, xo.gbuf_i);
    return hipGetLastError();
}

template <int BITS>
hipError_t launch_exact_b(const Index* ix, const QArgs& qa, const int32_t* probes, int64_t nq, int nprobe, int kk,
                          const int32_t* ovf, const int32_t* gate, int32_t* redo, int64_t* oi, float* oe,
                          const ExactOut& xo, hipStream_t st)
{
    if (ix->qplanes == 2) {
        if constexpr (BITS >= 5)
            return launch_exact_l<BITS, true>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        return hipErrorInvalidValue;
    }
    return launch_exact_l<BITS, false>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
}

// exact fallback for the flagged queries (returns at once on the device when
// the gate is 0)
hipError_t launch_exact(const Index* ix, const QArgs& qa, const int32_t* probes, int64_t nq, int nprobe, int kk,
                        const int32_t* ovf, const int32_t* gate, int32_t* redo, int64_t* oi, float* oe, hipStream_t st,
                        const ExactOut& xo = ExactOut{0, nullptr, nullptr, nullptr})
{
    if (nq <= 0) return hipSuccess;
    switch (ix->bits) {
        case 1: return launch_exact_b<1>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 2: return launch_exact_b<2>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 3: return launch_exact_b<3>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 4: return launch_exact_b<4>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 5: return launch_exact_b<5>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 6: return launch_exact_b<6>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        case 7: return launch_exact_b<7>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
        default: return launch_exact_b<8>(ix, qa, probes, nq, nprobe, kk, ovf, gate, redo, oi, oe, xo, st);
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Scan schedule: the stored value when it is valid for the index, else the
// built-in rule (two query tiles per item up to dp = 768; ring depth 6 when
// it divides the K-steps per group and the raw words are small (B <= 4),
// else the largest of 4, 3, 2, 1 that divides them; 8 ranks in round 1).
int scan_nqt(const Index* ix)
{
    if (ix->tune_nqt == 1) return 1;
    if (ix->tune_nqt == 2 && ix->dc <= kMaxDpNqt2) return 2;
    return ix->dc <= 768 ? 2 : 1;
}

bool scan_pd_valid(int pd, int dp, int bits)
{
    const int nkb = dp / 64;
    return (pd == 1 || pd == 2 || pd == 3 || pd == 4 || (pd == 6 && bits <= 4)) && nkb % pd == 0;
}

int scan_pd(const Index* ix)
{
    if (ix->tune_pd > 0 && scan_pd_valid(ix->tune_pd, ix->dc, ix->bits)) return ix->tune_pd;
    for (int pd : {6, 4, 3, 2})
        if (scan_pd_valid(pd, ix->dc, ix->bits)) return pd;
    return 1;
}

int scan_round1(const Index* ix) { return ix->tune_round1 > 0 ? ix->tune_round1 : kRound1; }
int scan_round2(const Index* ix) { return ix->tune_round2; }

hipError_t launch_scan1_fac(const uint8_t* codes_u, const int64_t* list_off, int64_t nlist, const float* cent_rot,
                            int ld, const float2* fac, const float* l1, int64_t n, int dp, int bits, float4* fac1,
                            hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan1_fac_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, codes_u, list_off,
                       (int)nlist, cent_rot, ld, fac, l1, n, dp, bits, fac1);
    return hipGetLastError();
}

hipError_t launch_scan_fac(const uint8_t* codes_u, const int64_t* list_off, int64_t nlist, const float* cent_rot,
                           const float2* fac, int64_t n, int dp, int ld, int bits, int metric, float2* sfac,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scan_fac_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, codes_u, list_off,
                       (int)nlist, cent_rot, fac, n, dp, ld, bits, metric != ERQ_METRIC_L2 ? 1 : 0, sfac);
    return hipGetLastError();
}

// items of one pair build: sum over lists of ceil(cnt/qpi) * ceil(n_l/vch) <=
// ceil(max_list/vch) * (P/kQT + nlist) for any qpi >= kQT (vch >= kVch2)
static int64_t desc_capacity(int64_t P, int64_t nlist, int64_t max_list) {
    const int64_t chunks = std::max<int64_t>(1, (max_list + kVch2 - 1) / kVch2);
    return chunks * (P / kQT + 1 + nlist);
}

size_t scan_workspace_bytes(int64_t nq, int nprobe, int64_t nlist, int kk, int dp, int64_t max_list)
{
    const int64_t P = nq * nprobe;
    size_t b = 0;
    b += align256(sizeof(int4) * desc_capacity(P, nlist, max_list));   // item descriptors
    b += 2 * align256(sizeof(int32_t) * nlist);            // cnt, fill
    b += align256(sizeof(int32_t) * kPairBlocks * nlist);  // per-block list counts
    b += 2 * align256(sizeof(int32_t) * (nlist + 1));      // pair / item offsets
    b += 2 * align256(sizeof(int32_t) * P);                // pair table (query, slot)
    b += align256(sizeof(unsigned) * nq);                  // bound per query
    b += 3 * align256(sizeof(int32_t) * nq);               // candidate counts, counts before a round, flags
    b += 3 * align256(sizeof(int32_t));                    // pass-B work counter, two overflow flags
    b += align256(sizeof(float) * nq * kCapQ);             // candidate buffers
    b += align256(sizeof(int32_t) * nq * kCapQ);
    b += align256(sizeof(int32_t) * 3);                    // fallback pairs, two-stage group counts
    b += 2 * align256((size_t)nq * dp);                    // int8 queries (high and low planes)
    b += align256(sizeof(int32_t) * nq);                   // sums of the low planes
    b += 2 * align256(sizeof(float) * nq);                 // delta/2, sum of int8 values
    b += align256(sizeof(float) * P);                      // ||s||^2 per pair
    b += align256(sizeof(int32_t) * nq);                   // flagged queries of a gated pair build
    return b;
}

int run_scan(Index* ix, const float* qrot, int64_t qld, int64_t nq, const int32_t* probes, const float* pdist,
             int nprobe, int kk, int64_t* out_ids, float* out_est, void* ws, size_t ws_bytes, hipStream_t st)
{
    const int64_t P = nq * nprobe;
    const int64_t nlist = ix->nlist;
    const int dp = ix->dc;                             // the code dimension
    if (ws_bytes < scan_workspace_bytes(nq, nprobe, nlist, kk, dp, ix->max_list))
        return fail(ERQ_ENOMEM, "erq_scan: workspace too small");
    if (nq == 0) return ERQ_OK;
    char* w = (char*)ws;
    auto take = [&](size_t bytes) { char* p = w; w += align256(bytes); return p; };
    const int64_t dcap = desc_capacity(P, nlist, ix->max_list);
    int4* desc = (int4*)take(sizeof(int4) * dcap);
    int32_t* cnt = (int32_t*)take(sizeof(int32_t) * nlist);
    int32_t* fill = (int32_t*)take(sizeof(int32_t) * nlist);
    int32_t* cnt2 = (int32_t*)take(sizeof(int32_t) * kPairBlocks * nlist);
    int32_t* poff = (int32_t*)take(sizeof(int32_t) * (nlist + 1));
    int32_t* ioff = (int32_t*)take(sizeof(int32_t) * (nlist + 1));
    int32_t* pq = (int32_t*)take(sizeof(int32_t) * P);
    int32_t* ps = (int32_t*)take(sizeof(int32_t) * P);
    unsigned* tkey = (unsigned*)take(sizeof(unsigned) * nq);
    int32_t* gcnt = (int32_t*)take(sizeof(int32_t) * nq);
    int32_t* gprev = (int32_t*)take(sizeof(int32_t) * nq);
    int32_t* ovf = (int32_t*)take(sizeof(int32_t) * nq);
    int32_t* work = (int32_t*)take(sizeof(int32_t));
    int32_t* anyf = (int32_t*)take(sizeof(int32_t));       // some query's buffer overflowed in a round
    int32_t* anyf2 = (int32_t*)take(sizeof(int32_t));      // ... at the final selection
    float* gbe = (float*)take(sizeof(float) * nq * kCapQ);
    int32_t* gbi = (int32_t*)take(sizeof(int32_t) * nq * kCapQ);
    int32_t* redo = (int32_t*)take(sizeof(int32_t) * 3);   // fallback pairs; two-stage groups, skipped
    int8_t* qint = (int8_t*)take((size_t)nq * dp);
    int8_t* qlo = (int8_t*)take((size_t)nq * dp);
    int32_t* qss_lo = (int32_t*)take(sizeof(int32_t) * nq);
    const bool lo = ix->qplanes == 2;
    float* qhd = (float*)take(sizeof(float) * nq);
    int32_t* qss = (int32_t*)take(sizeof(int32_t) * nq);
    float* sdist_ws = (float*)take(sizeof(float) * P);
    int32_t* qlist = (int32_t*)take(sizeof(int32_t) * nq);

    const int th = 256;
    auto zero = [&](int32_t* p, int64_t n) {
        if (n > 0) hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + th - 1) / th)), dim3(th), 0, st, p, n, 0);
    };
    const unsigned pblocks = (unsigned)((P + th - 1) / th);
    // pair table of the probes with rank in [rlo, rhi) (of flagged queries with
    // qmask), grouped by list; items split lists into chunks of vch members when vch > 0
    const bool lds_sort = nlist <= kHistMax;
    // the pair scan also zeroes the work counter and, for a build that is not
    // gated, both overflow flags
    // reuse: the pair table of these ranks is already built (the counts per
    // list in cnt, the pairs placed): only the items are derived again
    auto build_pairs = [&](int rlo, int rhi, const int32_t* qmask, int qpi, int vch, int vs, const int32_t* gate,
                           bool reuse = false) {
        if (gate) {                                      // usually empty: one launch
            hipLaunchKernelGGL(pair_build_gated_kernel, dim3(1), dim3(1024), 0, st, probes, nq, nprobe, (int)nlist,
                               rlo, rhi, qmask, ix->list_order, ix->list_off, qpi, vch, vs, cnt, poff, ioff, pq, ps,
                               desc, dcap, work, gate, qlist);
            return hipGetLastError();
        }
        if (reuse) {
        } else if (lds_sort) {
            hipLaunchKernelGGL(pair_hist_kernel, dim3(kPairBlocks), dim3(1024), 0, st, probes, P, nprobe,
                               (int)nlist, rlo, rhi, qmask, cnt2, gate);
            hipLaunchKernelGGL(pair_colsum_kernel, dim3((unsigned)((nlist + 63) / 64)), dim3(256), 0, st, cnt2,
                               (int)nlist, cnt, gate);
        } else {
            zero(cnt, nlist); zero(fill, nlist);
            if (P > 0)
                hipLaunchKernelGGL(pair_count_kernel, dim3(pblocks), dim3(th), 0, st, probes, P, nprobe, (int)nlist,
                                   rlo, rhi, qmask, cnt);
        }
        hipLaunchKernelGGL(pair_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, (int)nlist, ix->list_order,
                           ix->list_off, qpi, vch, vs, poff, ioff, lds_sort ? gate : nullptr, work,
                           gate ? nullptr : anyf, gate ? nullptr : anyf2);
        hipLaunchKernelGGL(item_desc_kernel, dim3((unsigned)((dcap + th - 1) / th)), dim3(th), 0, st, ioff,
                           ix->list_order, ix->list_off, poff, (int)nlist, qpi, vch, vs, dcap, desc);
        if (reuse) {
        } else if (lds_sort) {
            hipLaunchKernelGGL(pair_place_kernel, dim3(kPairBlocks), dim3(1024), 0, st, probes, P, nprobe,
                               (int)nlist, rlo, rhi, qmask, cnt2, poff, pq, ps, gate);
        } else if (P > 0) {
            hipLaunchKernelGGL(pair_scatter_kernel, dim3(pblocks), dim3(th), 0, st, probes, P, nprobe, (int)nlist,
                               rlo, rhi, qmask, poff, fill, pq, ps);
        }
        return hipGetLastError();
    };
    const size_t sel_lds = (size_t)kSelQ * sel_slots(kk) * (sizeof(float) + sizeof(int));
    auto select = [&](int mode, int post, int64_t* oi, float* oe) {
        const dim3 grid((unsigned)((nq + kSelQ - 1) / kSelQ));
        if (mode == 1)
            hipLaunchKernelGGL(buf_select_kernel<1>, grid, dim3(256), sel_lds, st, gcnt, gprev, gbe, gbi, nq, kk,
                               post, tkey, ovf, oi, oe, anyf2);
        else if (mode == 2)
            hipLaunchKernelGGL(buf_select_kernel<2>, grid, dim3(256), 0, st, gcnt, gprev, gbe, gbi, nq, kk, post,
                               tkey, ovf, oi, oe, anyf);
        else
            hipLaunchKernelGGL(buf_select_kernel<0>, grid, dim3(256), 0, st, gcnt, gprev, gbe, gbi, nq, kk, post,
                               tkey, ovf, oi, oe, anyf);
        return hipGetLastError();
    };
    const int qpiB = ix->qplanes == 2 ? kQT : scan_nqt(ix) * kQT;   // queries per item of the launched kernel
    const int pr = prof_begin(PK_SCAN, st);
    hipError_t e = hipSuccess;
    // queries to int8 once; ||s||^2 per pair from the probe distances, else computed
    hipLaunchKernelGGL(qprep_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, qrot, nq, dp, (int)qld, qint,
                       qhd, qss, lo ? qlo : nullptr, lo ? qss_lo : nullptr);
    const float* sdist = pdist;
    const bool ip = ix->metric != ERQ_METRIC_L2;
    if (!sdist && P > 0) {
        if (ip)
            hipLaunchKernelGGL(pair_s2_kernel<true>, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, st, qrot,
                               ix->cent_rot, probes, P, nprobe, (int)nlist, ix->dp, sdist_ws);
        else
            hipLaunchKernelGGL(pair_s2_kernel<false>, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, st, qrot,
                               ix->cent_rot, probes, P, nprobe, (int)nlist, ix->dp, sdist_ws);
        sdist = sdist_ws;
    }
    const QArgs qa{qint, qhd, qss, sdist, ip ? -__builtin_huge_valf() : 0.0f, lo ? qlo : nullptr,
                   lo ? qss_lo : nullptr};
    // Small batches (at most ix->small_q queries): the pair-grouped pipeline
    // (first bound, rounds, selects; about 35 launches) is set by its launch
    // count, not by work.  Each query's probed lists are instead split over S
    // workgroups that keep exact top-kk lists (exact_kernel, slice mode), and
    // one final select merges them: the same exact top-kk by (est, id).
    // With S below 16 (kk > 256 at nprobe >= 16) each workgroup would keep a
    // long exact list over a large share of the probed members; such calls
    // take the pipeline.
    const int small_s = std::min(std::min(nprobe, kSmallS), std::max(1, kCapQ / kk));
    if (nq <= ix->small_q && small_s >= std::min(nprobe, 16)) {
        const int pc = prof_begin(PK_SCAN_C, st);
        zero(gcnt, nq);
        hipError_t e = launch_exact(ix, qa, probes, nq, nprobe, kk, nullptr, nullptr, nullptr, nullptr, nullptr, st,
                                    ExactOut{small_s, gcnt, gbe, gbi});
        if (e == hipSuccess) {
            const size_t sel_lds0 = (size_t)kSelQ * sel_slots(kk) * (sizeof(float) + sizeof(int));
            hipLaunchKernelGGL(buf_select_kernel<1>, dim3((unsigned)((nq + kSelQ - 1) / kSelQ)), dim3(256), sel_lds0,
                               st, gcnt, gprev, gbe, gbi, nq, kk, 0, tkey, ovf, out_ids, out_est, anyf2);
            e = hipGetLastError();
        }
        prof_end(pc, st);
        prof_end(pr, st);
        if (e != hipSuccess) return fail(ERQ_EDEVICE, std::string("scan launch: ") + hipGetErrorString(e));
        return ERQ_OK;
    }
    const int64_t gridB = 1 << 20;                    // capped at the resident blocks
    // a pass-B launch over the pairs of probe ranks [rlo, rhi) (of flagged
    // queries with qmask); dense = the first-bound mode
    // the two-stage scan (Sec. 4.2) replaces pass B when the index has its 1-bit data and eps0 > 0
    const bool two = ix->eps0 > 0.0f && ix->msb && ix->fac1 && ix->qplanes == 1;
    // vs: members [0, vs) of every list are skipped (the first round after
    // the first bound, whose estimates of those members are kept)
    auto scan_round = [&](int rlo, int rhi, const int32_t* qmask, int dense, const int32_t* gate, int vs,
                          bool reuse = false) {
        const int vch = dense ? 0 : (two ? kVch2 : kVch);
        const int qpi = (dense && ix->qplanes != 2) ? kQT : qpiB;   // queries per item of the launched kernel
        hipError_t er = build_pairs(rlo, rhi, qmask, qpi, vch, dense ? 0 : vs, gate, reuse);
        if (er != hipSuccess) return er;
        ScanArgs b{qa, poff, pq, ps, ioff, desc, gridB, kk};
        BArgs bb{tkey, gcnt, gbe, gbi, work, vch, dense, nprobe, prof_stats_on() ? redo + 1 : nullptr};
        const int rec = prof_begin(dense ? PK_SCAN_A : PK_SCAN_B, st);   // one record per launch
        er = (two && !dense) ? launch2(ix, b, bb, st) : launchB(ix, b, bb, st);
        prof_end(rec, st);
        return er;
    };
    // first bound: all estimates of the first kDenseV members of the r0
    // nearest lists, in fixed buffer slots (+inf where a list is shorter)
    const int r0 = std::min(nprobe, kDenseR);
    hipLaunchKernelGGL(fill_dense_kernel, dim3((unsigned)((nq * kDenseR * kDenseV / 4 + th - 1) / th)), dim3(th), 0,
                       st, gbe, nq, gcnt, tkey, redo);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_round(0, r0, nullptr, 1, nullptr, 0);
    // bound; the buffer keeps the dense estimates at or under it (padding
    // dropped), so the first round skips the members [0, kDenseV) of the r0
    // nearest lists instead of estimating them again
    if (e == hipSuccess) e = select(0, 3, nullptr, nullptr);
    // pass B in rounds of increasing probe rank: [0, r0) (the first bound's
    // ranks, members past kDenseV only), [r0, round1) when round1 > r0,
    // [round1, round2) when round2 lies between round1 and nprobe, and the
    // rest.  Without a middle round, the rest is cut further while the
    // candidates it would let through exceed three quarters of what a
    // candidate buffer holds beside the kk kept (a bound taken from hi ranks
    // lets about kk * (rest / hi) candidates of the rest through): the next
    // round ends at g * hi, g = 16 halved until kk * (g - 1) <= kCapQ / 4.  At
    // nprobe 84 and kk 24 this keeps one round after the first; at nprobe
    // 1024 and kk 200 it gives [0, 4), [4, 16), [16, 64), [64, 256),
    // [256, 1024).  The count before each round is recorded by the select
    // before it.
    const int r1 = std::max(r0, std::min(nprobe, scan_round1(ix))), r2 = scan_round2(ix);
    int bounds[16] = {0, r0}, nround = 1;
    if (r1 > r0) bounds[++nround] = r1;
    if (r2 > r1 && r2 < nprobe) {
        bounds[++nround] = r2;
    } else {
        int g = 16;
        while (g > 2 && (int64_t)kk * (g - 1) > kCapQ / 4) g >>= 1;
        for (int hi = r1; hi > 0 && nround < 12 && (int64_t)4 * kk * (nprobe - hi) > (int64_t)3 * (kCapQ - kk) * hi;) {
            hi *= g;
            if (hi >= nprobe) break;
            bounds[++nround] = hi;
        }
    }
    bounds[++nround] = nprobe;
    for (int r = 0; r < nround && e == hipSuccess; ++r) {
        const int rlo = bounds[r], rhi = bounds[r + 1];
        if (rhi <= rlo) continue;
        const int vs = r == 0 ? kDenseV : 0;
        // the first round has the first bound's ranks: its pair table is reused
        e = scan_round(rlo, rhi, nullptr, 0, nullptr, vs, r == 0);   // its pair scan zeroes both flags
        // queries that overflowed: back to their count before the round, tighter bound, rescan the
        // round (skipped on the device when no query overflowed)
        if (e == hipSuccess) e = select(2, 0, nullptr, nullptr);
        if (e == hipSuccess) e = scan_round(rlo, rhi, ovf, 0, anyf, vs);
        if (e == hipSuccess && rhi < nprobe) e = select(0, 2, nullptr, nullptr);
    }
    // exact top-kk per query; queries whose buffer still overflowed: the exact fallback
    const int pc = prof_begin(PK_SCAN_C, st);
    if (e == hipSuccess) e = select(1, 0, out_ids, out_est);
    if (e == hipSuccess) e = launch_exact(ix, qa, probes, nq, nprobe, kk, ovf, anyf2, redo, out_ids, out_est, st);
    prof_end(pc, st);
    prof_end(pr, st);
    if (e != hipSuccess) return fail(ERQ_EDEVICE, std::string("scan launch: ") + hipGetErrorString(e));
    prof_note_redo(redo, st);               // pairs scanned by the exact fallback
    return ERQ_OK;
}

}  // namespace erq
