// IVF scan of Extended RaBitQ codes on the int8 matrix cores (Sec. 3.3,
// Sec. 4.1), in three steps per query batch:
//
//  1. pair build: (query, list) pairs of the probe table grouped by list
//     (count, exclusive scan, scatter); the work items are (list, tile of up
//     to 32 of its queries), enumerated longest list first.
//  2. scan: one workgroup (4 waves) per work item.  Prologue: for each of
//     its queries s' = q' - c' (FP32), int8 quantisation (symmetric, scale
//     max|s'|/127), ||s'||^2 and sum(s_int), written to LDS in the layout of
//     the B operand of v_mfma_i32_32x32x32_i8.  Main loop: every wave takes
//     32-vector code tiles of the list, unpacks the packed B-bit codes to
//     int8 in registers and accumulates <y_u, s_int> exactly in int32.
//     Epilogue: est = f_add + ||s||^2 + f_rescale * delta/2 *
//     (2 <y_u, s_int> - (2^B - 1) sum s_int)  (Eq. eq:dis to ip with Eq.
//     eq 3.3: represent), kept per lane in a sorted register list of the best
//     KK (est, id) with a threshold shared through LDS; the lists of the
//     8 lanes that saw a query are merged into its top-kk for this list.
//  3. merge: per query, the kk best over its probed lists.
#include "erq_common.h"

namespace erq {

namespace {

constexpr int kThreads = 256;
constexpr int kQT = 32;        // queries per work item (columns of the MFMA tile)

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

template <int KK>
__device__ inline void insert_sorted(float* le, int* li, float e, int i) {
#pragma unroll
    for (int t = 0; t < KK; ++t) {
        bool sw = lt(e, i, le[t], li[t]);
        float te = le[t]; int ti = li[t];
        le[t] = sw ? e : te; li[t] = sw ? i : ti;
        e = sw ? te : e; i = sw ? ti : i;
    }
}

template <int KK>
__device__ inline float kth_of(const float* le, int kk) {
    float c = le[KK - 1];
#pragma unroll
    for (int t = 0; t < KK; ++t) c = (t == kk - 1) ? le[t] : c;
    return c;
}

// ---------------------------------------------------------------------------
template <int BITS, int KK>
__global__ __launch_bounds__(kThreads, 2) void scan_kernel(
    const uint8_t* __restrict__ codes, const int64_t* __restrict__ tile_off,
    const int64_t* __restrict__ list_off, const float2* __restrict__ fac,
    const int64_t* __restrict__ ids, const float* __restrict__ cent_rot, int dp,
    const float* __restrict__ qrot, const int32_t* __restrict__ pair_off,
    const int32_t* __restrict__ pair_q, const int32_t* __restrict__ pair_slot,
    const int32_t* __restrict__ item_off, const int32_t* __restrict__ list_order, int nlist,
    int kk, float* __restrict__ res_est, int32_t* __restrict__ res_id)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ float s_s2[kQT], s_hd[kQT];
    __shared__ int s_ss[kQT], s_slot[kQT];
    __shared__ unsigned s_thr[kQT];
    __shared__ int s_item[2];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int item = blockIdx.x;
    if (item >= item_off[nlist]) return;
    if (tid == 0) {
        int lo = 0, hi = nlist;                    // largest r with item_off[r] <= item
        while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (item_off[mid] <= item) lo = mid; else hi = mid; }
        while (lo + 1 < nlist && item_off[lo + 1] <= item) ++lo;
        s_item[0] = list_order[lo];
        s_item[1] = item - item_off[lo];
    }
    if (tid < kQT) s_thr[tid] = 0xFFFFFFFFu;
    __syncthreads();
    const int l = s_item[0];
    const int qtile = s_item[1];
    const int p0 = pair_off[l] + qtile * kQT;
    const int mq = min(kQT, pair_off[l + 1] - p0);
    const int nkb = dp / 64;
    int8_t* qs = (int8_t*)smem;                  // B operand: (ks*64 + lane) * 16 bytes

    // ---- prologue: int8 residual queries ---------------------------------
    {
        const float* cv = cent_rot + (int64_t)l * dp;
        const int nch = dp / 16;                  // 16-dim chunks
        for (int jj = wid; jj < kQT; jj += 4) {
            if (jj >= mq) {
                for (int c = lane; c < nch; c += 64) {
                    const int ks = c >> 1, h = c & 1;
                    *(uint4*)(qs + ((ks * 2 + h) * kQT + jj) * 16) = make_uint4(0, 0, 0, 0);
                }
                continue;
            }
            const int q = pair_q[p0 + jj];
            const float* qv = qrot + (int64_t)q * dp;
            float sv[4][16];
            float amax = 0.0f, s2 = 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = lane + 64 * u;
                if (c < nch) {
#pragma unroll
                    for (int e = 0; e < 16; e += 4) {
                        float4 a = *(const float4*)(qv + c * 16 + e);
                        float4 b = *(const float4*)(cv + c * 16 + e);
                        sv[u][e + 0] = a.x - b.x; sv[u][e + 1] = a.y - b.y;
                        sv[u][e + 2] = a.z - b.z; sv[u][e + 3] = a.w - b.w;
                    }
#pragma unroll
                    for (int e = 0; e < 16; ++e) { amax = fmaxf(amax, fabsf(sv[u][e])); s2 += sv[u][e] * sv[u][e]; }
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                amax = fmaxf(amax, __shfl_xor(amax, o));
                s2 += __shfl_xor(s2, o);
            }
            const float inv = (amax > 0.0f) ? __fdiv_rn(127.0f, amax) : 0.0f;
            int ssum = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = lane + 64 * u;
                if (c < nch) {
                    uint32_t w4[4];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        uint32_t wd = 0;
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            int v = (int)rintf(sv[u][4 * d + b] * inv);
                            v = max(-127, min(127, v));
                            ssum += v;
                            wd |= ((uint32_t)(v & 0xFF)) << (8 * b);
                        }
                        w4[d] = wd;
                    }
                    const int ks = c >> 1, h = c & 1;
                    *(uint4*)(qs + ((ks * 2 + h) * kQT + jj) * 16) = make_uint4(w4[0], w4[1], w4[2], w4[3]);
                }
            }
            for (int o = 32; o > 0; o >>= 1) ssum += __shfl_xor(ssum, o);
            if (lane == 0) {
                s_s2[jj] = s2;
                s_hd[jj] = 0.5f * ((amax > 0.0f) ? __fdiv_rn(amax, 127.0f) : 0.0f);
                s_ss[jj] = ssum;
                s_slot[jj] = pair_slot[p0 + jj];
            }
        }
    }
    __syncthreads();

    // ---- main loop -------------------------------------------------------------
    constexpr int corr = 2 * (BITS == 8 ? 128 : 0) - ((1 << BITS) - 1);
    const int j = lane & 31;                     // query column of this lane
    const bool qvalid = j < mq;
    const float qs2 = qvalid ? s_s2[j] : 0.0f;
    const float qhd = qvalid ? s_hd[j] : 0.0f;
    const int qss = qvalid ? s_ss[j] : 0;
    float le[KK];
    int li[KK];
#pragma unroll
    for (int t = 0; t < KK; ++t) { le[t] = __builtin_huge_valf(); li[t] = 0x7FFFFFFF; }
    float cut = __builtin_huge_valf();

    const int64_t lbase = list_off[l];
    const int nl = (int)(list_off[l + 1] - lbase);
    const int ntile = (nl + 31) >> 5;
    const int64_t tbase = tile_off[l];
    const int64_t tile_bytes = (int64_t)4 * dp * BITS;
    const v4i* qb = (const v4i*)qs;

    for (int tt = wid; tt < ntile; tt += 4) {
        const uint8_t* tp = codes + (tbase + tt) * tile_bytes;
        v16i acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0;
        for (int kb = 0; kb < nkb; ++kb) {
            v4i a0, a1;
            load_codes<BITS>(tp + (int64_t)kb * 256 * BITS, lane, a0, a1);
            v4i b0 = qb[(kb * 2 + 0) * 64 + lane];
            v4i b1 = qb[(kb * 2 + 1) * 64 + lane];
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc, 0, 0, 0);
        }
        // epilogue
        const float shared_cut = key2f(s_thr[j]);
        const float c0 = fminf(cut, shared_cut);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int v = tt * 32 + row;
            const bool ok = qvalid && v < nl;
            float est = __builtin_huge_valf();
            if (ok) {
                float2 f = fac[lbase + v];
                const int ip2 = 2 * acc[r] + corr * qss;
                est = (f.x + qs2) + f.y * (qhd * (float)ip2);
            }
            const bool pass = ok && est <= c0;
            if (__any(pass)) {
                int id = 0x7FFFFFFF;
                if (pass) id = (int)ids[lbase + v];
                else est = __builtin_huge_valf();
                insert_sorted<KK>(le, li, est, id);
            }
        }
        cut = kth_of<KK>(le, kk);
        if (qvalid && cut < __builtin_huge_valf()) atomicMin(&s_thr[j], f2key(cut));
    }
    __syncthreads();                           // done with the B operand: reuse LDS

    // ---- merge the 8 lane lists of every query -----------------------------------
    // lanes j and j+32 of a wave hold the same query: keep the KK smallest of both
    {
        float oe[KK]; int oi[KK];
#pragma unroll
        for (int t = 0; t < KK; ++t) { oe[t] = __shfl_xor(le[t], 32); oi[t] = __shfl_xor(li[t], 32); }
        // smallest KK of two sorted lists: min(le[t], oe[KK-1-t]) is bitonic, then sort
#pragma unroll
        for (int t = 0; t < KK; ++t) {
            bool take = lt(oe[KK - 1 - t], oi[KK - 1 - t], le[t], li[t]);
            float e = take ? oe[KK - 1 - t] : le[t];
            int i = take ? oi[KK - 1 - t] : li[t];
            le[t] = e; li[t] = i;
        }
#pragma unroll
        for (int jj = KK / 2; jj > 0; jj >>= 1) {
#pragma unroll
            for (int t = 0; t < KK; ++t) {
                if ((t & jj) == 0) {
                    const int p = t + jj;
                    if (lt(le[p], li[p], le[t], li[t])) {
                        float e = le[t]; le[t] = le[p]; le[p] = e;
                        int i = li[t]; li[t] = li[p]; li[p] = i;
                    }
                }
            }
        }
    }
    float* me = (float*)smem;                         // [4][32][KK]
    int* mi = (int*)(smem + sizeof(float) * 4 * kQT * KK);
    if (lane < 32) {
#pragma unroll
        for (int t = 0; t < KK; ++t) {
            me[(wid * kQT + lane) * KK + t] = le[t];
            mi[(wid * kQT + lane) * KK + t] = li[t];
        }
    }
    __syncthreads();
    if (tid < mq) {
        int h[4] = {0, 0, 0, 0};
        const int slot = s_slot[tid];
        for (int o = 0; o < kk; ++o) {
            int bw = 0;
            float be = me[(0 * kQT + tid) * KK + h[0]];
            int bi = mi[(0 * kQT + tid) * KK + h[0]];
            for (int w = 1; w < 4; ++w) {
                float e = me[(w * kQT + tid) * KK + h[w]];
                int i = mi[(w * kQT + tid) * KK + h[w]];
                if (lt(e, i, be, bi)) { be = e; bi = i; bw = w; }
            }
            if (h[bw] < KK - 1) ++h[bw];
            else { me[(bw * kQT + tid) * KK + h[bw]] = __builtin_huge_valf(); mi[(bw * kQT + tid) * KK + h[bw]] = 0x7FFFFFFF; }
            res_est[(int64_t)slot * kk + o] = be;
            res_id[(int64_t)slot * kk + o] = (be < __builtin_huge_valf()) ? bi : -1;
        }
    }
}

// ---------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void pair_count_kernel(const int32_t* __restrict__ probes, int64_t np, int nlist,
                                  int32_t* __restrict__ cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int l = probes[i];
    if (l >= 0 && l < nlist) atomicAdd(&cnt[l], 1);
}

// single workgroup: pair_off (by list id) and item_off (by rank of list_order)
__global__ __launch_bounds__(1024) void pair_scan_kernel(const int32_t* __restrict__ cnt, int nlist,
                                                         const int32_t* __restrict__ list_order,
                                                         int32_t* __restrict__ pair_off,
                                                         int32_t* __restrict__ item_off)
{
    __shared__ int part_a[1024], part_b[1024];
    const int tid = threadIdx.x;
    const int chunk = (nlist + 1023) / 1024;
    const int beg = tid * chunk, end = min(nlist, beg + chunk);
    int sa = 0, sb = 0;
    for (int i = beg; i < end; ++i) { sa += cnt[i]; sb += (cnt[list_order[i]] + kQT - 1) / kQT; }
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
        item_off[i] = rb; rb += (cnt[list_order[i]] + kQT - 1) / kQT;
    }
    if (tid == 1023) { pair_off[nlist] = part_a[1023]; item_off[nlist] = part_b[1023]; }
}

__global__ void pair_scatter_kernel(const int32_t* __restrict__ probes, int64_t np, int nprobe, int nlist,
                                    const int32_t* __restrict__ pair_off, int32_t* __restrict__ fill,
                                    int32_t* __restrict__ pair_q, int32_t* __restrict__ pair_slot)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int l = probes[i];
    if (l < 0 || l >= nlist) return;
    int pos = pair_off[l] + atomicAdd(&fill[l], 1);
    pair_q[pos] = (int32_t)(i / nprobe);
    pair_slot[pos] = (int32_t)i;
}

// one wave per query: the kk best of its probed lists' top-kk lists
__global__ __launch_bounds__(256) void merge_kernel(const int32_t* __restrict__ probes, int64_t nq, int nprobe,
                                                    int nlist, int kk, const float* __restrict__ res_est,
                                                    const int32_t* __restrict__ res_id,
                                                    int64_t* __restrict__ out_ids, float* __restrict__ out_est)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    constexpr int U = 16;                 // nprobe <= 1024
    int hp[U];
    float he[U];
    int hi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = lane + 64 * u;
        hp[u] = 0;
        he[u] = __builtin_huge_valf();
        hi[u] = 0x7FFFFFFF;
        if (p < nprobe) {
            int l = probes[q * nprobe + p];
            if (l >= 0 && l < nlist) {
                const int64_t s = q * nprobe + p;
                he[u] = res_est[s * kk];
                int id = res_id[s * kk];
                hi[u] = id < 0 ? 0x7FFFFFFF : id;
                if (id < 0) he[u] = __builtin_huge_valf();
            }
        }
    }
    for (int o = 0; o < kk; ++o) {
        float be = __builtin_huge_valf();
        int bi = 0x7FFFFFFF, bu = -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (lt(he[u], hi[u], be, bi)) { be = he[u]; bi = hi[u]; bu = u; }
        float ge = be; int gi = bi; int gl = lane;
        for (int off = 32; off > 0; off >>= 1) {
            float oe = __shfl_xor(ge, off);
            int oi = __shfl_xor(gi, off);
            int ol = __shfl_xor(gl, off);
            if (lt(oe, oi, ge, gi) || (oe == ge && oi == gi && ol < gl)) { ge = oe; gi = oi; gl = ol; }
        }
        if (lane == 0) {
            const bool valid = ge < __builtin_huge_valf();
            out_ids[q * kk + o] = valid ? (int64_t)gi : -1;
            out_est[q * kk + o] = valid ? ge : __builtin_huge_valf();
        }
        if (lane == gl && bu >= 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (u == bu) {
                    const int64_t s = q * nprobe + lane + 64 * u;
                    hp[u] += 1;
                    if (hp[u] < kk) {
                        int id = res_id[s * kk + hp[u]];
                        he[u] = id < 0 ? __builtin_huge_valf() : res_est[s * kk + hp[u]];
                        hi[u] = id < 0 ? 0x7FFFFFFF : id;
                    } else {
                        he[u] = __builtin_huge_valf();
                        hi[u] = 0x7FFFFFFF;
                    }
                }
            }
        }
    }
}

template <int BITS, int KK>
hipError_t launch_scan_t(const Index* ix, const float* qrot, const int32_t* pair_off, const int32_t* pair_q,
                         const int32_t* pair_slot, const int32_t* item_off, int64_t max_items, int kk,
                         float* res_est, int32_t* res_id, hipStream_t st)
{
    size_t sm = (size_t)ix->dp * 32;
    size_t mb = (size_t)4 * kQT * KK * 8;
    if (mb > sm) sm = mb;
    if (sm > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)scan_kernel<BITS, KK>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((scan_kernel<BITS, KK>), dim3((unsigned)max_items), dim3(kThreads), sm, st,
                       ix->codes, ix->tile_off, ix->list_off, ix->fac, ix->ids, ix->cent_rot, ix->dp,
                       qrot, pair_off, pair_q, pair_slot, item_off, ix->list_order, (int)ix->nlist,
                       kk, res_est, res_id);
    return hipGetLastError();
}

template <int BITS>
hipError_t launch_scan_b(const Index* ix, const float* qrot, const int32_t* pair_off, const int32_t* pair_q,
                         const int32_t* pair_slot, const int32_t* item_off, int64_t max_items, int kk,
                         float* res_est, int32_t* res_id, hipStream_t st)
{
    if (kk <= 16) return launch_scan_t<BITS, 16>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st);
    if (kk <= 32) return launch_scan_t<BITS, 32>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st);
    return launch_scan_t<BITS, 64>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t scan_workspace_bytes(int64_t nq, int nprobe, int64_t nlist, int kk)
{
    const int64_t P = nq * nprobe;
    size_t b = 0;
    b += align256(sizeof(int32_t) * nlist);            // cnt
    b += align256(sizeof(int32_t) * nlist);            // fill
    b += align256(sizeof(int32_t) * (nlist + 1));      // pair_off
    b += align256(sizeof(int32_t) * (nlist + 1));      // item_off
    b += align256(sizeof(int32_t) * P);                // pair_q
    b += align256(sizeof(int32_t) * P);                // pair_slot
    b += align256(sizeof(float) * P * kk);             // res_est
    b += align256(sizeof(int32_t) * P * kk);           // res_id
    return b;
}

int run_scan(Index* ix, const float* qrot, int64_t nq, const int32_t* probes, int nprobe, int kk,
             int64_t* out_ids, float* out_est, void* ws, size_t ws_bytes, hipStream_t st)
{
    const int64_t P = nq * nprobe;
    const int64_t nlist = ix->nlist;
    if (ws_bytes < scan_workspace_bytes(nq, nprobe, nlist, kk))
        return fail(ERQ_ENOMEM, "erq_scan: workspace too small");
    char* w = (char*)ws;
    auto take = [&](size_t bytes) { char* p = w; w += align256(bytes); return p; };
    int32_t* cnt = (int32_t*)take(sizeof(int32_t) * nlist);
    int32_t* fill = (int32_t*)take(sizeof(int32_t) * nlist);
    int32_t* pair_off = (int32_t*)take(sizeof(int32_t) * (nlist + 1));
    int32_t* item_off = (int32_t*)take(sizeof(int32_t) * (nlist + 1));
    int32_t* pair_q = (int32_t*)take(sizeof(int32_t) * P);
    int32_t* pair_slot = (int32_t*)take(sizeof(int32_t) * P);
    float* res_est = (float*)take(sizeof(float) * P * kk);
    int32_t* res_id = (int32_t*)take(sizeof(int32_t) * P * kk);

    const int th = 256;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((nlist + th - 1) / th)), dim3(th), 0, st, fill, nlist, 0);
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((nlist + th - 1) / th)), dim3(th), 0, st, cnt, nlist, 0);
    if (P > 0) {
        hipLaunchKernelGGL(pair_count_kernel, dim3((unsigned)((P + th - 1) / th)), dim3(th), 0, st,
                           probes, P, (int)nlist, cnt);
    }
    hipLaunchKernelGGL(pair_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, (int)nlist, ix->list_order,
                       pair_off, item_off);
    if (P > 0) {
        hipLaunchKernelGGL(pair_scatter_kernel, dim3((unsigned)((P + th - 1) / th)), dim3(th), 0, st,
                           probes, P, nprobe, (int)nlist, pair_off, fill, pair_q, pair_slot);
    }
    ERQ_HIP(hipGetLastError());
    const int64_t max_items = (P + kQT - 1) / kQT + nlist;
    hipError_t e = hipSuccess;
    const int pr = prof_begin(PK_SCAN, st);
    if (P > 0) {
        switch (ix->bits) {
            case 1: e = launch_scan_b<1>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 2: e = launch_scan_b<2>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 3: e = launch_scan_b<3>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 4: e = launch_scan_b<4>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 5: e = launch_scan_b<5>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 6: e = launch_scan_b<6>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            case 7: e = launch_scan_b<7>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
            default: e = launch_scan_b<8>(ix, qrot, pair_off, pair_q, pair_slot, item_off, max_items, kk, res_est, res_id, st); break;
        }
    }
    prof_end(pr, st);
    if (e != hipSuccess) return fail(ERQ_EDEVICE, std::string("scan launch: ") + hipGetErrorString(e));
    const int pm = prof_begin(PK_MERGE, st);
    if (nq > 0) {
        hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, probes, nq, nprobe,
                           (int)nlist, kk, res_est, res_id, out_ids, out_est);
    }
    prof_end(pm, st);
    ERQ_HIP(hipGetLastError());
    return ERQ_OK;
}

}  // namespace erq
