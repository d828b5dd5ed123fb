// Selection and list building:
//  * row_topk: the k smallest entries of each row of a distance matrix,
//    ascending by (value, column) -- the nprobe nearest centroids of the IVF
//    probe (Sec. 4.1) and the nearest centroid of a k-means assignment.
//    Exact radix select on the order-preserving integer image of the floats
//    (4 passes of 8 bits), then a stable compaction and a bitonic sort.
//  * IVF list construction: the member count of every list.
//  * residuals r = x - c and ||r||^2 (FP64 accumulate) in list order.
#include "erq_common.h"

namespace erq {

namespace {

__device__ inline unsigned f2key(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kSelThreads = 256;
constexpr int kSelMaxK = 1024;

// R > 0: thread t keeps keys [t*R, t*R + R) of the row in registers (N <=
// 256*R), so the row is read from memory once; R == 0: every pass reads the
// row from memory.  Both use contiguous per-thread chunks, which keeps the
// compaction stable (ties in value go by column index).
template <int R>
__global__ __launch_bounds__(kSelThreads) void row_topk_kernel(
    const float* __restrict__ D, int64_t N, int k, int32_t* __restrict__ oidx, float* __restrict__ oval)
{
    __shared__ unsigned hist[256];
    __shared__ unsigned skey[kSelMaxK];
    __shared__ int sidx[kSelMaxK];
    __shared__ unsigned scan_l[kSelThreads / 64], scan_e[kSelThreads / 64];
    __shared__ unsigned s_digit, s_kr, s_wsum[kSelThreads / 64];
    const int tid = threadIdx.x;
    const int64_t row = blockIdx.x;
    const float* d = D + row * N;
    const int kk = (int)min<int64_t>(k, N);
    const int64_t chunk = R > 0 ? R : (N + kSelThreads - 1) / kSelThreads;
    const int64_t beg = min<int64_t>(N, tid * chunk), end = min(N, beg + chunk);
    constexpr int RR = R > 0 ? R : 1;
    unsigned kreg[RR];
    if constexpr (R > 0) {
        if (end - beg == R && ((uintptr_t)(d + beg) & 15) == 0) {
            // a whole chunk: 16-byte loads, 64 contiguous bytes per thread
            static_assert(R % 4 == 0, "chunks of whole float4s");
#pragma unroll
            for (int u = 0; u < R; u += 4) {
                const float4 v = *(const float4*)(d + beg + u);
                kreg[u] = f2key(v.x); kreg[u + 1] = f2key(v.y); kreg[u + 2] = f2key(v.z); kreg[u + 3] = f2key(v.w);
            }
        } else {
#pragma unroll
            for (int u = 0; u < R; ++u) kreg[u] = (beg + u < end) ? f2key(d[beg + u]) : 0u;
        }
    }
    auto key_at = [&](int64_t j, int u) -> unsigned {
        if constexpr (R > 0) return kreg[u];
        else return f2key(d[j]);
    };
    unsigned prefix = 0, mask = 0;
    unsigned kr = (unsigned)kk;                 // rank (1-based) still to locate
    for (int pass = 0; pass < 4 && kk > 0; ++pass) {
        const int shift = 24 - 8 * pass;
        hist[tid] = 0;
        __syncthreads();
        // runs of equal digits are counted in a register first: the leading
        // digit of similar distances is nearly constant, and one LDS bin hit
        // by every thread would serialise the atomics
        unsigned run_d = 0xFFFFFFFFu, run_n = 0;
#pragma unroll
        for (int u = 0; u < RR; ++u) {
            for (int64_t j = beg + u; j < end; j += RR) {
                const unsigned key = key_at(j, u);
                if ((key & mask) == prefix) {
                    const unsigned dg = (key >> shift) & 0xFF;
                    if (dg != run_d) {
                        if (run_n) atomicAdd(&hist[run_d], run_n);
                        run_d = dg; run_n = 0;
                    }
                    ++run_n;
                }
                if (R > 0) break;
            }
        }
        if (run_n) atomicAdd(&hist[run_d], run_n);
        __syncthreads();
        // bin of the kr-th smallest: one bin per thread, block-wide prefix sum
        {
            const int lane = tid & 63, wid = tid >> 6;
            const unsigned v = hist[tid];
            unsigned x = v;
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_wsum[wid] = x;
            __syncthreads();
            unsigned base = 0;
            for (int w = 0; w < wid; ++w) base += s_wsum[w];
            const unsigned incl = base + x, excl = incl - v;
            if (excl < kr && kr <= incl) { s_digit = (unsigned)tid; s_kr = kr - excl; }
            __syncthreads();
        }
        prefix |= s_digit << shift;
        kr = s_kr;
        mask |= 0xFFu << shift;
    }
    const unsigned kth = prefix;                // key of the k-th smallest
    const unsigned need_eq = kr;                // how many equal to kth are taken
    // stable compaction over the contiguous chunks
    unsigned nl = 0, ne = 0;
#pragma unroll
    for (int u = 0; u < RR; ++u) {
        for (int64_t j = beg + u; j < end; j += RR) {
            const unsigned key = key_at(j, u);
            nl += key < kth;
            ne += key == kth;
            if (R > 0) break;
        }
    }
    // exclusive prefix sums of both counts over the threads (chunk order)
    unsigned pl, pe;
    {
        const int lane = tid & 63, wid = tid >> 6;
        unsigned x = nl, y = ne;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned xu = __shfl_up(x, o), yu = __shfl_up(y, o);
            if (lane >= o) { x += xu; y += yu; }
        }
        if (lane == 63) { scan_l[wid] = x; scan_e[wid] = y; }
        __syncthreads();
        unsigned bl = 0, be = 0;
        for (int w = 0; w < wid; ++w) { bl += scan_l[w]; be += scan_e[w]; }
        pl = bl + x - nl;
        pe = be + y - ne;
    }
    const unsigned nless = (unsigned)kk - need_eq;
    if (kk > 0) {
#pragma unroll
        for (int u = 0; u < RR; ++u) {
            for (int64_t j = beg + u; j < end; j += RR) {
                const unsigned key = key_at(j, u);
                if (key < kth) { skey[pl] = key; sidx[pl] = (int)j; ++pl; }
                else if (key == kth) {
                    if (pe < need_eq) { skey[nless + pe] = key; sidx[nless + pe] = (int)j; }
                    ++pe;
                }
                if (R > 0) break;
            }
        }
    }
    int S = 1;
    while (S < kk) S <<= 1;
    for (int t = kk + tid; t < S; t += kSelThreads) { skey[t] = 0xFFFFFFFFu; sidx[t] = 0x7FFFFFFF; }
    for (int kb = 2; kb <= S; kb <<= 1)
        for (int j = kb >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int t = tid; t < S / 2; t += kSelThreads) {
                int i = 2 * t - (t & (j - 1)), p = i + j;
                bool up = (i & kb) == 0;
                unsigned k0 = skey[i], k1 = skey[p];
                int i0 = sidx[i], i1 = sidx[p];
                bool first0 = k0 < k1 || (k0 == k1 && i0 < i1);
                if (first0 != up) { skey[i] = k1; skey[p] = k0; sidx[i] = i1; sidx[p] = i0; }
            }
        }
    __syncthreads();
    for (int t = tid; t < k; t += kSelThreads) {
        if (t < kk) {
            oidx[row * k + t] = sidx[t];
            if (oval) oval[row * k + t] = d[sidx[t]];
        } else {
            oidx[row * k + t] = -1;
            if (oval) oval[row * k + t] = __builtin_huge_valf();
        }
    }
}

// ---- list construction ---------------------------------------------------
__global__ void count_kernel(const int32_t* __restrict__ assign, int64_t n, int64_t nlist, int32_t* __restrict__ cnt,
                             int32_t* __restrict__ bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t l = assign[i];
    if (l < 0 || l >= nlist) { atomicOr(bad, 1); return; }
    atomicAdd(&cnt[l], 1);
}

// residual rows in list order: res[v] = x[ids[v]] - cent[assign[ids[v]]]; norm2 in FP64
__global__ void residual_kernel(const float* __restrict__ x, const int64_t* __restrict__ ids,
                                const int32_t* __restrict__ assign, const float* __restrict__ cent,
                                int64_t n, int dp, float* __restrict__ res, float* __restrict__ norm2)
{
    int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (v >= n) return;
    int64_t id = ids[v];
    const float* xr = x + id * (int64_t)dp;
    const float* cr = cent + (int64_t)assign[id] * dp;
    float* rr = res + v * (int64_t)dp;
    double s = 0.0;
    for (int i = lane; i < dp; i += 64) {
        float t = xr[i] - cr[i];
        rr[i] = t;
        s += (double)t * (double)t;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) norm2[v] = (float)s;
}

}  // namespace

hipError_t launch_row_topk(const float* D, int64_t n, int64_t N, int k, int32_t* idx, float* val,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)n), b(kSelThreads);
    if (N <= 4 * kSelThreads) hipLaunchKernelGGL(row_topk_kernel<4>, g, b, 0, st, D, N, k, idx, val);
    else if (N <= 8 * kSelThreads) hipLaunchKernelGGL(row_topk_kernel<8>, g, b, 0, st, D, N, k, idx, val);
    else if (N <= 16 * kSelThreads) hipLaunchKernelGGL(row_topk_kernel<16>, g, b, 0, st, D, N, k, idx, val);
    else if (N <= 32 * kSelThreads) hipLaunchKernelGGL(row_topk_kernel<32>, g, b, 0, st, D, N, k, idx, val);
    else hipLaunchKernelGGL(row_topk_kernel<0>, g, b, 0, st, D, N, k, idx, val);
    return hipGetLastError();
}

hipError_t launch_count(const int32_t* assign, int64_t n, int64_t nlist, int32_t* cnt, int32_t* bad, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, assign, n, nlist, cnt, bad);
    return hipGetLastError();
}

hipError_t launch_residual(const float* x, const int64_t* ids, const int32_t* assign, const float* cent,
                           int64_t n, int dp, float* res, float* norm2, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, x, ids, assign, cent,
                       n, dp, res, norm2);
    return hipGetLastError();
}

}  // namespace erq
