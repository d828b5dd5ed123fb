// Exact re-rank of the best estimated candidates with the raw vectors.  The
// paper's own setting keeps no raw vectors (Sec. 2.1, Sec. 4.1); this step
// is the optional exact pass on top of it: squared Euclidean distances in
// FP32 of kc gathered rows, then the k smallest by (distance, id); for the
// inner-product metrics the distance is the negated inner product.
#include "erq_common.h"

namespace erq {

namespace {

constexpr int kMaxKc = 1024;

// One block per query.  cand: nq x kc (stride kc); the query re-ranks its
// first kcq = kc_q[iq] candidates (all kc when kc_q is null) and keeps the
// kq = k_q[iq] (else k) best; kcq == 0 copies its first kq candidates and
// their estimates (cand_est) unchanged.  Ids outside [0, n) count as missing.
template <bool IP>
__global__ __launch_bounds__(256) void rerank_kernel(const float* __restrict__ raw, int64_t n, int dp,
                                                     const float* __restrict__ q, const int64_t* __restrict__ cand,
                                                     const float* __restrict__ cand_est, int kc, int k,
                                                     const int32_t* __restrict__ kc_q, const int32_t* __restrict__ k_q,
                                                     int64_t* __restrict__ out_ids, float* __restrict__ out_d)
{
    __shared__ float sd[kMaxKc];
    __shared__ long long si[kMaxKc];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t iq = blockIdx.x;
    const float* qv = q + iq * (int64_t)dp;
    const int kq = k_q ? k_q[iq] : k;
    const int kcq = kc_q ? kc_q[iq] : kc;
    if (kcq == 0) {                                  // no re-rank for this query
        for (int t = tid; t < k; t += 256) {
            const bool ok = t < kq && cand[iq * kc + t] >= 0;
            out_ids[iq * k + t] = ok ? cand[iq * kc + t] : -1;
            out_d[iq * k + t] = ok ? cand_est[iq * kc + t] : __builtin_huge_valf();
        }
        return;
    }
    const int64_t* cq = cand + iq * kc;
    // wave wid takes candidates wid, wid + 4, ... in batches of CB, whose row
    // loads are issued together; each distance is summed in the same order
    // as one candidate at a time
    constexpr int CB = 8;
    for (int c0 = wid; c0 < kcq; c0 += 4 * CB) {
        long long id[CB];
        float s[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int c = c0 + 4 * b;
            id[b] = (c < kcq) ? cq[c] : -1;
            if (id[b] >= n) id[b] = -1;
            s[b] = 0.0f;
        }
        for (int i = lane * 4; i < dp; i += 256) {
            const float4 qq = *(const float4*)(qv + i);
            float4 a[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b)
                a[b] = (id[b] >= 0) ? *(const float4*)(raw + id[b] * (int64_t)dp + i) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if constexpr (IP) {
                    s[b] -= a[b].x * qq.x + a[b].y * qq.y + a[b].z * qq.z + a[b].w * qq.w;
                } else {
                    const float d0 = a[b].x - qq.x, d1 = a[b].y - qq.y, d2 = a[b].z - qq.z, d3 = a[b].w - qq.w;
                    s[b] += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            for (int o = 32; o > 0; o >>= 1) s[b] += __shfl_xor(s[b], o);
            const int c = c0 + 4 * b;
            if (lane == 0 && c < kcq) {
                sd[c] = (id[b] >= 0) ? s[b] : __builtin_huge_valf();
                si[c] = (id[b] >= 0) ? id[b] : 0x7FFFFFFFFFFFFFFFLL;
            }
        }
    }
    int S = 1;
    while (S < kcq) S <<= 1;
    for (int t = kcq + tid; t < S; t += 256) { sd[t] = __builtin_huge_valf(); si[t] = 0x7FFFFFFFFFFFFFFFLL; }
    for (int kb = 2; kb <= S; kb <<= 1)
        for (int j = kb >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int t = tid; t < S / 2; t += 256) {
                int i = 2 * t - (t & (j - 1)), p = i + j;
                bool up = (i & kb) == 0;
                float d0 = sd[i], d1 = sd[p];
                long long i0 = si[i], i1 = si[p];
                bool first0 = d0 < d1 || (d0 == d1 && i0 < i1);
                if (first0 != up) { sd[i] = d1; sd[p] = d0; si[i] = i1; si[p] = i0; }
            }
        }
    __syncthreads();
    for (int t = tid; t < k; t += 256) {
        const bool valid = t < kq && t < kcq && sd[t] < __builtin_huge_valf();
        out_ids[iq * k + t] = valid ? si[t] : -1;
        out_d[iq * k + t] = valid ? sd[t] : __builtin_huge_valf();
    }
}

}  // namespace

hipError_t launch_rerank(const float* raw, int64_t n, int dp, const float* q, int64_t nq, const int64_t* cand,
                         const float* cand_est, int kc, int k, const int32_t* kc_q, const int32_t* k_q,
                         int64_t* out_ids, float* out_d, hipStream_t st, int metric)
{
    if (nq <= 0) return hipSuccess;
    if (metric != ERQ_METRIC_L2)
        hipLaunchKernelGGL(rerank_kernel<true>, dim3((unsigned)nq), dim3(256), 0, st, raw, n, dp, q, cand, cand_est,
                           kc, k, kc_q, k_q, out_ids, out_d);
    else
        hipLaunchKernelGGL(rerank_kernel<false>, dim3((unsigned)nq), dim3(256), 0, st, raw, n, dp, q, cand, cand_est,
                           kc, k, kc_q, k_q, out_ids, out_d);
    return hipGetLastError();
}

namespace {
// one wave per row: s = sum of squares (FP32, fixed order), row / sqrt(s)
__global__ __launch_bounds__(256) void normalize_kernel(const float* __restrict__ x, int64_t n, int dp,
                                                        float* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const float* xr = x + r * dp;
    float s = 0.0f;
    for (int i = lane; i < dp; i += 64) s += xr[i] * xr[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float nrm = __fsqrt_rn(s);
    for (int i = lane; i < dp; i += 64) out[r * dp + i] = (nrm > 0.0f) ? __fdiv_rn(xr[i], nrm) : 0.0f;
}
}  // namespace

hipError_t launch_normalize(const float* x, int64_t n, int dp, float* out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, x, n, dp, out);
    return hipGetLastError();
}

}  // namespace erq
