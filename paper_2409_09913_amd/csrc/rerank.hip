// Exact re-rank of the best estimated candidates with the raw vectors.  The
// paper's own setting keeps no raw vectors (Sec. 2.1, Sec. 4.1); this step
// is the optional exact pass on top of it: squared Euclidean distances in
// FP32 of kc gathered rows, then the k smallest by (distance, id).
#include "erq_common.h"

namespace erq {

namespace {

constexpr int kMaxKc = 256;

__global__ __launch_bounds__(256) void rerank_kernel(const float* __restrict__ raw, int dp,
                                                     const float* __restrict__ q, const int64_t* __restrict__ cand,
                                                     int kc, int k, int64_t* __restrict__ out_ids,
                                                     float* __restrict__ out_d)
{
    __shared__ float sd[kMaxKc];
    __shared__ long long si[kMaxKc];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t iq = blockIdx.x;
    const float* qv = q + iq * (int64_t)dp;
    for (int c = wid; c < kc; c += 4) {
        const long long id = cand[iq * kc + c];
        float s = 0.0f;
        if (id >= 0) {
            const float* xv = raw + id * (int64_t)dp;
            for (int i = lane * 4; i < dp; i += 256) {
                float4 a = *(const float4*)(xv + i);
                float4 b = *(const float4*)(qv + i);
                float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
                s += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
            }
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        }
        if (lane == 0) {
            sd[c] = (id >= 0) ? s : __builtin_huge_valf();
            si[c] = (id >= 0) ? id : 0x7FFFFFFFFFFFFFFFLL;
        }
    }
    int S = 1;
    while (S < kc) S <<= 1;
    for (int t = kc + tid; t < S; t += 256) { sd[t] = __builtin_huge_valf(); si[t] = 0x7FFFFFFFFFFFFFFFLL; }
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
        const bool valid = t < kc && sd[t] < __builtin_huge_valf();
        out_ids[iq * k + t] = valid ? si[t] : -1;
        out_d[iq * k + t] = valid ? sd[t] : __builtin_huge_valf();
    }
}

}  // namespace

hipError_t launch_rerank(const float* raw, int dp, const float* q, int64_t nq, const int64_t* cand,
                         int kc, int k, int64_t* out_ids, float* out_d, hipStream_t st)
{
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(rerank_kernel, dim3((unsigned)nq), dim3(256), 0, st, raw, dp, q, cand, kc, k, out_ids, out_d);
    return hipGetLastError();
}

}  // namespace erq
