// IVF list construction (Sec. 4.1: the lists come from k-means, each
// vector is centred on its own list's centroid, Sec. 5.1):
//  * a stable bucket sort of the rows by list (members of a list in
//    ascending row order), without atomics whose order could change a result;
//  * per-list means with FP64 sums in member order (the k-means update), so
//    the same input gives the same centroids bit for bit on every run;
//  * a row gather (the k-means initial centroids).
#include <algorithm>

#include "erq_common.h"

namespace erq {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortMaxBlocks = 128;
constexpr int kMeanChunk = 1024;      // members per partial sum

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// blocks of the bucket sort: at most kSortMaxBlocks, and at most 16M per-block
// list counters in total
int sort_blocks(int64_t n, int64_t nlist) {
    int64_t g = std::min<int64_t>(kSortMaxBlocks, std::max<int64_t>(1, ((int64_t)1 << 24) / std::max<int64_t>(nlist, 1)));
    g = std::min<int64_t>(g, std::max<int64_t>(1, (n + kSortThreads - 1) / kSortThreads));
    return (int)g;
}

// cnt2[b][l] = rows of block b's contiguous chunk in list l
__global__ __launch_bounds__(kSortThreads) void bucket_count_kernel(const int32_t* __restrict__ assign, int64_t n,
                                                                    int64_t nlist, int64_t chunk,
                                                                    int32_t* __restrict__ cnt2)
{
    const int64_t b = blockIdx.x;
    const int64_t r0 = b * chunk, r1 = min(n, r0 + chunk);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kSortThreads) atomicAdd(&cnt2[b * nlist + assign[r]], 1);
}

// per list: base2[b][l] = list_off[l] + rows of list l in blocks before b (in place over cnt2)
__global__ void bucket_base_kernel(int32_t* __restrict__ cnt2, int64_t nlist, int G, const int64_t* __restrict__ list_off)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlist) return;
    int64_t run = list_off[l];
    for (int b = 0; b < G; ++b) {
        const int32_t c = cnt2[(int64_t)b * nlist + l];
        cnt2[(int64_t)b * nlist + l] = (int32_t)run;
        run += c;
    }
}

// Block b places the rows of its chunk in rounds of kSortThreads rows: a row's
// rank among the round's earlier rows of the same list (LDS), then one atomic
// per list group of the round on the block's own counter, read back by the
// group through LDS.  Only block b touches its counters, and the rounds are
// ordered by barriers, so positions ascend with the row number.
__global__ __launch_bounds__(kSortThreads) void bucket_place_kernel(const int32_t* __restrict__ assign, int64_t n,
                                                                    int64_t nlist, int64_t chunk,
                                                                    int32_t* __restrict__ base2,
                                                                    int32_t* __restrict__ ids32)
{
    __shared__ int32_t s_l[kSortThreads];
    __shared__ int32_t s_base[kSortThreads];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t r0 = b * chunk, r1 = min(n, r0 + chunk);
    for (int64_t rb = r0; rb < r1; rb += kSortThreads) {
        const int64_t r = rb + t;
        const int32_t l = (r < r1) ? assign[r] : -1;
        s_l[t] = l;
        __syncthreads();
        int rank = 0, first = t, cnt = 0;
        if (l >= 0) {
            for (int u = 0; u < kSortThreads; ++u) {
                if (s_l[u] == l) {
                    if (u < t) { ++rank; first = min(first, u); }
                    ++cnt;
                }
            }
            if (first == t) s_base[t] = atomicAdd(&base2[b * nlist + l], cnt);
        }
        __syncthreads();
        if (l >= 0) ids32[s_base[first] + rank] = (int32_t)r;
        __syncthreads();
    }
}

// partial FP64 sums of one (list, chunk of kMeanChunk members): thread t sums
// dimensions t, t + 256, ... over the chunk's members in order
__global__ __launch_bounds__(256) void list_psum_kernel(const float* __restrict__ x, int dp,
                                                        const int32_t* __restrict__ ids32,
                                                        const int64_t* __restrict__ list_off,
                                                        const int32_t* __restrict__ chunk_list,
                                                        const int32_t* __restrict__ chunk_first,
                                                        double* __restrict__ psum)
{
    const int64_t c = blockIdx.x;
    const int l = chunk_list[c];
    const int64_t m0 = list_off[l] + (int64_t)chunk_first[c] * kMeanChunk;
    const int64_t m1 = min(list_off[l + 1], m0 + kMeanChunk);
    for (int d = threadIdx.x; d < dp; d += 256) {
        double acc = 0.0;
#pragma unroll 8
        for (int64_t v = m0; v < m1; ++v) acc += (double)x[(int64_t)ids32[v] * dp + d];
        psum[c * dp + d] = acc;
    }
}

// mean of list l from its chunks' partial sums in chunk order; an empty list keeps its centroid
__global__ __launch_bounds__(256) void list_mean_kernel(const double* __restrict__ psum, int dp,
                                                        const int64_t* __restrict__ list_off,
                                                        const int32_t* __restrict__ list_chunk0, float* __restrict__ cent)
{
    const int l = blockIdx.x;
    const int64_t cnt = list_off[l + 1] - list_off[l];
    if (cnt == 0) return;
    const int c0 = list_chunk0[l], c1 = list_chunk0[l + 1];
    for (int d = threadIdx.x; d < dp; d += 256) {
        double s = 0.0;
        for (int c = c0; c < c1; ++c) s += psum[(int64_t)c * dp + d];
        cent[(int64_t)l * dp + d] = (float)(s / (double)cnt);
    }
}

__global__ void gather_rows_kernel(const float* __restrict__ x, int dp, const int64_t* __restrict__ rows, int64_t m,
                                   float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * dp) return;
    const int64_t r = i / dp;
    out[i] = x[rows[r] * dp + (i - r * dp)];
}

}  // namespace

size_t bucket_scratch_bytes(int64_t n, int64_t nlist)
{
    return a256(sizeof(int32_t) * (size_t)sort_blocks(n, nlist) * (size_t)nlist);
}

hipError_t launch_bucket_sort(const int32_t* assign, int64_t n, int64_t nlist, const int64_t* list_off,
                              int32_t* ids32, void* scratch, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int G = sort_blocks(n, nlist);
    const int64_t chunk = (n + G - 1) / G;
    int32_t* cnt2 = (int32_t*)scratch;
    hipError_t e = hipMemsetAsync(cnt2, 0, sizeof(int32_t) * (size_t)G * nlist, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_count_kernel, dim3(G), dim3(kSortThreads), 0, st, assign, n, nlist, chunk, cnt2);
    hipLaunchKernelGGL(bucket_base_kernel, dim3((unsigned)((nlist + 255) / 256)), dim3(256), 0, st, cnt2, nlist, G,
                       list_off);
    hipLaunchKernelGGL(bucket_place_kernel, dim3(G), dim3(kSortThreads), 0, st, assign, n, nlist, chunk, cnt2, ids32);
    return hipGetLastError();
}

// chunk tables: chunk -> (list, index within the list), list -> first chunk
static void mean_chunks(const std::vector<int64_t>& off, std::vector<int32_t>& clist, std::vector<int32_t>& cfirst,
                        std::vector<int32_t>& l0)
{
    const int64_t C = (int64_t)off.size() - 1;
    l0.assign(C + 1, 0);
    clist.clear();
    cfirst.clear();
    for (int64_t l = 0; l < C; ++l) {
        l0[l] = (int32_t)clist.size();
        const int64_t nc = (off[l + 1] - off[l] + kMeanChunk - 1) / kMeanChunk;
        for (int64_t c = 0; c < nc; ++c) { clist.push_back((int32_t)l); cfirst.push_back((int32_t)c); }
    }
    l0[C] = (int32_t)clist.size();
}

size_t list_mean_scratch_bytes(const std::vector<int64_t>& off, int dp)
{
    std::vector<int32_t> cl, cf, l0;
    mean_chunks(off, cl, cf, l0);
    return a256(sizeof(double) * std::max<size_t>(cl.size(), 1) * dp) + 2 * a256(sizeof(int32_t) * std::max<size_t>(cl.size(), 1)) +
           a256(sizeof(int32_t) * l0.size());
}

hipError_t launch_list_mean(const float* x, int dp, const int32_t* ids32, const std::vector<int64_t>& off,
                            const int64_t* list_off, float* cent, void* scratch, hipStream_t st)
{
    std::vector<int32_t> cl, cf, l0;
    mean_chunks(off, cl, cf, l0);
    const size_t nc = cl.size();
    char* w = (char*)scratch;
    double* psum = (double*)w; w += a256(sizeof(double) * std::max<size_t>(nc, 1) * dp);
    int32_t* d_cl = (int32_t*)w; w += a256(sizeof(int32_t) * std::max<size_t>(nc, 1));
    int32_t* d_cf = (int32_t*)w; w += a256(sizeof(int32_t) * std::max<size_t>(nc, 1));
    int32_t* d_l0 = (int32_t*)w;
    hipError_t e = hipSuccess;
    if (nc) e = hipMemcpyAsync(d_cl, cl.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nc) e = hipMemcpyAsync(d_cf, cf.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_l0, l0.data(), sizeof(int32_t) * l0.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    if (nc) hipLaunchKernelGGL(list_psum_kernel, dim3((unsigned)nc), dim3(256), 0, st, x, dp, ids32, list_off, d_cl, d_cf, psum);
    const int64_t C = (int64_t)off.size() - 1;
    hipLaunchKernelGGL(list_mean_kernel, dim3((unsigned)C), dim3(256), 0, st, psum, dp, list_off, d_l0, cent);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);      // the host chunk tables go out of scope
    return e;
}

hipError_t launch_gather_rows(const float* x, int dp, const int64_t* rows, int64_t m, float* out, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((m * dp + 255) / 256)), dim3(256), 0, st, x, dp, rows, m, out);
    return hipGetLastError();
}

}  // namespace erq
