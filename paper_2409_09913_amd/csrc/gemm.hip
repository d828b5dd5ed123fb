// Dense FP32 / BF16 matrix-core GEMM for the rotation by P (Sec. 3.4: the
// data and the queries are multiplied by P^{-1} = P^T) and for the squared
// distances of the coarse IVF probe (Sec. 4.1).
//
// Workgroup tile 128 x 128, 4 waves each owning 64 x 64 = 2 x 2 tiles of the
// 32 x 32 MFMA.  FP32: v_mfma_f32_32x32x2_f32, K staged 16 at a time.
// BF16: v_mfma_f32_32x32x16_bf16 with FP32 accumulation, K staged 32 at a
// time, inputs rounded to BF16 (nearest even) while staging.
#include "erq_common.h"

namespace erq {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int BM = 128, BN = 128;

// 32x32 MFMA output element (lane, reg) -> (row, col) within the tile
__device__ inline int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ inline unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (unsigned short)(u >> 16);   // inf / nan
    unsigned r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}

// EPI: 0 = store C; 1 = store ||a||^2 + ||b||^2 - 2 C
template <int EPI>
__global__ __launch_bounds__(256) void gemm_f32_kernel(
    const float* __restrict__ A, int64_t n, int K, const float* __restrict__ B, int N, int b_trans,
    float* __restrict__ out, int64_t ldo, const float* __restrict__ an2, const float* __restrict__ bn2)
{
    constexpr int BK = 16;
    // two LDS buffers: the next K-tile is loaded into registers while the
    // current one is multiplied, then stored to the other buffer
    __shared__ float As[2][BK][BM + 4];
    __shared__ float Bs[2][BK][BN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.y * BM;
    const int col0 = blockIdx.x * BN;
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    v16f acc[2][2];
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    // 128 x 16 floats per operand = 2 float4 per thread
    float4 ra[2], rb[2];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i;
            const int m = e >> 2, kq = (e & 3) * 4;
            const int64_t gr = row0 + m;
            ra[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gr < n && k0 + kq < K) ra[i] = *(const float4*)(A + gr * (int64_t)K + k0 + kq);
            if (!b_trans) {
                const int kk = e / (BN / 4), nq = (e % (BN / 4)) * 4;
                rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k0 + kk < K && col0 + nq < N) rb[i] = *(const float4*)(B + (int64_t)(k0 + kk) * N + col0 + nq);
            } else {
                const int gc = col0 + m;
                rb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (gc < N && k0 + kq < K) rb[i] = *(const float4*)(B + (int64_t)gc * K + k0 + kq);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = tid + 256 * i;
            const int m = e >> 2, kq = (e & 3) * 4;
            As[buf][kq + 0][m] = ra[i].x; As[buf][kq + 1][m] = ra[i].y;
            As[buf][kq + 2][m] = ra[i].z; As[buf][kq + 3][m] = ra[i].w;
            if (!b_trans) {
                const int kk = e / (BN / 4), nq = (e % (BN / 4)) * 4;
                *(float4*)&Bs[buf][kk][nq] = rb[i];
            } else {
                Bs[buf][kq + 0][m] = rb[i].x; Bs[buf][kq + 1][m] = rb[i].y;
                Bs[buf][kq + 2][m] = rb[i].z; Bs[buf][kq + 3][m] = rb[i].w;
            }
        }
    };
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) load(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 2) {
            float a0 = As[cur][ks + (lane >> 5)][wm + (lane & 31)];
            float a1 = As[cur][ks + (lane >> 5)][wm + 32 + (lane & 31)];
            float b0 = Bs[cur][ks + (lane >> 5)][wn + (lane & 31)];
            float b1 = Bs[cur][ks + (lane >> 5)][wn + 32 + (lane & 31)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int gc = col0 + wn + 32 * b + (lane & 31);
            if (gc >= N) continue;
            for (int r = 0; r < 16; ++r) {
                const int64_t gr = row0 + wm + 32 * a + out_row(lane, r);
                if (gr >= n) continue;
                float v = acc[a][b][r];
                if (EPI == 1) v = (an2[gr] + bn2[gc]) - 2.0f * v;
                out[gr * ldo + gc] = v;
            }
        }
}

__global__ __launch_bounds__(256) void gemm_bf16_kernel(
    const float* __restrict__ A, int64_t n, int K, const float* __restrict__ B, int N, int b_trans,
    float* __restrict__ out, int64_t ldo)
{
    constexpr int BK = 32;
    // row-major by the contraction index so that a lane reads 8 consecutive k
    __shared__ unsigned short As[BM][BK + 8];
    __shared__ unsigned short Bs[BN][BK + 8];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.y * BM;
    const int col0 = blockIdx.x * BN;
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    v16f acc[2][2];
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = tid; e < BM * BK / 4; e += 256) {
            int m = e / (BK / 4), kq = (e % (BK / 4)) * 4;
            int64_t gr = row0 + m;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gr < n && k0 + kq < K) v = *(const float4*)(A + gr * (int64_t)K + k0 + kq);
            As[m][kq + 0] = f2bf(v.x); As[m][kq + 1] = f2bf(v.y); As[m][kq + 2] = f2bf(v.z); As[m][kq + 3] = f2bf(v.w);
        }
        if (!b_trans) {
            for (int e = tid; e < BK * BN / 4; e += 256) {
                int kk = e / (BN / 4), nq = (e % (BN / 4)) * 4;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k0 + kk < K && col0 + nq < N) v = *(const float4*)(B + (int64_t)(k0 + kk) * N + col0 + nq);
                Bs[nq + 0][kk] = f2bf(v.x); Bs[nq + 1][kk] = f2bf(v.y); Bs[nq + 2][kk] = f2bf(v.z); Bs[nq + 3][kk] = f2bf(v.w);
            }
        } else {
            for (int e = tid; e < BN * BK / 4; e += 256) {
                int nn = e / (BK / 4), kq = (e % (BK / 4)) * 4;
                int gc = col0 + nn;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (gc < N && k0 + kq < K) v = *(const float4*)(B + (int64_t)gc * K + k0 + kq);
                Bs[nn][kq + 0] = f2bf(v.x); Bs[nn][kq + 1] = f2bf(v.y); Bs[nn][kq + 2] = f2bf(v.z); Bs[nn][kq + 3] = f2bf(v.w);
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            v8bf a0, a1, b0, b1;
            __builtin_memcpy(&a0, &As[wm + (lane & 31)][kk], 16);
            __builtin_memcpy(&a1, &As[wm + 32 + (lane & 31)][kk], 16);
            __builtin_memcpy(&b0, &Bs[wn + (lane & 31)][kk], 16);
            __builtin_memcpy(&b1, &Bs[wn + 32 + (lane & 31)][kk], 16);
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int gc = col0 + wn + 32 * b + (lane & 31);
            if (gc >= N) continue;
            for (int r = 0; r < 16; ++r) {
                const int64_t gr = row0 + wm + 32 * a + out_row(lane, r);
                if (gr < n) out[gr * ldo + gc] = acc[a][b][r];
            }
        }
}

}  // namespace

hipError_t launch_gemm(const float* A, int64_t n, int K, const float* B, int N, int b_trans,
                       int precision, float* out, int64_t ldo, hipStream_t st)
{
    if (n <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((n + BM - 1) / BM));
    if (precision == 1)
        hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, A, n, K, B, N, b_trans, out, ldo);
    else
        hipLaunchKernelGGL(gemm_f32_kernel<0>, grid, dim3(256), 0, st, A, n, K, B, N, b_trans, out, ldo,
                           (const float*)nullptr, (const float*)nullptr);
    return hipGetLastError();
}

// dist = ||a||^2 + ||b||^2 - 2 a.b, with norms an2 (n) and bn2 (N) precomputed
// FP32 -> two BF16 planes: hi = bf16(x) and lo = bf16(x - hi) (x - hi is
// exact, so x = hi + lo to 2^-17 relative); bit patterns, 4 elements per
// thread, n a multiple of 4.
__global__ __launch_bounds__(256) void split_bf16_kernel(const float* __restrict__ x, int64_t n,
                                                         unsigned short* __restrict__ hi,
                                                         unsigned short* __restrict__ lo)
{
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i >= n) return;
    const float4 v = *(const float4*)(x + i);
    const float xv[4] = {v.x, v.y, v.z, v.w};
    unsigned h[4], l[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        h[c] = f2bf(xv[c]);
        l[c] = f2bf(xv[c] - __uint_as_float(h[c] << 16));
    }
    *(uint2*)(hi + i) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    *(uint2*)(lo + i) = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
}

__device__ inline uint4 ld16(const unsigned short* p, bool ok) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (ok) v = *(const uint4*)p;
    return v;
}

// EPI 1: squared distances ||a||^2 + ||b||^2 - 2 a.b of the coarse probe;
// EPI 2: negated inner products -a.b (the probe of the inner-product
// metrics); EPI 0: a.b (the query rotation).  Products on the BF16 matrix cores, from
// operands split beforehand into hi
// and lo BF16 planes (split_bf16_kernel): a.b = lo.hi + hi.lo + hi.hi per
// 16-wide K chunk, FP32 accumulation.  Each product is off by at most
// 2^-15 |a_i b_i| (the dropped lo.lo and the two split residuals), so a
// distance by at most 2^-14 sum|a_i b_i| plus FP32 accumulation: a few units
// in the 5th digit, enough to order centroids except near-ties.  A is n x K,
// B is N x K (row-major planes), K a multiple of 32.  Tile 128 x 128, K
// staged 32 at a time in one LDS buffer (40 KB, so several blocks share a
// CU); the next K-tile is loaded into registers while the current one is
// multiplied.
template <int EPI>
__global__ __launch_bounds__(256, 3) void sqdist_bf16x3_kernel(
    const unsigned short* __restrict__ Ahg, const unsigned short* __restrict__ Alg, int64_t n, int K,
    const unsigned short* __restrict__ Bhg, const unsigned short* __restrict__ Blg, int N,
    float* __restrict__ out, int64_t ldo, const float* __restrict__ an2, const float* __restrict__ bn2)
{
    constexpr int BK = 32, LD = BK + 8;
    __shared__ __align__(16) unsigned short Ah[BM][LD], Al[BM][LD], Bh[BN][LD], Bl[BN][LD];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.y * BM;
    const int col0 = blockIdx.x * BN;
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    v16f acc[2][2];
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    // per K-tile and plane: 128 rows x 32 k = 512 chunks of 16 bytes; thread
    // tid moves chunks tid and tid + 256 (row m = e/4, k offset 8*(e%4))
    const int m0 = tid >> 2, m1 = m0 + 64, kq = (tid & 3) * 8;
    const bool a0 = row0 + m0 < n, a1 = row0 + m1 < n, b0 = col0 + m0 < N, b1 = col0 + m1 < N;
    const unsigned short* pa0h = Ahg + (row0 + m0) * K + kq;
    const unsigned short* pa1h = Ahg + (row0 + m1) * K + kq;
    const unsigned short* pa0l = Alg + (row0 + m0) * K + kq;
    const unsigned short* pa1l = Alg + (row0 + m1) * K + kq;
    const unsigned short* pb0h = Bhg + (int64_t)(col0 + m0) * K + kq;
    const unsigned short* pb1h = Bhg + (int64_t)(col0 + m1) * K + kq;
    const unsigned short* pb0l = Blg + (int64_t)(col0 + m0) * K + kq;
    const unsigned short* pb1l = Blg + (int64_t)(col0 + m1) * K + kq;
    uint4 r0 = ld16(pa0h, a0), r1 = ld16(pa1h, a1), r2 = ld16(pa0l, a0), r3 = ld16(pa1l, a1);
    uint4 r4 = ld16(pb0h, b0), r5 = ld16(pb1h, b1), r6 = ld16(pb0l, b0), r7 = ld16(pb1l, b1);
    *(uint4*)&Ah[m0][kq] = r0; *(uint4*)&Ah[m1][kq] = r1; *(uint4*)&Al[m0][kq] = r2; *(uint4*)&Al[m1][kq] = r3;
    *(uint4*)&Bh[m0][kq] = r4; *(uint4*)&Bh[m1][kq] = r5; *(uint4*)&Bl[m0][kq] = r6; *(uint4*)&Bl[m1][kq] = r7;
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) {                                 // next K-tile into registers while this one is multiplied
            const int k1 = k0 + BK;
            r0 = ld16(pa0h + k1, a0); r1 = ld16(pa1h + k1, a1); r2 = ld16(pa0l + k1, a0); r3 = ld16(pa1l + k1, a1);
            r4 = ld16(pb0h + k1, b0); r5 = ld16(pb1h + k1, b1); r6 = ld16(pb0l + k1, b0); r7 = ld16(pb1l + k1, b1);
        }
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            v8bf ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                __builtin_memcpy(&ah[t], &Ah[wm + 32 * t + (lane & 31)][kk], 16);
                __builtin_memcpy(&al[t], &Al[wm + 32 * t + (lane & 31)][kk], 16);
                __builtin_memcpy(&bh[t], &Bh[wn + 32 * t + (lane & 31)][kk], 16);
                __builtin_memcpy(&bl[t], &Bl[wn + 32 * t + (lane & 31)][kk], 16);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
                }
        }
        __syncthreads();                        // every read of this K-tile is done
        if (more) {
            *(uint4*)&Ah[m0][kq] = r0; *(uint4*)&Ah[m1][kq] = r1; *(uint4*)&Al[m0][kq] = r2; *(uint4*)&Al[m1][kq] = r3;
            *(uint4*)&Bh[m0][kq] = r4; *(uint4*)&Bh[m1][kq] = r5; *(uint4*)&Bl[m0][kq] = r6; *(uint4*)&Bl[m1][kq] = r7;
            __syncthreads();
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int gc = col0 + wn + 32 * b + (lane & 31);
            if (gc >= N) continue;
            for (int r = 0; r < 16; ++r) {
                const int64_t gr = row0 + wm + 32 * a + out_row(lane, r);
                if (gr >= n) continue;
                if constexpr (EPI == 1) out[gr * ldo + gc] = (an2[gr] + bn2[gc]) - 2.0f * acc[a][b][r];
                else if constexpr (EPI == 2) out[gr * ldo + gc] = -acc[a][b][r];
                else out[gr * ldo + gc] = acc[a][b][r];
            }
        }
}

// Transposed split of a K x N row-major matrix: hi/lo planes of its
// transpose (N x K), for the B operand of sqdist_bf16x3_kernel.
__global__ __launch_bounds__(256) void split_bf16_t_kernel(const float* __restrict__ x, int K, int N,
                                                           unsigned short* __restrict__ hi,
                                                           unsigned short* __restrict__ lo)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // output index: row j of N, column k of K
    if (i >= (int64_t)K * N) return;
    const int64_t j = i / K, k = i - j * K;
    const float v = x[k * N + j];
    const unsigned h = f2bf(v);
    hi[i] = (unsigned short)h;
    lo[i] = f2bf(v - __uint_as_float(h << 16));
}

hipError_t launch_split_bf16_t(const float* x, int K, int N, unsigned short* hi, unsigned short* lo, hipStream_t st)
{
    const int64_t n = (int64_t)K * N;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(split_bf16_t_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, K, N, hi, lo);
    return hipGetLastError();
}

// out = A.B^T (n x N, leading dimension ldo) from the BF16 hi/lo planes of A
// (n x K) and B (N x K); same products and error as the probe's distances
hipError_t launch_gemm_bf16x3(const unsigned short* Ah, const unsigned short* Al, int64_t n,
                              const unsigned short* Bh, const unsigned short* Bl, int64_t N, int K,
                              float* out, int64_t ldo, hipStream_t st)
{
    if (n <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((n + BM - 1) / BM));
    hipLaunchKernelGGL(sqdist_bf16x3_kernel<0>, grid, dim3(256), 0, st, Ah, Al, n, K, Bh, Bl, (int)N, out, ldo,
                       (const float*)nullptr, (const float*)nullptr);
    return hipGetLastError();
}

// Rows of X (n x K, K a multiple of 4) -> their BF16 hi/lo planes (as
// split_bf16_kernel) and squared norms ||x||^2 (FP32); one wave per row,
// 4 consecutive elements per lane
__global__ __launch_bounds__(256) void split_norm_kernel(const float* __restrict__ X, int64_t n, int K,
                                                         unsigned short* __restrict__ hi,
                                                         unsigned short* __restrict__ lo, float* __restrict__ n2)
{
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    float s = 0.0f;
    for (int k = 4 * lane; k < K; k += 256) {
        const int64_t i = r * (int64_t)K + k;
        const float4 v = *(const float4*)(X + i);
        const float xv[4] = {v.x, v.y, v.z, v.w};
        unsigned h[4], l[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            s += xv[c] * xv[c];
            h[c] = f2bf(xv[c]);
            l[c] = f2bf(xv[c] - __uint_as_float(h[c] << 16));
        }
        *(uint2*)(hi + i) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        *(uint2*)(lo + i) = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) n2[r] = s;
}

hipError_t launch_split_norm(const float* X, int64_t n, int K, unsigned short* hi, unsigned short* lo, float* n2,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(split_norm_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, n, K, hi, lo, n2);
    return hipGetLastError();
}

hipError_t launch_split_bf16(const float* x, int64_t n, unsigned short* hi, unsigned short* lo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)((n / 4 + 255) / 256)), dim3(256), 0, st, x, n, hi, lo);
    return hipGetLastError();
}

hipError_t launch_sqdist_pre(const unsigned short* Ah, const unsigned short* Al, int64_t n,
                             const unsigned short* Bh, const unsigned short* Bl, int64_t N, int K,
                             const float* an2, const float* bn2, float* out, hipStream_t st, int neg_ip)
{
    if (n <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((n + BM - 1) / BM));
    if (neg_ip)
        hipLaunchKernelGGL(sqdist_bf16x3_kernel<2>, grid, dim3(256), 0, st, Ah, Al, n, K, Bh, Bl, (int)N, out,
                           (int64_t)N, an2, bn2);
    else
        hipLaunchKernelGGL(sqdist_bf16x3_kernel<1>, grid, dim3(256), 0, st, Ah, Al, n, K, Bh, Bl, (int)N, out,
                           (int64_t)N, an2, bn2);
    return hipGetLastError();
}

}  // namespace erq
