// Sampling of the random orthogonal matrix P of Sec. 3.2.1 (the codebook is
// fixed by P alone, and P is sampled once per index).  Haar-distributed
// orthogonal matrix: the Q factor of the QR decomposition of a dp x dp matrix
// of independent standard normals, with the signs of R's diagonal folded into
// Q (Mezzadri, "How to generate random matrices from the classical compact
// groups", Notices AMS 2007), which makes Q exactly Haar.  Host code, FP64:
//  * normals: Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy
//    as 1, 2, 3", SC 2011) keyed by the seed, counter = the index of a pair of
//    entries; two 53-bit uniforms per call, Box-Muller;
//  * QR: Householder reflections on the column-major matrix, then Q
//    accumulated backwards from the identity; columns of the trailing update
//    are independent, so they are split over host threads, and every column
//    is computed by the same sequential sums whatever the thread count.
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "erq_common.h"

namespace erq {

namespace {

struct Philox { uint32_t c[4]; };

inline void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
    const uint64_t p = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

// Philox4x32 with 10 rounds: multipliers 0xD2511F53, 0xCD9E8D57 and key
// increments 0x9E3779B9, 0xBB67AE85 (the published constants)
Philox philox10(Philox x, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, x.c[0], hi0, lo0);
        mulhilo(0xCD9E8D57u, x.c[2], hi1, lo1);
        Philox y;
        y.c[0] = hi1 ^ x.c[1] ^ k0;
        y.c[1] = lo1;
        y.c[2] = hi0 ^ x.c[3] ^ k1;
        y.c[3] = lo0;
        x = y;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// uniform in (0, 1) from 64 random bits (53 significant bits, never 0)
inline double u53(uint32_t a, uint32_t b) {
    const uint64_t m = (((uint64_t)a << 32) | b) >> 11;
    return ((double)m + 0.5) * 0x1p-53;
}

// entry pair idx -> two independent standard normals
void normal_pair(uint64_t seed, uint64_t idx, double& z0, double& z1) {
    Philox x{{(uint32_t)idx, (uint32_t)(idx >> 32), 0x45525131u /* stream tag */, 0u}};
    const Philox r = philox10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = u53(r.c[0], r.c[1]), u2 = u53(r.c[2], r.c[3]);
    const double rad = std::sqrt(-2.0 * std::log(u1));
    const double ang = 6.283185307179586476925286766559 * u2;
    z0 = rad * std::cos(ang);
    z1 = rad * std::sin(ang);
}

// runs f(j) for j in [lo, hi) over host threads (contiguous blocks of columns)
template <class F>
void for_columns(int lo, int hi, int nthr, F f) {
    const int n = hi - lo;
    if (n <= 0) return;
    if (nthr <= 1 || n < 64) {
        for (int j = lo; j < hi; ++j) f(j);
        return;
    }
    const int t = std::min(nthr, n / 32);
    std::vector<std::thread> th;
    th.reserve(t);
    for (int w = 0; w < t; ++w) {
        const int a = lo + (int)((int64_t)n * w / t), b = lo + (int)((int64_t)n * (w + 1) / t);
        th.emplace_back([=]() { for (int j = a; j < b; ++j) f(j); });
    }
    for (auto& x : th) x.join();
}

}  // namespace

// 64 random bits for (seed, stream tag, counter): one Philox4x32-10 block
uint64_t philox_u64(uint64_t seed, uint32_t tag, uint64_t counter)
{
    Philox x{{(uint32_t)counter, (uint32_t)(counter >> 32), tag, 0u}};
    const Philox r = philox10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
    return ((uint64_t)r.c[0] << 32) | r.c[1];
}

// P (row-major dp x dp, FP32) <- Haar orthogonal matrix of the seed
void sample_rotation(int dp, uint64_t seed, float* P)
{
    const int n = dp;
    std::vector<double> A((size_t)n * n);           // column-major: A[j*n + i] = a_ij
    for (uint64_t e = 0; e < (uint64_t)n * n; e += 2) {
        double z0, z1;
        normal_pair(seed, e / 2, z0, z1);
        A[e] = z0;
        if (e + 1 < (uint64_t)n * n) A[e + 1] = z1;
    }
    const int nthr = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<double> V((size_t)n * n, 0.0);      // Householder vectors, column k from row k
    std::vector<double> rsign(n, 1.0);
    for (int k = 0; k < n; ++k) {
        double* a = &A[(size_t)k * n];
        double s = 0.0;
        for (int i = k; i < n; ++i) s += a[i] * a[i];
        const double nrm = std::sqrt(s);
        double* v = &V[(size_t)k * n];
        if (nrm == 0.0) {                           // (probability 0) identity reflection
            rsign[k] = 1.0;
            continue;
        }
        const double alpha = (a[k] >= 0.0) ? -nrm : nrm;   // R_kk
        rsign[k] = (alpha >= 0.0) ? 1.0 : -1.0;
        for (int i = k; i < n; ++i) v[i] = a[i];
        v[k] -= alpha;
        double vn = 0.0;
        for (int i = k; i < n; ++i) vn += v[i] * v[i];
        vn = std::sqrt(vn);
        for (int i = k; i < n; ++i) v[i] /= vn;
        a[k] = alpha;
        for (int i = k + 1; i < n; ++i) a[i] = 0.0;
        for_columns(k + 1, n, nthr, [&](int j) {
            double* c = &A[(size_t)j * n];
            double w = 0.0;
            for (int i = k; i < n; ++i) w += v[i] * c[i];
            w *= 2.0;
            for (int i = k; i < n; ++i) c[i] -= w * v[i];
        });
    }
    // Q = H_0 H_1 ... H_{n-1} applied to the identity, from the last reflection back
    std::vector<double> Q((size_t)n * n, 0.0);       // column-major
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int k = n - 1; k >= 0; --k) {
        const double* v = &V[(size_t)k * n];
        bool zero = true;
        for (int i = k; i < n && zero; ++i) zero = v[i] == 0.0;
        if (zero) continue;
        for_columns(k, n, nthr, [&](int j) {
            double* c = &Q[(size_t)j * n];
            double w = 0.0;
            for (int i = k; i < n; ++i) w += v[i] * c[i];
            w *= 2.0;
            for (int i = k; i < n; ++i) c[i] -= w * v[i];
        });
    }
    // Haar: column j of Q times sign(R_jj); P = Q row-major
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) P[(size_t)i * n + j] = (float)(Q[(size_t)j * n + i] * rsign[j]);
}

}  // namespace erq
