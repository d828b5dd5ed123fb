// Algorithm 1 (Quantize) of Extended RaBitQ, Sec. 3.2.2, on gfx950.
//
// One workgroup of 256 threads per vector.  In the orthant of r' every
// coordinate has magnitude a_i; level k_i in [0, K] (K = 2^{B-1}-1) means
// y_i = +-(k_i + 1/2).  Level k_i moves to m at the critical value
// t = m / a_i.  Instead of a heap, the critical values are taken in
// ascending order window by window:
//   1. sort a descending (ties: dimension ascending) in LDS;
//   2. a window is the set of events whose key d = a/m (d descending ==
//      t ascending) lies in [x, d_cur); x is found by bisection on the bit
//      pattern of the double x, counting events with one binary search per
//      level; a window holds at most CAP events (CAP >= 2 dp, and an exact
//      tie group has at most dp events, so bisection always succeeds);
//   3. the window's events are ordered by (d desc, dim asc): for B <= 4
//      each goes to its rank (every level's events are already in order; the
//      rank adds, per other level, a binary search on exact products), for
//      larger B they are gathered and bitonic-sorted; then prefix-summed in
//      integers: 2<y,r'> as int64 fixed point (a scaled
//      by the power of two that puts max a in [1,2), 40 fractional bits) and
//      4||y||^2 exactly; the objective double(2S1)/sqrt(double(4S2)) of every
//      event is compared, keeping the first strict maximum;
//   4. the levels of the best event's state are recovered by one binary
//      search per level (a replay of the enumeration up to that event).
// Pruning (B >= 5): in a range of events S1 and S2 only grow, so every
// objective in it is at most S1(end)/sqrt(S2(start)); prefix sums of the
// fixed-point magnitudes give both ends from the per-level counts.  A range
// whose bound is <= the best so far, or below the best of a few grid points
// k_i = min(K, floor(t a_i)) (minus a 1e-12 margin), holds no first strict
// maximum and is skipped without enumeration.
// Keys d = a/m are correctly rounded doubles of an FP32 a and m <= 127;
// distinct ratios differ by more than 2^-39 relative, so the double keys order
// the events exactly as the exact critical values do.
#include "erq_common.h"

namespace erq {

namespace {

constexpr int kThreads = 256;
constexpr int kRedLL = 48;           // int64 reduction slots (block_sum3 uses 32..43)

__device__ inline double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline long long wave_sum_ll(long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// event p0 = (level m0, dim d0) before p1 in key order (d = a/m descending,
// dim ascending): a0/m0 > a1/m1 decided as a0*m1 > a1*m0, exact in double
// (24-bit magnitudes times levels below 2^7); distinct ratios give distinct
// keys in the same order, so this is the order of the rounded keys.
// 0xFFFFFFFF is padding, after every event.
__device__ inline bool ev_before(const float* adim, unsigned p0, unsigned p1) {
    if (p1 == 0xFFFFFFFFu) return p0 != 0xFFFFFFFFu;
    if (p0 == 0xFFFFFFFFu) return false;
    const unsigned d0 = p0 & 0xFFFu, d1 = p1 & 0xFFFu;
    const double x0 = (double)adim[d0] * (double)(p1 >> 12), x1 = (double)adim[d1] * (double)(p0 >> 12);
    return x0 > x1 || (x0 == x1 && d0 < d1);
}

// number of j in [0, n) with fl(A[j]/m) >= x  (A sorted descending)
__device__ inline int count_ge(const float* A, int n, int m, double x) {
    int lo = 0, hi = n;
    const double dm = (double)m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((double)A[mid] / dm >= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// number of j with (fl(A[j]/m), I[j]) at or before (d, i) in key order
__device__ inline int count_upto(const float* A, const unsigned short* I, int n, int m, double d, int i) {
    int lo = 0, hi = n;
    const double dm = (double)m;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        double k = (double)A[mid] / dm;
        bool le = (k > d) || (k == d && I[mid] <= i);
        if (le) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// block-wide sums of three int64 values (all threads get the totals); uses
// red[32, 44) of the reduction scratch; ends with a barrier
__device__ inline void block_sum3(long long* red, long long& a, long long& b, long long& c) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum_ll(a); b = wave_sum_ll(b); c = wave_sum_ll(c);
    if (lane == 0) { red[32 + 3 * wid] = a; red[33 + 3 * wid] = b; red[34 + 3 * wid] = c; }
    __syncthreads();
    a = red[32] + red[35] + red[38] + red[41];
    b = red[33] + red[36] + red[39] + red[42];
    c = red[34] + red[37] + red[40] + red[43];
    __syncthreads();
}

struct Smem {
    float* A; unsigned short* I; long long* afx; long long* ps; float* adim; unsigned* pay;   // I: dims < 4096
    unsigned short* pay16;     // the same payloads in 16 bits when not keyed (level <= 7, dim < 4096)
    int* cprev; int* cnext; int* loff;
    long long* red_ll; double* red_d; float* red_f; int* misc;
};

// A window holds (level, dimension) payloads only: 32-bit for the sort
// (B >= 5, keyed = 1), which compares events through the magnitudes by
// dimension (adim), 16-bit for ranks (B <= 4).
__device__ inline Smem carve(char* base, int SA, int dp, int cap, int bb, int keyed) {
    Smem s;
    size_t o = 0;
    s.adim = keyed ? (float*)(base + o) : nullptr; o += keyed ? sizeof(float) * dp : 0;
    s.afx = (long long*)(base + o); o += sizeof(long long) * dp;
    s.ps = (long long*)(base + o); o += bb ? sizeof(long long) * (dp + 1) : 0;
    s.red_ll = (long long*)(base + o); o += sizeof(long long) * kRedLL;
    s.red_d = (double*)(base + o); o += sizeof(double) * 8;
    s.A = (float*)(base + o); o += sizeof(float) * SA;
    s.I = (unsigned short*)(base + o); o += sizeof(unsigned short) * SA;
    s.pay = (unsigned*)(base + o);
    s.pay16 = (unsigned short*)(base + o);
    o += (keyed ? sizeof(unsigned) : sizeof(unsigned short)) * cap;
    s.cprev = (int*)(base + o); o += sizeof(int) * 128;
    s.cnext = (int*)(base + o); o += sizeof(int) * 128;
    s.loff = (int*)(base + o); o += sizeof(int) * 132;
    s.red_f = (float*)(base + o); o += sizeof(float) * 8;
    s.misc = (int*)(base + o); o += sizeof(int) * 16;
    return s;
}

__host__ __device__ inline size_t smem_bytes(int SA, int dp, int cap, int bb, int keyed) {
    return (keyed ? sizeof(float) * dp : 0) + sizeof(long long) * dp + (bb ? sizeof(long long) * (dp + 1) : 0) +
           sizeof(long long) * kRedLL +
           sizeof(double) * 8 + sizeof(float) * SA + sizeof(unsigned short) * SA +
           (keyed ? sizeof(unsigned) : sizeof(unsigned short)) * cap +
           sizeof(int) * (128 + 128 + 132) + sizeof(float) * 8 + sizeof(int) * 16;
}

}  // namespace

// KEYED (B >= 5): windows are sorted, and may be pruned (bb); else (B <= 4)
// events are placed by rank with 16-bit payloads.  Each instantiation keeps
// only its own path, so the rank one fits six blocks per CU.
template <bool KEYED>
__global__ __launch_bounds__(kThreads, KEYED ? 5 : 6) void quantize_kernel(
    const float* __restrict__ rrot, int64_t n_vec, int dp, int bits, int SA, int cap,
    const float* __restrict__ norm2, uint8_t* __restrict__ codes, float* __restrict__ f_add,
    float* __restrict__ f_rescale, float* __restrict__ cos_oo, float2* __restrict__ fac, int bb)
{
    // bb != 0: windows are pruned by the bound below (needs SA+1 prefix sums in LDS)
    extern __shared__ __align__(16) char smem_raw[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int64_t row = blockIdx.x;
    if (row >= n_vec) return;
    bb = KEYED ? bb : 0;
    Smem s = carve(smem_raw, SA, dp, cap, bb, KEYED);
    const float* r = rrot + row * (int64_t)dp;
    const int K = (1 << (bits - 1)) - 1;
    const int half = 1 << (bits - 1);

    // ---- load, magnitudes, max ------------------------------------------
    float lmax = 0.0f;
    for (int i = tid; i < SA; i += kThreads) {
        float a = (i < dp) ? fabsf(r[i]) : -1.0f;
        s.A[i] = a; s.I[i] = (unsigned short)i;
        if (KEYED && i < dp) s.adim[i] = a;
        lmax = fmaxf(lmax, a);
    }
    lmax = wave_max_f(lmax);
    if (lane == 0) s.red_f[wid] = lmax;
    __syncthreads();
    const float amax = fmaxf(fmaxf(s.red_f[0], s.red_f[1]), fmaxf(s.red_f[2], s.red_f[3]));

    // ---- fixed point of a (by dimension) ---------------------------------
    int ex = 0;
    if (amax > 0.0f) { (void)frexp((double)amax, &ex); ex -= 1; }   // amax in [2^ex, 2^{ex+1})
    long long s1part = 0;
    for (int i = tid; i < dp; i += kThreads) {
        long long v = 0;
        if (amax > 0.0f) v = (long long)rint(ldexp((double)fabsf(r[i]), 40 - ex));
        s.afx[i] = v;
        s1part += v;
    }
    s1part = wave_sum_ll(s1part);
    __syncthreads();                 // red_f reads done before reuse below
    if (lane == 0) s.red_ll[wid] = s1part;

    // ---- sort a descending, ties by dimension ascending (bitonic) ---------
    for (int k = 2; k <= SA; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int t = tid; t < SA / 2; t += kThreads) {
                int i = 2 * t - (t & (j - 1));
                int p = i + j;
                bool up = ((i & k) == 0);          // "up" = descending-by-key block
                float a0 = s.A[i], a1 = s.A[p];
                int i0 = s.I[i], i1 = s.I[p];
                bool first0 = (a0 > a1) || (a0 == a1 && i0 < i1);   // element i before p
                if (first0 != up) {
                    s.A[i] = a1; s.A[p] = a0; s.I[i] = (unsigned short)i1; s.I[p] = (unsigned short)i0;
                }
            }
        }
    }
    __syncthreads();
    long long s1base = s.red_ll[0] + s.red_ll[1] + s.red_ll[2] + s.red_ll[3];
    long long s2base = dp;
    // n = number of non-zero magnitudes
    if (tid == 0) {
        int lo = 0, hi = dp;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (s.A[mid] > 0.0f) lo = mid + 1; else hi = mid; }
        s.misc[0] = lo;
    }
    for (int m = tid; m < 128; m += kThreads) s.cprev[m] = 0;
    __syncthreads();
    const int nnz = s.misc[0];
    const long long total = (long long)nnz * K;

    // ---- prefix sums of the fixed-point magnitudes in sorted order ------------
    // ps[j] = sum of afx over the j largest magnitudes, so the state after all
    // events with key >= x follows from the per-level counts alone
    if (bb) {
        const int L = (SA + kThreads - 1) / kThreads;
        const int b0 = tid * L;
        long long loc = 0;
        for (int t = 0; t < L; ++t) { const int j = b0 + t; if (j < nnz) loc += s.afx[s.I[j]]; }
        long long inc = loc;
        for (int o = 1; o < 64; o <<= 1) { const long long u = __shfl_up(inc, o); if (lane >= o) inc += u; }
        if (lane == 63) s.red_ll[24 + wid] = inc;
        __syncthreads();
        long long run = inc - loc;
        for (int w = 0; w < wid; ++w) run += s.red_ll[24 + w];
        for (int t = 0; t < L; ++t) {
            const int j = b0 + t;
            if (j <= dp) s.ps[j] = run;
            if (j < nnz) run += s.afx[s.I[j]];
        }
        if (tid == kThreads - 1 && SA == dp) s.ps[dp] = run;     // the total (else written at j = dp)
        __syncthreads();
    }
    // ---- seed: the best of a few grid points k_i = min(K, floor(t a_i)) ------
    // Any grid point's objective is at most the maximum over the critical
    // values (Algorithm 1 is exact over G), so v_seed bounds the maximum from
    // below; it only prunes, the recorded argmax still comes from enumeration.
    constexpr int kSeeds = 8;
    double v_seed = 0.0;
    if (bb && K > 0 && amax > 0.0f) {
        const double fs[kSeeds] = {0.6, 0.75, 0.85, 0.95, 1.05, 1.15, 1.3, 1.5};
        long long c1[kSeeds], c2[kSeeds];
        for (int q = 0; q < kSeeds; ++q) { c1[q] = 0; c2[q] = 0; }
        for (int i = tid; i < dp; i += kThreads) {
            const double a = (double)fabsf(r[i]);
            const long long fx = s.afx[i];
            for (int q = 0; q < kSeeds; ++q) {
                const double t = fs[q] * ((double)K + 0.5) / (double)amax;
                const long long k = (long long)fmin((double)K, floor(t * a));
                c1[q] += fx * (2 * k + 1);
                c2[q] += (2 * k + 1) * (2 * k + 1);
            }
        }
        for (int q = 0; q < kSeeds; q += 1) {
            long long z = 0;
            block_sum3(s.red_ll, c1[q], c2[q], z);
            const double v = (double)c1[q] / sqrt((double)c2[q]);
            v_seed = fmax(v_seed, v);
        }
    }
    // prune below this; the margin covers rounding in the objective
    const double v_thr = v_seed * (1.0 - 1e-12);

    // ---- windows ------------------------------------------------------------
    long long done = 0;
    double d_cur = __builtin_huge_val();
    double best_v = 0.0;            // strict improvement over 0 needed (v_max starts at 0)
    double best_d = 0.0;
    int best_i = -1;
    long long best_s2 = dp;
    const double xmin = (nnz > 0 && K > 0) ? (double)s.A[nnz - 1] / (double)K : 0.0;

    // bound of a range [xx, d_cur): S1 at its end over sqrt(S2 at its start)
    // (both only grow event by event); d1, d2, dn: the range's S1, S2 and
    // event count from the per-level counts and the prefix sums
    auto ub_at = [&](double xx, long long& d1, long long& d2, long long& dn) {
        d1 = 0; d2 = 0; dn = 0;
        if (tid < K) {
            const int hi = count_ge(s.A, nnz, tid + 1, xx), lo = s.cprev[tid];
            d1 = 2 * (s.ps[hi] - s.ps[lo]);
            d2 = 8 * (long long)(tid + 1) * (hi - lo);
            dn = hi - lo;
        }
        block_sum3(s.red_ll, d1, d2, dn);
        return (double)(s1base + d1) / sqrt((double)s2base);
    };
    // no event of a range with this bound can be the first strict maximum:
    // ub <= best_v cannot improve strictly; ub < v_thr lies below the seed
    auto prunable = [&](double ub) { return ub <= best_v || ub < v_thr; };
    // skip every event with key in [xs, d_cur): the state advances without enumeration
    auto skip_to = [&](double xs) {
        long long d1, d2, dn;
        if (tid < K) s.cnext[tid] = count_ge(s.A, nnz, tid + 1, xs);
        ub_at(xs, d1, d2, dn);
        s1base += d1;
        s2base += d2;
        done += dn;
        d_cur = xs;
        __syncthreads();
        if (tid < K) s.cprev[tid] = s.cnext[tid];
        __syncthreads();
        return dn;
    };
    // the smallest x in [xmin, xhi] whose range [x, d_cur) is prunable, given
    // that [xhi, d_cur) is (bisection on the bit pattern of the double)
    auto farthest_prunable = [&](double xhi) {
        long long e1, e2, en;
        if (prunable(ub_at(xmin, e1, e2, en))) return xmin;
        unsigned long long lo_b = __double_as_longlong(xmin);
        unsigned long long hi_b = __double_as_longlong(xhi);
        for (int it = 0; it < 40 && hi_b - lo_b > 1; ++it) {
            const unsigned long long mid_b = lo_b + ((hi_b - lo_b) >> 1);
            if (prunable(ub_at(__longlong_as_double(mid_b), e1, e2, en))) hi_b = mid_b;
            else lo_b = mid_b;
        }
        return __longlong_as_double(hi_b);
    };

    for (int guard = 0; done < total && guard < (1 << 22); ++guard) {
        // choose x: all remaining if they fit, else bisect on the bit pattern
        double x;
        {
            const long long remain = total - done;
            if (remain <= cap) {
                x = xmin;
            } else {
                unsigned long long lo_b = __double_as_longlong(xmin);   // cnt(lo) - done > cap
                unsigned long long hi_b = __double_as_longlong(d_cur);  // cnt(hi) - done == 0 (or small)
                x = d_cur;
                while (true) {
                    unsigned long long mid_b = lo_b + ((hi_b - lo_b) >> 1);
                    double xm = __longlong_as_double(mid_b);
                    if (tid == 0) s.misc[1] = 0;
                    __syncthreads();
                    if (tid < K) atomicAdd(&s.misc[1], count_ge(s.A, nnz, tid + 1, xm));
                    __syncthreads();
                    long long c = (long long)s.misc[1] - done;
                    __syncthreads();
                    if (c > cap) lo_b = mid_b;
                    else {
                        hi_b = mid_b;
                        x = xm;
                        if (2 * c >= cap) break;
                    }
                    if (hi_b - lo_b <= 1) break;
                }
            }
        }
        // per-level ranges [cprev[m], cnext[m]) and their offsets
        if (tid < K) s.cnext[tid] = count_ge(s.A, nnz, tid + 1, x);
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int m = 0; m < K; ++m) { s.loff[m] = acc; acc += s.cnext[m] - s.cprev[m]; }
            s.loff[K] = acc;
        }
        __syncthreads();
        const int W = s.loff[K];
        if (W <= 0) break;            // cannot happen (a tie group has <= dp <= cap/2 events); never spin
        // ---- bound: every objective in the window is at most
        //      UB = (S1 at its end) / sqrt(S2 at its start); S1, S2 only grow.
        //      UB <= best_v: no strict improvement; UB < v_thr: below the seed,
        //      hence below the maximum.  Such a window is skipped, and the skip
        //      is extended as far as the bound allows (bisection).
        if (bb) {
            long long d1, d2, dn;
            if (prunable(ub_at(x, d1, d2, dn))) {
                skip_to(farthest_prunable(x));
                continue;
            }
        }
        int S = 1;
        while (S < W) S <<= 1;
        if (!KEYED) {
            // few levels (B <= 4): ranks, no sort stages
            // every event of the window goes straight to its rank by (d desc, dim
            // asc): its rank in its own level's run (sorted by a descending, dim
            // ascending, so by d descending) plus, for every other level, the
            // number of that run's window events before it, by binary search.
            // a'/m' > a/m is decided as a'*m > a*m', exact in double (24-bit
            // magnitudes times levels below 2^7), which orders the events as
            // their keys do (distinct ratios give distinct keys in the same order)
            for (int t = tid; t < W; t += kThreads) {
                int lo = 0, hi = K;            // largest m with loff[m] <= t
                while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (s.loff[mid] <= t) lo = mid; else hi = mid; }
                const int m = lo + 1;
                const int j = s.cprev[lo] + (t - s.loff[lo]);
                const float a = s.A[j];
                const int dim = s.I[j];
                int rank = t - s.loff[lo];
                for (int l2 = 0; l2 < K; ++l2) {
                    if (l2 == lo) continue;
                    const double am2 = (double)a * (double)(l2 + 1);
                    int b = s.cprev[l2], e = s.cnext[l2];
                    while (b < e) {                // first event of run l2 that does not come before
                        const int mid = (b + e) >> 1;
                        const double pm = (double)s.A[mid] * (double)m;
                        if (pm > am2 || (pm == am2 && s.I[mid] < dim)) b = mid + 1;
                        else e = mid;
                    }
                    rank += b - s.cprev[l2];
                }
                s.pay16[rank] = (unsigned short)((m << 12) | dim);
            }
            __syncthreads();
        } else {
            // many levels: gather, then a bitonic sort of the window
            // gather
            for (int t = tid; t < S; t += kThreads) {
                if (t < W) {
                    int lo = 0, hi = K;            // largest m with loff[m] <= t
                    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (s.loff[mid] <= t) lo = mid; else hi = mid; }
                    int m = lo + 1;
                    int j = s.cprev[lo] + (t - s.loff[lo]);
                    s.pay[t] = ((unsigned)m << 12) | (unsigned)s.I[j];
                } else {
                    s.pay[t] = 0xFFFFFFFFu;
                }
            }
            // bitonic sort of the window by (d desc, dim asc)
            for (int k = 2; k <= S; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    __syncthreads();
                    for (int t = tid; t < S / 2; t += kThreads) {
                        int i = 2 * t - (t & (j - 1));
                        int p = i + j;
                        bool up = ((i & k) == 0);
                        unsigned p0 = s.pay[i], p1 = s.pay[p];
                        bool first0 = ev_before(s.adim, p0, p1);
                        if (first0 != up) { s.pay[i] = p1; s.pay[p] = p0; }
                    }
                }
            }
            __syncthreads();
        }
        // integer prefix sums over the window; each thread owns a contiguous chunk
        const int L = (S + kThreads - 1) / kThreads;
        const int beg = tid * L, end = min(W, beg + L);
        long long ls1 = 0, ls2 = 0;
        for (int t = beg; t < end; ++t) {
            unsigned pp = KEYED ? s.pay[t] : (unsigned)s.pay16[t];
            ls1 += 2 * s.afx[pp & 0xFFFu];
            ls2 += 8 * (long long)(pp >> 12);
        }
        // block exclusive scan of (ls1, ls2)
        long long i1 = ls1, i2 = ls2;
        for (int o = 1; o < 64; o <<= 1) {
            long long u1 = __shfl_up(i1, o), u2 = __shfl_up(i2, o);
            if (lane >= o) { i1 += u1; i2 += u2; }
        }
        if (lane == 63) { s.red_ll[2 * wid] = i1; s.red_ll[2 * wid + 1] = i2; }
        __syncthreads();
        long long w1 = 0, w2 = 0;
        for (int w = 0; w < wid; ++w) { w1 += s.red_ll[2 * w]; w2 += s.red_ll[2 * w + 1]; }
        const long long tot1 = s.red_ll[0] + s.red_ll[2] + s.red_ll[4] + s.red_ll[6];
        const long long tot2 = s.red_ll[1] + s.red_ll[3] + s.red_ll[5] + s.red_ll[7];
        long long c1 = s1base + w1 + i1 - ls1;
        long long c2 = s2base + w2 + i2 - ls2;
        double tb = 0.0; int tpos = -1; long long ts2 = 0;
        for (int t = beg; t < end; ++t) {
            unsigned pp = KEYED ? s.pay[t] : (unsigned)s.pay16[t];
            c1 += 2 * s.afx[pp & 0xFFFu];
            c2 += 8 * (long long)(pp >> 12);
            double v = (double)c1 / sqrt((double)c2);
            if (v > tb) { tb = v; tpos = t; ts2 = c2; }
        }
        // block argmax: largest v, earliest position
        __syncthreads();
        {
            double bv = tb; int bp = (tpos < 0) ? 0x7FFFFFFF : tpos; long long bs2 = ts2;
            for (int o = 32; o > 0; o >>= 1) {
                double ov = __shfl_xor(bv, o);
                int op = __shfl_xor(bp, o);
                long long os2 = __shfl_xor(bs2, o);
                if (ov > bv || (ov == bv && op < bp)) { bv = ov; bp = op; bs2 = os2; }
            }
            if (lane == 0) { s.red_d[wid] = bv; s.misc[4 + wid] = bp; s.red_ll[16 + wid] = bs2; }
        }
        __syncthreads();
        {
            double bv = s.red_d[0]; int bp = s.misc[4]; long long bs2 = s.red_ll[16];
            for (int w = 1; w < 4; ++w) {
                double ov = s.red_d[w]; int op = s.misc[4 + w];
                if (ov > bv || (ov == bv && op < bp)) { bv = ov; bp = op; bs2 = s.red_ll[16 + w]; }
            }
            if (bp != 0x7FFFFFFF && bv > best_v) {
                best_v = bv;
                const unsigned bpay = KEYED ? s.pay[bp] : (unsigned)s.pay16[bp];
                best_i = (int)(bpay & 0xFFFu);
                // the key of the best event, as the sort would have stored it
                best_d = (double)(KEYED ? s.adim[best_i] : fabsf(r[best_i])) / (double)(bpay >> 12);
                best_s2 = bs2;
            }
        }
        s1base += tot1;
        s2base += tot2;
        done += W;
        d_cur = x;
        __syncthreads();
        if (tid < K) s.cprev[tid] = s.cnext[tid];
        __syncthreads();
    }

    // ---- replay: levels of the state at the best event ------------------------
    if (tid < K) s.cnext[tid] = (best_i >= 0) ? count_upto(s.A, s.I, nnz, tid + 1, best_d, best_i) : 0;
    __syncthreads();
    double ip = 0.0;
    uint8_t* crow = codes + row * (int64_t)dp;
    for (int j = tid; j < dp; j += kThreads) {
        int lev = 0;
        if (j < nnz && K > 0) {
            int lo = 0, hi = K;            // k = #{m : cnext[m-1] > j}, non-increasing in m
            while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (s.cnext[mid - 1] > j) lo = mid; else hi = mid - 1; }
            lev = lo;
        }
        int dim = s.I[j];
        float rv = r[dim];
        bool pos = !(rv < 0.0f);
        crow[dim] = (uint8_t)(pos ? half + lev : half - 1 - lev);
        ip += ((double)lev + 0.5) * (double)fabsf(rv);
    }
    // ||r||^2
    double nr = 0.0;
    if (norm2 == nullptr)
        for (int i = tid; i < dp; i += kThreads) { double v = (double)r[i]; nr += v * v; }
    ip = wave_sum_d(ip);
    nr = wave_sum_d(nr);
    __syncthreads();
    if (lane == 0) { s.red_d[wid] = ip; s.red_d[4 + wid] = nr; }
    __syncthreads();
    if (tid == 0) {
        double ipt = (s.red_d[0] + s.red_d[1]) + (s.red_d[2] + s.red_d[3]);
        double nr2 = norm2 ? (double)norm2[row] : (s.red_d[4] + s.red_d[5]) + (s.red_d[6] + s.red_d[7]);
        double ny = (double)best_s2 * 0.25;
        if (best_i < 0) ny = 0.25 * dp;
        float fa = 0.0f, fr = 0.0f, co = 1.0f;
        if (nr2 > 0.0 && ipt > 0.0) {
            fa = (float)nr2;
            fr = (float)(-2.0 * nr2 / ipt);
            co = (float)(ipt / (sqrt(ny) * sqrt(nr2)));
        }
        if (f_add) f_add[row] = fa;
        if (f_rescale) f_rescale[row] = fr;
        if (cos_oo) cos_oo[row] = co;
        if (fac) fac[row] = make_float2(fa, fr);
    }
}

hipError_t launch_quantize(const float* rrot, int64_t n, int dp, int bits, const float* norm2,
                           uint8_t* codes, float* f_add, float* f_rescale, float* cos_oo,
                           float2* fac, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int SA = 1;
    while (SA < dp) SA <<= 1;
    int cap = 1;
    while (cap < 2 * dp) cap <<= 1;
    // B >= 5 (sorted windows, pruned or bisected): 2048 keeps three blocks
    // per CU at dp 768; the window must stay a power of two >= 2 dp
    const int cap_floor = bits >= 5 ? 2048 : 4096;
    if (cap < cap_floor) cap = cap_floor;
    // pruning pays off from B = 5 (15+ levels, many windows per vector) and
    // needs its prefix sums to fit in LDS
    const int keyed = bits >= 5;
    int bb = (bits >= 5 && smem_bytes(SA, dp, cap, 1, keyed) <= 160 * 1024) ? 1 : 0;
    // ranks (B <= 4): one window for all of a vector's events when their
    // payloads fit in a third of the LDS (at least three blocks per CU): no
    // bisection for the window ends
    if (!keyed) {
        const int K = (1 << (bits - 1)) - 1;
        const int call = (K * dp + 63) & ~63;
        if (call > cap && smem_bytes(SA, dp, call, 0, 0) <= 53 * 1024) cap = call;
    }
    size_t sm = smem_bytes(SA, dp, cap, bb, keyed);
    const void* fn = keyed ? (const void*)quantize_kernel<true> : (const void*)quantize_kernel<false>;
    if (sm > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    if (keyed)
        hipLaunchKernelGGL(quantize_kernel<true>, dim3((unsigned)n), dim3(kThreads), sm, st,
                           rrot, n, dp, bits, SA, cap, norm2, codes, f_add, f_rescale, cos_oo, fac, bb);
    else
        hipLaunchKernelGGL(quantize_kernel<false>, dim3((unsigned)n), dim3(kThreads), sm, st,
                           rrot, n, dp, bits, SA, cap, norm2, codes, f_add, f_rescale, cos_oo, fac, bb);
    return hipGetLastError();
}

}  // namespace erq
