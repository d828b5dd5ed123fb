/*
 * erq_oracle.c -- slow, plain CPU reference of Extended RaBitQ
 * (Gao et al., "Practical and Asymptotically Optimal Quantization of
 * High-Dimensional Vectors in Euclidean Space for Approximate Nearest
 * Neighbor Search", arXiv 2409.09913).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Style: scalar loops, FP64 for everything the paper states in real numbers;
 * FP32 only where a decision is taken in the GPU kernel's own precision (the
 * int8 query quantisation, which the paper does not have).  OpenMP is used
 * only across independent vectors / queries.  Build:
 *   gcc -O2 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off erq_oracle.c -lm
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Rotation.  Sec. 3.2.1 / Sec. 3.4: data and queries are multiplied by      */
/* P^{-1} = P^T.  With row vectors, r'^T = r^T P, i.e. out = x * P.          */
/* ------------------------------------------------------------------------ */
void orc_rotate(const double* x, int64_t n, int dp, const double* P, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const double* xr = x + r * (int64_t)dp;
        double* orow = out + r * (int64_t)dp;
        for (int j = 0; j < dp; ++j) orow[j] = 0.0;
        for (int k = 0; k < dp; ++k) {
            double xv = xr[k];
            const double* prow = P + (int64_t)k * dp;
            for (int j = 0; j < dp; ++j) orow[j] += xv * prow[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Quantize), Sec. 3.2.2.                                       */
/*                                                                          */
/* Work in the orthant of o' (Lemma 3.1 footnote): a_i = |o'_i|, sign s_i    */
/* (reading: sgn(0) = +1, as in App. B).  A grid point of G in that orthant  */
/* is y_i = s_i (k_i + 1/2), k_i in {0..K}, K = 2^{B-1}-1.  Rounding t*o'    */
/* to the nearest point of G gives k_i = min(K, floor(t a_i)); k_i moves     */
/* from m-1 to m at the critical value t = m / a_i, m = 1..K.                */
/*                                                                          */
/* The critical values are visited in ascending order with a min-heap (the   */
/* paper's O(2^B D log D) method).  Readings:                               */
/*  - order: t = m/a_i compared exactly (m*a_j vs m'*a_i as an error-free   */
/*    two-product); equal t broken by the dimension index, ascending.       */
/*  - after every single event the objective <y,o'>/||y|| is evaluated and  */
/*    kept if strictly larger than the best so far (v_max starts at 0, so   */
/*    the t = 0 state itself is never a candidate).                          */
/*  - arithmetic of the objective: 2<y,o'> is accumulated exactly as an     */
/*    int64 fixed point (a_i scaled by the power of two that puts max a in  */
/*    [1,2), 40 fractional bits, round-half-even) and 4||y||^2 exactly as an */
/*    integer; v = double(2S1) / sqrt(double(4S2)), correctly rounded.       */
/*    This makes the sums independent of summation order.                   */
/*  - the returned code is the state reached at the best event (a replay of */
/*    the enumeration), not a re-rounding of t_max * o', which at t_max     */
/*    sits exactly on a rounding boundary.                                  */
/*  - B = 1 has no critical values; the code is the sign pattern (RaBitQ).  */
/* Output code: y_u = y + (2^B - 1)/2, i.e. 2^{B-1}+k_i for s_i = +1 and     */
/* 2^{B-1}-1-k_i for s_i = -1.                                              */
/* ------------------------------------------------------------------------ */

typedef struct { int m; int i; } orc_event;

/* exact comparison of t_a = ma / a[ia] and t_b = mb / a[ib] (a > 0):
   t_a < t_b  <=>  ma * a[ib] < mb * a[ia].  Each product is represented
   exactly as (p, e) with p = fl(x), e = x - p (fma), then compared
   lexicographically; ties in t fall back to the dimension index. */
static int orc_ev_less(orc_event x, orc_event y, const double* a)
{
    double p1 = (double)x.m * a[y.i];
    double e1 = fma((double)x.m, a[y.i], -p1);
    double p2 = (double)y.m * a[x.i];
    double e2 = fma((double)y.m, a[x.i], -p2);
    if (p1 != p2) return p1 < p2;
    if (e1 != e2) return e1 < e2;
    return x.i < y.i;
}

static void orc_heap_push(orc_event* h, int* n, orc_event v, const double* a)
{
    int c = (*n)++;
    h[c] = v;
    while (c > 0) {
        int p = (c - 1) / 2;
        if (!orc_ev_less(h[c], h[p], a)) break;
        orc_event t = h[c]; h[c] = h[p]; h[p] = t;
        c = p;
    }
}

static orc_event orc_heap_pop(orc_event* h, int* n, const double* a)
{
    orc_event top = h[0];
    h[0] = h[--(*n)];
    int c = 0;
    for (;;) {
        int l = 2 * c + 1, r = l + 1, s = c;
        if (l < *n && orc_ev_less(h[l], h[s], a)) s = l;
        if (r < *n && orc_ev_less(h[r], h[s], a)) s = r;
        if (s == c) break;
        orc_event t = h[c]; h[c] = h[s]; h[s] = t;
        c = s;
    }
    return top;
}

/* Runs the enumeration.  If stop_after >= 0, stops after that many events
   and leaves the levels in k[]; otherwise runs to the end and returns the
   1-based index of the best event (0 = no event) and its objective. */
static int64_t orc_enumerate(const double* a, const int64_t* afx, int dp, int K,
                             int64_t stop_after, int* k, orc_event* heap,
                             double* vbest_out)
{
    int hn = 0;
    int64_t s1 = 0, s2 = dp;               /* 2*S1 (fixed point), 4*S2 */
    for (int i = 0; i < dp; ++i) { k[i] = 0; s1 += afx[i]; }
    if (K >= 1)
        for (int i = 0; i < dp; ++i)
            if (a[i] > 0.0) { orc_event e = {1, i}; orc_heap_push(heap, &hn, e, a); }
    double vmax = 0.0;
    int64_t best = 0, count = 0;
    while (hn > 0) {
        if (stop_after >= 0 && count == stop_after) break;
        orc_event e = orc_heap_pop(heap, &hn, a);
        ++count;
        k[e.i] = e.m;
        s1 += 2 * afx[e.i];
        s2 += 8 * (int64_t)e.m;               /* (2m+1)^2 - (2m-1)^2 */
        double v = (double)s1 / sqrt((double)s2);
        if (v > vmax) { vmax = v; best = count; }
        if (e.m < K) { orc_event nx = {e.m + 1, e.i}; orc_heap_push(heap, &hn, nx, a); }
    }
    if (vbest_out) *vbest_out = vmax;
    return best;
}

/* Quantise one rotated vector o' (any positive scale) to B bits.
   Outputs: code[dp] (y_u), *ip_y_o = <y, o'> (FP64), *norm_y2 = ||y||^2,
   *n_events = number of critical values enumerated.  Returns 0, or -1 on a
   bad argument. */
int orc_quantize_one(const double* o, int dp, int B, uint8_t* code,
                     double* ip_y_o, double* norm_y2, int64_t* n_events)
{
    if (dp <= 0 || B < 1 || B > 8) return -1;
    const int K = (1 << (B - 1)) - 1;
    const int half = 1 << (B - 1);
    double* a = (double*)malloc(sizeof(double) * dp);
    int64_t* afx = (int64_t*)malloc(sizeof(int64_t) * dp);
    int* k = (int*)malloc(sizeof(int) * dp);
    orc_event* heap = (orc_event*)malloc(sizeof(orc_event) * (dp + 1));
    double amax = 0.0;
    for (int i = 0; i < dp; ++i) { a[i] = fabs(o[i]); if (a[i] > amax) amax = a[i]; }
    int64_t nev = 0;
    if (amax > 0.0) {
        int e = ilogb(amax);                    /* amax in [2^e, 2^{e+1}) */
        for (int i = 0; i < dp; ++i) afx[i] = llrint(ldexp(a[i], 40 - e));
        int64_t best = orc_enumerate(a, afx, dp, K, -1, k, heap, NULL);
        for (int i = 0; i < dp; ++i) if (a[i] > 0.0) nev += K;
        orc_enumerate(a, afx, dp, K, best, k, heap, NULL);   /* replay */
    } else {
        for (int i = 0; i < dp; ++i) k[i] = 0;
    }
    double ip = 0.0, ny = 0.0;
    for (int i = 0; i < dp; ++i) {
        int pos = !(o[i] < 0.0);                 /* sgn(0) = +1 */
        double y = (pos ? 1.0 : -1.0) * (k[i] + 0.5);
        code[i] = (uint8_t)(pos ? half + k[i] : half - 1 - k[i]);
        ip += y * o[i];
        ny += y * y;
    }
    if (ip_y_o) *ip_y_o = ip;
    if (norm_y2) *norm_y2 = ny;
    if (n_events) *n_events = nev;
    free(a); free(afx); free(k); free(heap);
    return 0;
}

/* The objective <y,o'>/||y|| of Eq. (eq 3.2: optimization) for a given code,
   in FP64 (used by tests to compare codes by value). */
double orc_objective(const double* o, int dp, int B, const uint8_t* code)
{
    double ip = 0.0, ny = 0.0, off = ((double)((1 << B) - 1)) / 2.0;
    for (int i = 0; i < dp; ++i) {
        double y = (double)code[i] - off;
        ip += y * o[i];
        ny += y * y;
    }
    return ip / sqrt(ny);
}

/* Batched quantisation of n rotated vectors, with the two per-vector
   factors of Sec. 3.3 / Sec. 5.1.  norm2[r] = ||o_r - c||^2 (the caller
   passes it; NULL -> ||o'||^2).  Factors (reading of the two stored floats):
     f_add     = ||r||^2
     f_rescale = -2 ||r||^2 / <y, r'>
   so that est = f_add + ||s||^2 + f_rescale * <y, s'>  equals
   Eq. (eq:dis to ip) with <o,q> replaced by <o_bar,q>/<o_bar,o> and
   <o_bar,q> from Eq. (eq 3.3: represent).  cos_oo[r] = <o_bar, o>.
   A zero residual gives f_add = f_rescale = 0 (distance = ||s||^2). */
int orc_quantize(const double* rrot, int64_t n, int dp, int B, const double* norm2,
                 uint8_t* codes, double* f_add, double* f_rescale, double* cos_oo)
{
    if (dp <= 0 || B < 1 || B > 8 || n < 0) return -1;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(|:bad)
    for (int64_t r = 0; r < n; ++r) {
        const double* o = rrot + r * (int64_t)dp;
        double ip, ny;
        if (orc_quantize_one(o, dp, B, codes + r * (int64_t)dp, &ip, &ny, NULL) != 0) { bad = 1; continue; }
        double nr2;
        if (norm2) nr2 = norm2[r];
        else { nr2 = 0.0; for (int i = 0; i < dp; ++i) nr2 += o[i] * o[i]; }
        if (nr2 > 0.0 && ip > 0.0) {
            f_add[r] = nr2;
            f_rescale[r] = -2.0 * nr2 / ip;
            if (cos_oo) cos_oo[r] = ip / (sqrt(ny) * sqrt(nr2));
        } else {
            f_add[r] = 0.0; f_rescale[r] = 0.0;
            if (cos_oo) cos_oo[r] = 1.0;
        }
    }
    return bad ? -1 : 0;
}

/* Index phase of Sec. 3.4 with IVF centring (Sec. 4.1, Sec. 5.1): for every
   vector, r = x - c_{list(x)}, ||r||^2, r' = P^T r, then Algorithm 1 and the
   factors.  assign[r] = list of row r; cent is C x dp.  Also returns r' (FP64)
   if rrot_out != NULL. */
int orc_encode(const double* x, int64_t n, int dp, const double* cent,
               const int32_t* assign, const double* P, int B,
               uint8_t* codes, double* f_add, double* f_rescale, double* cos_oo,
               double* rrot_out)
{
    if (dp <= 0 || B < 1 || B > 8 || n < 0) return -1;
    double* rr = rrot_out ? rrot_out : (double*)malloc(sizeof(double) * (size_t)n * dp);
    double* nr2 = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* res = (double*)malloc(sizeof(double) * (size_t)n * dp);
    for (int64_t r = 0; r < n; ++r) {
        const double* c = cent + (int64_t)assign[r] * dp;
        double s = 0.0;
        for (int i = 0; i < dp; ++i) {
            double v = x[r * (int64_t)dp + i] - c[i];
            res[r * (int64_t)dp + i] = v;
            s += v * v;
        }
        nr2[r] = s;
    }
    orc_rotate(res, n, dp, P, rr);
    int rc = orc_quantize(rr, n, dp, B, nr2, codes, f_add, f_rescale, cos_oo);
    free(res); free(nr2);
    if (!rrot_out) free(rr);
    return rc;
}

/* Encoding with a random projection to d < D dimensions before quantising
   (App. C): the estimate of <r, s> is (D/d) <P_d r, P_d s> (Johnson-
   Lindenstrauss), and the inner product of the d-dimensional projections is
   estimated by the extended codes.  With r'_d = the first d coordinates of
   P^T r (P^T r rotated by the full P, then cut to d rows = a d x D random
   orthogonal projection), the two stored floats are
     f_add = ||r||^2 (all D coordinates),
     f_rescale = -(2 D / d) ||r'_d||^2 / <y, r'_d>,
   so est = f_add + ||s||^2 + f_rescale <y, s'_d> with ||s||^2 over all D
   coordinates.  d == D is orc_encode. */
int orc_encode_proj(const double* x, int64_t n, int dp, int dc, const double* cent,
                    const int32_t* assign, const double* P, int B,
                    uint8_t* codes, double* f_add, double* f_rescale)
{
    if (dp <= 0 || dc <= 0 || dc > dp || B < 1 || B > 8 || n < 0) return -1;
    double* res = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * dp);
    double* rr = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * dp);
    double* rd = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * dc);
    double* nr2 = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* co = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t r = 0; r < n; ++r) {
        const double* c = cent + (int64_t)assign[r] * dp;
        double s = 0.0;
        for (int i = 0; i < dp; ++i) {
            const double v = x[r * (int64_t)dp + i] - c[i];
            res[r * (int64_t)dp + i] = v;
            s += v * v;
        }
        nr2[r] = s;
    }
    orc_rotate(res, n, dp, P, rr);
    for (int64_t r = 0; r < n; ++r)
        for (int i = 0; i < dc; ++i) rd[r * (int64_t)dc + i] = rr[r * (int64_t)dp + i];
    int rc = orc_quantize(rd, n, dc, B, NULL, codes, f_add, f_rescale, co);    /* norm2 = ||r'_d||^2 */
    for (int64_t r = 0; r < n; ++r) {
        f_rescale[r] *= (double)dp / (double)dc;
        f_add[r] = nr2[r];
    }
    free(res); free(rr); free(rd); free(nr2); free(co);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Query side.                                                               */
/* ------------------------------------------------------------------------ */

/* int8 quantisation of a rotated query q' (FP32), once per query.  The
   paper keeps q' in floating point (Sec. 3.3); the symmetric int8 form is
   this implementation's addition (reading), decided in FP32 exactly as the
   kernel does: amax = max|q'_i|, inv = 127/amax,
   q_i = clamp(rint(q'_i * inv), -127, 127) (round half to even),
   delta = amax/127; amax = 0 gives zeros. */
void orc_query_quant(const float* s, int dp, int8_t* sq, float* delta, int32_t* ssum)
{
    float amax = 0.0f;
    for (int i = 0; i < dp; ++i) { float v = fabsf(s[i]); if (v > amax) amax = v; }
    int32_t sum = 0;
    if (amax > 0.0f) {
        float inv = 127.0f / amax;
        for (int i = 0; i < dp; ++i) {
            float t = rintf(s[i] * inv);
            int v = (int)t;
            if (v > 127) v = 127;
            if (v < -127) v = -127;
            sq[i] = (int8_t)v;
            sum += v;
        }
        *delta = amax / 127.0f;
    } else {
        for (int i = 0; i < dp; ++i) sq[i] = 0;
        *delta = 0.0f;
    }
    *ssum = sum;
}

/* Estimated squared distance with a float query, Eq. (eq:dis to ip) and
   Eq. (eq 3.3: represent), in FP64:
     <o_bar, q> = ( <y_u, q'> - (2^B-1)/2 * sum q'_i ) / ||y||  with q' = s'/||s||
     est = ||r||^2 + ||s||^2 - 2 ||r|| ||s|| <o_bar,q> / <o_bar,o>.
   Inputs: code (y_u), s' (FP64, rotated query residual), ||r||^2 and
   <o_bar,o> of the vector. */
double orc_est_paper(const uint8_t* code, int dp, int B, const double* s,
                     double norm_r2, double cos_oo)
{
    double ns2 = 0.0;
    for (int i = 0; i < dp; ++i) ns2 += s[i] * s[i];
    if (norm_r2 <= 0.0) return ns2;
    double ns = sqrt(ns2);
    if (ns == 0.0) return norm_r2;
    double ipu = 0.0, qs = 0.0, ny = 0.0, off = ((double)((1 << B) - 1)) / 2.0;
    for (int i = 0; i < dp; ++i) {
        double q = s[i] / ns;
        ipu += (double)code[i] * q;
        qs += q;
        double y = (double)code[i] - off;
        ny += y * y;
    }
    double obq = (ipu - off * qs) / sqrt(ny);
    return norm_r2 + ns2 - 2.0 * sqrt(norm_r2) * ns * obq / cos_oo;
}

/* Estimated squared distance with the int8 query (factor form), FP64.
   The residual of the list is s' = q' - c' (rotation is linear), so
     <y, s'> = <y, q'> - <y, c'>,   y = y_u - (2^B-1)/2 (centred code),
   and with q' ~= delta * q_int:
     2<y, q'> ~= delta * ( 2<y_u, q_int> - (2^B-1) * sum q_int )
     est = f_add + ||s||^2 + f_rescale * <y, s'>          (Eq. eq:dis to ip).
   ip_u = <y_u, q_int> is an exact integer; ybc = <y, c'>. */
static double orc_est_int8(int64_t ip_u, int32_t qsum, int B, double delta, double ybc,
                           double ns2, double f_add, double f_rescale)
{
    double two_ip = delta * (double)(2 * ip_u - (int64_t)((1 << B) - 1) * qsum);
    return f_add + ns2 + f_rescale * (0.5 * two_ip - ybc);
}

/* Two int8 planes of the query (this implementation's addition for large B,
   where the one-plane rounding error Delta/2 per coordinate is as large as
   the estimator's own error): with t_i = q'_i * inv (FP32, inv = 127/amax
   as in orc_query_quant), q_hi = clamp(rint(t_i), +-127) is the one-plane
   code, and the remainder t_i - q_hi (exact in FP32, in [-1/2, 1/2]) is
   quantised again with 254 levels per unit, q_lo = rint((t_i - q_hi) * 254)
   (in [-127, 127]), so that q' ~= delta * (q_hi + q_lo / 254), decided in
   FP32 exactly as the kernel does. */
void orc_query_quant2(const float* s, int dp, int8_t* sh, int8_t* sl, float* delta, int32_t* sum_hi,
                      int32_t* sum_lo)
{
    orc_query_quant(s, dp, sh, delta, sum_hi);
    int32_t sum = 0;
    float amax = 0.0f;
    for (int i = 0; i < dp; ++i) { float v = fabsf(s[i]); if (v > amax) amax = v; }
    if (amax > 0.0f) {
        const float inv = 127.0f / amax;
        for (int i = 0; i < dp; ++i) {
            const float t = s[i] * inv;
            const float r = t - (float)sh[i];
            int v = (int)rintf(r * 254.0f);
            if (v > 127) v = 127;
            if (v < -127) v = -127;
            sl[i] = (int8_t)v;
            sum += v;
        }
    } else {
        for (int i = 0; i < dp; ++i) sl[i] = 0;
    }
    *sum_lo = sum;
}

/* The int8 estimator with the two query planes: 2<y, q'> ~= delta * ((2
   ip_hi - (2^B-1) sum q_hi) + (2 ip_lo - (2^B-1) sum q_lo) / 254). */
static double orc_est_int8x2(int64_t ip_hi, int64_t ip_lo, int32_t qs_hi, int32_t qs_lo, int B, double delta,
                             double ybc, double ns2, double f_add, double f_rescale)
{
    const int64_t m = (1 << B) - 1;
    const double two_ip = delta * ((double)(2 * ip_hi - m * qs_hi) + (double)(2 * ip_lo - m * qs_lo) / 254.0);
    return f_add + ns2 + f_rescale * (0.5 * two_ip - ybc);
}

/* ------------------------------------------------------------------------ */
/* Ordering helpers: ascending (value, id).                                  */
/* ------------------------------------------------------------------------ */
typedef struct { double d; int64_t id; } orc_cand;

static int orc_cand_cmp(const void* pa, const void* pb)
{
    const orc_cand* x = (const orc_cand*)pa;
    const orc_cand* y = (const orc_cand*)pb;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

/* keep the k smallest of cand[0..n) in out (sorted); pad with (+inf, -1). */
static void orc_take_k(orc_cand* cand, int64_t n, int k, int64_t* ids, double* dists)
{
    qsort(cand, (size_t)n, sizeof(orc_cand), orc_cand_cmp);
    for (int j = 0; j < k; ++j) {
        if (j < n) { ids[j] = cand[j].id; dists[j] = cand[j].d; }
        else { ids[j] = -1; dists[j] = INFINITY; }
    }
}

/* Coarse probe of IVF (Sec. 4.1): the nprobe centroids nearest to q in FP64
   squared Euclidean distance, ties broken by the centroid index. */
void orc_probe(const float* q, int64_t nq, const float* cent, int64_t C, int dp,
               int nprobe, int32_t* probes, double* pdist)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)C);
        int64_t* tid = (int64_t*)malloc(sizeof(int64_t) * (size_t)nprobe);
        double* td = (double*)malloc(sizeof(double) * (size_t)nprobe);
        #pragma omp for schedule(dynamic, 4)
        for (int64_t iq = 0; iq < nq; ++iq) {
            const float* qv = q + iq * (int64_t)dp;
            for (int64_t j = 0; j < C; ++j) {
                const float* cv = cent + j * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) { double d = (double)qv[i] - (double)cv[i]; s += d * d; }
                c[j].d = s; c[j].id = j;
            }
            orc_take_k(c, C, nprobe, tid, td);
            for (int j = 0; j < nprobe; ++j) {
                probes[iq * nprobe + j] = (int32_t)tid[j];
                if (pdist) pdist[iq * nprobe + j] = td[j];
            }
        }
        free(c); free(tid); free(td);
    }
}

int orc_search_ld(const int64_t* list_off, const int64_t* ids, const uint8_t* codes,
                  const float* f_add, const float* f_rescale, const double* cos_oo,
                  const float* crot, int64_t C, int dp, int ld, int B,
                  const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
                  int kk, int est_mode, int64_t* out_ids, double* out_d);

/* IVF search with the int8 estimator (Sec. 4.1 with Sec. 3.3).  Index:
   list_off[C+1], ids[N] (row ids), codes[N x dp] (y_u, list order),
   f_add/f_rescale[N] (FP32 as stored), crot[C x dp] rotated centroids (FP32).
   Queries: qrot[nq x dp] rotated (FP32), probes[nq x nprobe].  Every query
   is quantised to int8 once; for every probed list s' = q' - c' and ||s||^2
   in FP64 (exact differences of the FP32 inputs); every member gets an
   estimate; the kk smallest (est, id) are returned.  est_mode 3 = the
   int8 query in two planes (orc_query_quant2); est_mode 2 = float
   query with the stored factors (f_add + ||s||^2 + f_rescale <y, s'>, FP64);
   est_mode 0 = int8 query
   (factor form), 1 = float query (paper form, uses cos_oo). */
int orc_search(const int64_t* list_off, const int64_t* ids, const uint8_t* codes,
               const float* f_add, const float* f_rescale, const double* cos_oo,
               const float* crot, int64_t C, int dp, int B,
               const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
               int kk, int est_mode, int64_t* out_ids, double* out_d)
{
    return orc_search_ld(list_off, ids, codes, f_add, f_rescale, cos_oo, crot, C, dp, dp, B, qrot, nq, probes,
                         nprobe, kk, est_mode, out_ids, out_d);
}

/* The scan of orc_search when the codes cover only the first dp of the ld
   coordinates of the rotated queries and centroids (the projection of
   App. C): ||s||^2 is taken over all ld coordinates, everything else over the
   first dp.  ld == dp is orc_search. */
int orc_search_ld(const int64_t* list_off, const int64_t* ids, const uint8_t* codes,
                  const float* f_add, const float* f_rescale, const double* cos_oo,
                  const float* crot, int64_t C, int dp, int ld, int B,
                  const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
                  int kk, int est_mode, int64_t* out_ids, double* out_d)
{
    if (dp <= 0 || B < 1 || B > 8 || kk < 1) return -1;
    int bad = 0;
    #pragma omp parallel reduction(|:bad)
    {
        double* sd = (double*)malloc(sizeof(double) * dp);
        int8_t* qq = (int8_t*)malloc((size_t)dp);
        int8_t* ql = (int8_t*)malloc((size_t)dp);
        const double half = ((double)((1 << B) - 1)) / 2.0;
        int64_t cap = 1024;
        orc_cand* cand = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)cap);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            int64_t nc = 0;
            float delta; int32_t qsum, qsum_lo = 0;
            if (est_mode == 3) orc_query_quant2(qrot + iq * (int64_t)ld, dp, qq, ql, &delta, &qsum, &qsum_lo);
            else orc_query_quant(qrot + iq * (int64_t)ld, dp, qq, &delta, &qsum);
            for (int p = 0; p < nprobe; ++p) {
                int32_t l = probes[iq * nprobe + p];
                if (l < 0) continue;                 /* padding: the query probes fewer lists */
                if (l >= C) { bad = 1; continue; }
                const float* qv = qrot + iq * (int64_t)ld;
                const float* cv = crot + (int64_t)l * ld;
                double ns2 = 0.0;
                for (int i = 0; i < dp; ++i) { sd[i] = (double)qv[i] - (double)cv[i]; ns2 += sd[i] * sd[i]; }
                for (int i = dp; i < ld; ++i) { const double t = (double)qv[i] - (double)cv[i]; ns2 += t * t; }
                int64_t lo = list_off[l], hi = list_off[l + 1];
                if (nc + (hi - lo) > cap) {
                    while (nc + (hi - lo) > cap) cap *= 2;
                    cand = (orc_cand*)realloc(cand, sizeof(orc_cand) * (size_t)cap);
                }
                for (int64_t v = lo; v < hi; ++v) {
                    const uint8_t* cd = codes + v * (int64_t)dp;
                    double est;
                    if (est_mode == 2) {
                        /* float query, factor form (reading C-11): f_add + ||s||^2 + f_rescale <y, s'> */
                        double ys = 0.0;
                        for (int i = 0; i < dp; ++i) ys += ((double)cd[i] - half) * sd[i];
                        est = (double)f_add[v] + ns2 + (double)f_rescale[v] * ys;
                    } else if (est_mode == 0) {
                        int64_t ip = 0;
                        double ybc = 0.0;
                        for (int i = 0; i < dp; ++i) {
                            ip += (int64_t)cd[i] * (int64_t)qq[i];
                            ybc += ((double)cd[i] - half) * (double)cv[i];
                        }
                        est = orc_est_int8(ip, qsum, B, (double)delta, ybc, ns2,
                                           (double)f_add[v], (double)f_rescale[v]);
                    } else if (est_mode == 3) {
                        int64_t ih = 0, il = 0;
                        double ybc = 0.0;
                        for (int i = 0; i < dp; ++i) {
                            ih += (int64_t)cd[i] * (int64_t)qq[i];
                            il += (int64_t)cd[i] * (int64_t)ql[i];
                            ybc += ((double)cd[i] - half) * (double)cv[i];
                        }
                        est = orc_est_int8x2(ih, il, qsum, qsum_lo, B, (double)delta, ybc, ns2,
                                             (double)f_add[v], (double)f_rescale[v]);
                    } else {
                        est = orc_est_paper(cd, dp, B, sd, (double)f_add[v], cos_oo[v]);
                    }
                    cand[nc].d = est; cand[nc].id = ids[v]; ++nc;
                }
            }
            orc_take_k(cand, nc, kk, out_ids + iq * kk, out_d + iq * kk);
        }
        free(sd); free(qq); free(ql); free(cand);
    }
    return bad ? -1 : 0;
}

/* Exact re-rank: squared Euclidean distance (FP64) between q and each raw
   candidate row; the k smallest (dist, id).  cand ids < 0 are skipped. */
void orc_rerank(const float* x, int dp, const float* q, int64_t nq,
                const int64_t* cand, int kc, int k, int64_t* out_ids, double* out_d)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(kc > 0 ? kc : 1));
        #pragma omp for schedule(dynamic, 4)
        for (int64_t iq = 0; iq < nq; ++iq) {
            int64_t n = 0;
            for (int j = 0; j < kc; ++j) {
                int64_t id = cand[iq * kc + j];
                if (id < 0) continue;
                const float* xv = x + id * (int64_t)dp;
                const float* qv = q + iq * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) { double d = (double)xv[i] - (double)qv[i]; s += d * d; }
                c[n].d = s; c[n].id = id; ++n;
            }
            orc_take_k(c, n, k, out_ids + iq * k, out_d + iq * k);
        }
        free(c);
    }
}

/* Exact k nearest neighbours by FP64 brute force (ground truth for recall). */
void orc_knn(const float* x, int64_t n, int dp, const float* q, int64_t nq, int k,
             int64_t* out_ids, double* out_d)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(n > 0 ? n : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            const float* qv = q + iq * (int64_t)dp;
            for (int64_t r = 0; r < n; ++r) {
                const float* xv = x + r * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) { double d = (double)xv[i] - (double)qv[i]; s += d * d; }
                c[r].d = s; c[r].id = r;
            }
            orc_take_k(c, n, k, out_ids + iq * k, out_d + iq * k);
        }
        free(c);
    }
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Inner-product metric (the paper's conclusion: the method adapts to inner  */
/* product and cosine).  With c the list centroid and r = o_r - c:          */
/*   <o_r, q_r> = <c, q_r> + <r, q_r>,   <r, q_r> = ||r|| <o, q'>,           */
/* and <o, q'> is estimated as <o_bar, q'>/<o_bar, o> (Lemma 2.1, unbiased  */
/* for any q' by linearity), which with the stored factors is               */
/*   <r, q_r> ~ ||r||^2 <y, q'> / <y, r'> = -(f_rescale / 2) <y, q'>.       */
/* Results are ordered by the NEGATED inner product (smallest first), so   */
/* the top-k are the largest inner products.  <c, q_r> = <c', q'> (the     */
/* rotation preserves inner products), in FP64 from the rotated inputs.    */
/* est_mode 0: int8 query (decided in FP32 like the L2 scan); 2: float     */
/* query with the stored factors; 1: float query, paper form with          */
/* <o_bar, o> (cos_oo) and ||r|| = sqrt(f_add).                            */
/* ------------------------------------------------------------------------ */
int orc_search_ip(const int64_t* list_off, const int64_t* ids, const uint8_t* codes,
                  const float* f_add, const float* f_rescale, const double* cos_oo,
                  const float* crot, int64_t C, int dp, int B,
                  const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
                  int kk, int est_mode, int64_t* out_ids, double* out_d)
{
    if (dp <= 0 || B < 1 || B > 8 || kk < 1) return -1;
    int bad = 0;
    #pragma omp parallel reduction(|:bad)
    {
        int8_t* qq = (int8_t*)malloc((size_t)dp);
        const double half = ((double)((1 << B) - 1)) / 2.0;
        int64_t cap = 1024;
        orc_cand* cand = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)cap);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            int64_t nc = 0;
            float delta; int32_t qsum;
            const float* qv = qrot + iq * (int64_t)dp;
            orc_query_quant(qv, dp, qq, &delta, &qsum);
            double qs = 0.0, qn = 0.0;
            for (int i = 0; i < dp; ++i) { qs += (double)qv[i]; qn += (double)qv[i] * qv[i]; }
            for (int p = 0; p < nprobe; ++p) {
                int32_t l = probes[iq * nprobe + p];
                if (l < 0) continue;
                if (l >= C) { bad = 1; continue; }
                const float* cv = crot + (int64_t)l * dp;
                double cq = 0.0;
                for (int i = 0; i < dp; ++i) cq += (double)cv[i] * (double)qv[i];
                int64_t lo = list_off[l], hi = list_off[l + 1];
                if (nc + (hi - lo) > cap) {
                    while (nc + (hi - lo) > cap) cap *= 2;
                    cand = (orc_cand*)realloc(cand, sizeof(orc_cand) * (size_t)cap);
                }
                for (int64_t v = lo; v < hi; ++v) {
                    const uint8_t* cd = codes + v * (int64_t)dp;
                    double rq;                                  /* estimate of <r, q_r> */
                    if (est_mode == 0) {
                        int64_t ip = 0;
                        for (int i = 0; i < dp; ++i) ip += (int64_t)cd[i] * (int64_t)qq[i];
                        const double yq = 0.5 * (double)delta * (double)(2 * ip - (int64_t)((1 << B) - 1) * qsum);
                        rq = -0.5 * (double)f_rescale[v] * yq;
                    } else if (est_mode == 2) {
                        double yq = 0.0;
                        for (int i = 0; i < dp; ++i) yq += ((double)cd[i] - half) * (double)qv[i];
                        rq = -0.5 * (double)f_rescale[v] * yq;
                    } else {
                        /* ||r|| <o_bar, q'> / <o_bar, o>, <o_bar, q'> = (<y_u, q'> - half sum q') / ||y|| */
                        double yu = 0.0, ny = 0.0;
                        for (int i = 0; i < dp; ++i) {
                            yu += (double)cd[i] * (double)qv[i];
                            const double y = (double)cd[i] - half;
                            ny += y * y;
                        }
                        rq = (f_add[v] > 0.0f) ? sqrt((double)f_add[v]) * ((yu - half * qs) / sqrt(ny)) / cos_oo[v] : 0.0;
                    }
                    cand[nc].d = -(cq + rq); cand[nc].id = ids[v]; ++nc;
                }
            }
            (void)qn;
            orc_take_k(cand, nc, kk, out_ids + iq * kk, out_d + iq * kk);
        }
        free(qq); free(cand);
    }
    return bad ? -1 : 0;
}

/* The nprobe centroids of largest inner product with q (FP64), ties by id;
   pdist receives the negated inner products. */
void orc_probe_ip(const float* q, int64_t nq, const float* cent, int64_t C, int dp,
                  int nprobe, int32_t* probes, double* pdist)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)C);
        int64_t* tid = (int64_t*)malloc(sizeof(int64_t) * (size_t)nprobe);
        double* td = (double*)malloc(sizeof(double) * (size_t)nprobe);
        #pragma omp for schedule(dynamic, 4)
        for (int64_t iq = 0; iq < nq; ++iq) {
            const float* qv = q + iq * (int64_t)dp;
            for (int64_t j = 0; j < C; ++j) {
                const float* cv = cent + j * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) s += (double)qv[i] * (double)cv[i];
                c[j].d = -s; c[j].id = j;
            }
            orc_take_k(c, C, nprobe, tid, td);
            for (int j = 0; j < nprobe; ++j) {
                probes[iq * nprobe + j] = (int32_t)tid[j];
                if (pdist) pdist[iq * nprobe + j] = td[j];
            }
        }
        free(c); free(tid); free(td);
    }
}

/* Exact re-rank / k-NN by largest inner product (values: negated inner
   products, ascending; cand ids < 0 skipped). */
void orc_rerank_ip(const float* x, int dp, const float* q, int64_t nq,
                   const int64_t* cand, int kc, int k, int64_t* out_ids, double* out_d)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(kc > 0 ? kc : 1));
        #pragma omp for schedule(dynamic, 4)
        for (int64_t iq = 0; iq < nq; ++iq) {
            int64_t n = 0;
            for (int j = 0; j < kc; ++j) {
                int64_t id = cand[iq * kc + j];
                if (id < 0) continue;
                const float* xv = x + id * (int64_t)dp;
                const float* qv = q + iq * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) s += (double)xv[i] * (double)qv[i];
                c[n].d = -s; c[n].id = id; ++n;
            }
            orc_take_k(c, n, k, out_ids + iq * k, out_d + iq * k);
        }
        free(c);
    }
}

void orc_knn_ip(const float* x, int64_t n, int dp, const float* q, int64_t nq, int k,
                int64_t* out_ids, double* out_d)
{
    #pragma omp parallel
    {
        orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(n > 0 ? n : 1));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            const float* qv = q + iq * (int64_t)dp;
            for (int64_t r = 0; r < n; ++r) {
                const float* xv = x + r * (int64_t)dp;
                double s = 0.0;
                for (int i = 0; i < dp; ++i) s += (double)xv[i] * (double)qv[i];
                c[r].d = -s; c[r].id = r;
            }
            orc_take_k(c, n, k, out_ids + iq * k, out_d + iq * k);
        }
        free(c);
    }
}

/* ------------------------------------------------------------------------ */
/* MSB-first two-stage scan (Sec. 4.2).                                      */
/* ------------------------------------------------------------------------ */
/* The most significant bit of every coordinate of y_u is RaBitQ's 1-bit code
   x_b of the same residual (both are its orthant), so
     y_u = 2^(B-1) x_b + y_last                       (Eq. 4.2, decomposition)
   with y_last the B-1 low bits.  The 1-bit estimate is RaBitQ's (the B = 1
   case of the method) with the factors of the same residual: for the
   centred code x = x_b - 1/2, <x, r'> = ||r'||_1 / 2 =: l1 / 2, hence
     f1 = -2 ||r||^2 / <x, r'> = -4 f_add / l1,
     est1 = f_add + ||s||^2 + f1 <x, s'>,
   and with the int8 query of orc_search, 2<x, q'> ~= delta (2<x_b, q_int> -
   sum q_int).  Lemma 2.1 bounds the error of the unit-vector inner product
   behind est1 by sqrt(1 - c^2)/c * eps0/sqrt(D - 1), where
   c = <o_bar0, o> = <x, r'>/(||x|| ||r||) = l1/(sqrt(D) ||r||); scaled to
   the squared distance (est = ||r||^2 + ||s||^2 - 2 ||r|| ||s|| <o, q>):
     lb = est1 - 2 ||r|| ||s|| sqrt(1 - c^2)/c * eps0/sqrt(D - 1).
   Members with r = 0 (f_add = 0) or l1 = 0 have an exact est1 = ||s||^2. */
static void orc_msb_lb(const uint8_t* cd, int dp, int B, const int8_t* qq, double delta, int32_t qsum,
                       const float* cv, double ns2, double f_add, double l1, double eps0,
                       int64_t* ip_msb, double* est1, double* lb)
{
    int64_t ipm = 0;
    double xc = 0.0;
    for (int i = 0; i < dp; ++i) {
        const int xb = cd[i] >> (B - 1);
        ipm += (int64_t)xb * (int64_t)qq[i];
        xc += ((double)xb - 0.5) * (double)cv[i];
    }
    *ip_msb = ipm;
    if (!(f_add > 0.0) || !(l1 > 0.0)) { *est1 = ns2; *lb = ns2; return; }
    const double f1 = -4.0 * f_add / l1;
    const double xs = 0.5 * delta * (double)(2 * ipm - (int64_t)qsum) - xc;     /* <x, s'> */
    *est1 = f_add + ns2 + f1 * xs;
    const double nr = sqrt(f_add), c = l1 / (sqrt((double)dp) * nr);
    const double cc = c < 1.0 ? c : 1.0;
    *lb = *est1 - 2.0 * nr * sqrt(ns2) * sqrt(1.0 - cc * cc) / cc * eps0 / sqrt((double)dp - 1.0);
}

/* The paper's procedure for one query at a time, in a fixed order (probe
   rank, then list order): a candidate whose lower bound lb exceeds the
   kk-th best full estimate found so far is dropped; otherwise its full
   estimate is completed from the reused <x_b, q_int>:
     <y_u, q_int> = 2^(B-1) <x_b, q_int> + <y_last, q_int>   (Eq. 4.2, simplify)
   and evaluated exactly as in orc_search (est_mode 0).  l1[N]: ||r'||_1 per
   member (list order).  n_full[nq] (or NULL): full estimates computed. */
int orc_search_two_stage(const int64_t* list_off, const int64_t* ids, const uint8_t* codes,
                         const float* f_add, const float* f_rescale, const double* l1,
                         const float* crot, int64_t C, int dp, int B,
                         const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
                         int kk, double eps0, int64_t* out_ids, double* out_d, int64_t* n_full)
{
    if (dp <= 1 || B < 2 || B > 8 || kk < 1) return -1;
    int bad = 0;
    #pragma omp parallel reduction(|:bad)
    {
        double* sd = (double*)malloc(sizeof(double) * dp);
        int8_t* qq = (int8_t*)malloc((size_t)dp);
        orc_cand* top = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)(kk + 1));
        const double half = ((double)((1 << B) - 1)) / 2.0;
        const int lowmask = (1 << (B - 1)) - 1;
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            float delta; int32_t qsum;
            const float* qv = qrot + iq * (int64_t)dp;
            orc_query_quant(qv, dp, qq, &delta, &qsum);
            int nt = 0;                               /* top[0..nt) ascending by (est, id) */
            int64_t nf = 0;
            for (int p = 0; p < nprobe; ++p) {
                const int32_t l = probes[iq * nprobe + p];
                if (l < 0) continue;
                if (l >= C) { bad = 1; continue; }
                const float* cv = crot + (int64_t)l * dp;
                double ns2 = 0.0;
                for (int i = 0; i < dp; ++i) { sd[i] = (double)qv[i] - (double)cv[i]; ns2 += sd[i] * sd[i]; }
                for (int64_t v = list_off[l]; v < list_off[l + 1]; ++v) {
                    const uint8_t* cd = codes + v * (int64_t)dp;
                    int64_t ipm; double est1, lb;
                    orc_msb_lb(cd, dp, B, qq, (double)delta, qsum, cv, ns2, (double)f_add[v], l1[v], eps0,
                               &ipm, &est1, &lb);
                    if (nt == kk && lb > top[kk - 1].d) continue;        /* pruned by the 1-bit bound */
                    int64_t ipl = 0;
                    double ybc = 0.0;
                    for (int i = 0; i < dp; ++i) {
                        ipl += (int64_t)(cd[i] & lowmask) * (int64_t)qq[i];
                        ybc += ((double)cd[i] - half) * (double)cv[i];
                    }
                    const int64_t ipu = ipm * (int64_t)(1 << (B - 1)) + ipl;
                    orc_cand c;
                    c.d = orc_est_int8(ipu, qsum, B, (double)delta, ybc, ns2, (double)f_add[v],
                                       (double)f_rescale[v]);
                    c.id = ids[v];
                    ++nf;
                    /* insert into the sorted top list */
                    int pos = nt;
                    while (pos > 0 && orc_cand_cmp(&c, &top[pos - 1]) < 0) { top[pos] = top[pos - 1]; --pos; }
                    top[pos] = c;
                    if (nt < kk) ++nt;
                }
            }
            for (int j = 0; j < kk; ++j) {
                if (j < nt) { out_ids[iq * kk + j] = top[j].id; out_d[iq * kk + j] = top[j].d; }
                else { out_ids[iq * kk + j] = -1; out_d[iq * kk + j] = INFINITY; }
            }
            if (n_full) n_full[iq] = nf;
        }
        free(sd); free(qq); free(top);
    }
    return bad ? -1 : 0;
}

/* est1 and lb (above) of given candidates: cand[nq x m] member ids (< 0
   skipped, giving +inf), each looked up in the query's probed lists. */
int orc_msb_bounds(const int64_t* list_off, const int64_t* ids, int64_t N, const uint8_t* codes,
                   const float* f_add, const double* l1, const float* crot, int64_t C, int dp, int B,
                   const float* qrot, int64_t nq, const int32_t* probes, int nprobe,
                   const int64_t* cand, int m, double eps0, double* out_est1, double* out_lb)
{
    if (dp <= 1 || B < 2 || B > 8) return -1;
    int64_t maxid = -1;
    for (int64_t v = 0; v < N; ++v) if (ids[v] > maxid) maxid = ids[v];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxid + 2));
    for (int64_t i = 0; i <= maxid; ++i) pos[i] = -1;
    for (int64_t v = 0; v < N; ++v) pos[ids[v]] = v;
    int bad = 0;
    #pragma omp parallel reduction(|:bad)
    {
        int8_t* qq = (int8_t*)malloc((size_t)dp);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t iq = 0; iq < nq; ++iq) {
            float delta; int32_t qsum;
            const float* qv = qrot + iq * (int64_t)dp;
            orc_query_quant(qv, dp, qq, &delta, &qsum);
            for (int j = 0; j < m; ++j) {
                out_est1[iq * m + j] = INFINITY; out_lb[iq * m + j] = INFINITY;
                const int64_t id = cand[iq * m + j];
                if (id < 0 || id > maxid || pos[id] < 0) continue;
                const int64_t v = pos[id];
                int l = -1;
                for (int p = 0; p < nprobe; ++p) {
                    const int32_t t = probes[iq * nprobe + p];
                    if (t >= 0 && t < C && list_off[t] <= v && v < list_off[t + 1]) { l = t; break; }
                }
                if (l < 0) { bad = 1; continue; }
                const float* cv = crot + (int64_t)l * dp;
                double ns2 = 0.0;
                for (int i = 0; i < dp; ++i) { const double d = (double)qv[i] - (double)cv[i]; ns2 += d * d; }
                int64_t ipm;
                orc_msb_lb(codes + v * (int64_t)dp, dp, B, qq, (double)delta, qsum, cv, ns2, (double)f_add[v],
                           l1[v], eps0, &ipm, &out_est1[iq * m + j], &out_lb[iq * m + j]);
            }
        }
        free(qq);
    }
    free(pos);
    return bad ? -1 : 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
