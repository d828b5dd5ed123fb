// C ABI of liberq.so: argument validation, the index object, and the order
// in which the kernels of each call are enqueued.
#include <algorithm>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <numeric>

#include <unordered_set>

#include "erq_common.h"

namespace erq {

// launchers defined in the other translation units
hipError_t launch_split_bf16(const float* x, int64_t n, unsigned short* hi, unsigned short* lo, hipStream_t st);
hipError_t launch_split_norm(const float* X, int64_t n, int K, unsigned short* hi, unsigned short* lo, float* n2,
                             hipStream_t st);
hipError_t launch_split_bf16_t(const float* x, int K, int N, unsigned short* hi, unsigned short* lo, hipStream_t st);
hipError_t launch_gemm_bf16x3(const unsigned short* Ah, const unsigned short* Al, int64_t n,
                              const unsigned short* Bh, const unsigned short* Bl, int64_t N, int K,
                              float* out, int64_t ldo, hipStream_t st);
hipError_t launch_sqdist_pre(const unsigned short* Ah, const unsigned short* Al, int64_t n,
                             const unsigned short* Bh, const unsigned short* Bl, int64_t N, int K,
                             const float* an2, const float* bn2, float* out, hipStream_t st, int neg_ip);
hipError_t launch_pack_n(const uint8_t* codes, const int64_t* list_off, const int64_t* tile_off,
                         int64_t nlist, int dp, int bits, int64_t ntiles, uint8_t* packed, hipStream_t st);
hipError_t launch_unpack_n(const uint8_t* packed, const int64_t* list_off, const int64_t* tile_off,
                           int64_t nlist, int dp, int bits, int64_t ntiles, uint8_t* codes, hipStream_t st);
hipError_t launch_count(const int32_t* assign, int64_t n, int64_t nlist, int32_t* cnt, int32_t* bad, hipStream_t st);

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) { g_err = msg; return code; }

// ---- kernel timing registry ---------------------------------------------------
namespace {
struct ProfRec { int kernel; hipEvent_t a, b; };
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
bool g_prof_on = false;
bool g_prof_stats = false;     // also count pass-C pairs (synchronises after each scan)
const char* const kProfNames[PK_COUNT] = {"scan", "quantize", "rotate", "probe", "rerank",
                                          "scan_a", "scan_b", "scan_c"};
int64_t g_redo_total = 0, g_redo_calls = 0;
int64_t g_groups_total = 0, g_groups_skipped = 0;   // two-stage scan: groups, groups without full codes
}  // namespace

int prof_begin(int kernel, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return -1;
    ProfRec r{kernel, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    hipEventRecord(r.a, st);
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}

bool prof_stats_on()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on && g_prof_stats;
}

void prof_note_redo(const int32_t* dev_count, hipStream_t st)
{
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on || !g_prof_stats) return;
    }
    int32_t h[3] = {0, 0, 0};
    if (hipMemcpyAsync(h, dev_count, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return;
    if (hipStreamSynchronize(st) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_redo_total += h[0];
    g_redo_calls += 1;
    g_groups_total += h[1];
    g_groups_skipped += h[2];
}

void prof_end(int rec, hipStream_t st)
{
    if (rec < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (rec < (int)g_prof.size()) hipEventRecord(g_prof[rec].b, st);
}

void free_index_storage(Index* ix)
{
    hipFree(ix->cent); hipFree(ix->cent_rot); hipFree(ix->list_off); hipFree(ix->tile_off);
    hipFree(ix->cent_hi); hipFree(ix->cent_lo); hipFree(ix->cent_n2);
    ix->cent_hi = ix->cent_lo = nullptr; ix->cent_n2 = nullptr;
    hipFree(ix->list_order); hipFree(ix->ids); hipFree(ix->fac); hipFree(ix->sfac); hipFree(ix->codes);
    hipFree(ix->msb); hipFree(ix->fac1);
    ix->cent = ix->cent_rot = nullptr; ix->list_off = ix->tile_off = nullptr; ix->list_order = nullptr;
    ix->ids = nullptr; ix->fac = nullptr; ix->sfac = nullptr; ix->codes = nullptr;
    ix->msb = nullptr; ix->fac1 = nullptr;
    ix->n = 0; ix->ntiles = 0; ix->h_list_off.clear(); ix->max_list = 0;
}

namespace {

__global__ void interleave_fac_kernel(const float* a, const float* b, int64_t n, float2* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_float2(a[i], b[i]);
}
__global__ void split_fac_kernel(const float2* f, int64_t n, float* a, float* b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { if (a) a[i] = f[i].x; if (b) b[i] = f[i].y; }
}
__global__ void check_ids_kernel(const int64_t* ids, int64_t n, int32_t* bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (ids[i] < 0 || ids[i] >= n)) atomicOr(bad, 1);
}
__global__ void fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void iota_i32(int32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}
__global__ void widen_i32(const int32_t* a, int64_t n, int64_t* b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
__global__ void gather_topk_kernel(const int32_t* idx, int64_t n, int k, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = idx[i * k];
}
// first kout columns of (ids, est); with k_q, columns past the query's own k are (-1, +inf)
__global__ void copy_cols_kernel(const int64_t* ids, const float* est, int64_t nq, int kin, int kout,
                                 const int32_t* k_q, int64_t* oi, float* oe) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq * kout) return;
    int64_t q = i / kout; int t = (int)(i % kout);
    const bool in = !k_q || t < k_q[q];
    oi[i] = in ? ids[q * kin + t] : -1;
    oe[i] = in ? est[q * kin + t] : __builtin_huge_valf();
}

// ||r'||_1 of each row of a rotated batch (one wave per row, FP64 sum)
__global__ void row_l1_kernel(const float* rot, int64_t m, int d, float* out) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m) return;
    double s = 0.0;
    for (int i = lane; i < d; i += 64) s += fabs((double)rot[r * d + i]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[r] = (float)s;
}

// the most significant bit of each B-bit code value (RaBitQ's 1-bit code)
__global__ void msb_kernel(const uint8_t* in, int64_t count, int shift, uint8_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (uint8_t)(in[i] >> shift);
}

// projection fix-up: f_add = ||r||^2 over all dp coordinates, f_rescale
// scaled by dp / dc (App. C)
__global__ void proj_fac_kernel(const float* nrm, int64_t n, float scale, float2* fac) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    fac[i] = make_float2(nrm[i], fac[i].y * scale);
}

// Per-query search parameters clamped to the batch maxima: nprobe in
// [1, nprobe], k in [1, kmax], re-rank depth 0 or in [k, rrmax] (rrmax 0: no
// re-rank); null arrays give the maxima.  Probe ranks past a query's own
// nprobe become -1, which every later step skips.
__global__ void query_params_kernel(int64_t nq, int nprobe, int kmax, int rrmax, const int32_t* np_in,
                                    const int32_t* k_in, const int32_t* rr_in, int32_t* k_out, int32_t* rr_out,
                                    int32_t* probes) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const int np = np_in ? min(max(np_in[i], 1), nprobe) : nprobe;
    const int k = k_in ? min(max(k_in[i], 1), kmax) : kmax;
    int rr = rr_in ? rr_in[i] : rrmax;
    rr = (rr <= 0 || rrmax == 0) ? 0 : min(max(rr, k), rrmax);
    k_out[i] = k;
    rr_out[i] = rr;
    for (int p = np; p < nprobe; ++p) probes[i * nprobe + p] = -1;
}

inline unsigned blocks(int64_t n, int th = 256) { return (unsigned)((n + th - 1) / th); }
constexpr int kMaxSmallQ = 1024;               // largest threshold of the small-batch scan path
constexpr int kBuildKmeansIters = 10;          // Lloyd rounds of erq_index_build without centroids
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_dp(int dp, const char* who) {
    if (dp < 64 || dp > kMaxDp || dp % 64 != 0)
        return fail(ERQ_ESHAPE, std::string(who) + ": dp must be a multiple of 64 in [64, 4096]");
    return ERQ_OK;
}

// host-side list metadata: tile offsets and the longest-first order
int set_list_meta(Index* ix, const std::vector<int64_t>& off, hipStream_t st) {
    const int64_t C = ix->nlist;
    std::vector<int64_t> toff(C + 1, 0);
    int64_t mx = 0;
    for (int64_t l = 0; l < C; ++l) {
        int64_t sz = off[l + 1] - off[l];
        if (sz < 0) return fail(ERQ_EINVAL, "list offsets must be non-decreasing");
        mx = std::max(mx, sz);
        toff[l + 1] = toff[l] + (sz + kTileV - 1) / kTileV;
    }
    std::vector<int32_t> order(C);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return (off[a + 1] - off[a]) > (off[b + 1] - off[b]);
    });
    ix->h_list_off = off;
    ix->max_list = mx;
    ix->ntiles = toff[C];
    ERQ_HIP(hipMalloc(&ix->list_off, sizeof(int64_t) * (C + 1)));
    ERQ_HIP(hipMalloc(&ix->tile_off, sizeof(int64_t) * (C + 1)));
    ERQ_HIP(hipMalloc(&ix->list_order, sizeof(int32_t) * std::max<int64_t>(C, 1)));
    ERQ_HIP(hipMemcpyAsync(ix->list_off, off.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, st));
    ERQ_HIP(hipMemcpyAsync(ix->tile_off, toff.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, st));
    ERQ_HIP(hipMemcpyAsync(ix->list_order, order.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, st));
    ERQ_HIP(hipStreamSynchronize(st));       // host vectors go out of scope
    return ERQ_OK;
}

// BF16 hi/lo planes and squared norms of the index's raw centroids (the
// probe's fixed operand), from ix->cent
hipError_t alloc_cent_planes(Index* ix, hipStream_t st)
{
    const int64_t C = ix->nlist, dp = ix->dp;
    hipError_t e = hipMalloc(&ix->cent_hi, sizeof(unsigned short) * C * dp);
    if (e == hipSuccess) e = hipMalloc(&ix->cent_lo, sizeof(unsigned short) * C * dp);
    if (e == hipSuccess) e = hipMalloc(&ix->cent_n2, sizeof(float) * C);
    if (e == hipSuccess) e = launch_split_norm(ix->cent, C, (int)dp, ix->cent_hi, ix->cent_lo, ix->cent_n2, st);
    return e;
}

// Pd = the first dc columns of P (dp x dc, row-major) when dc < dp: the
// build's rotation then yields only the coordinates the codes keep
int set_projection_matrix(Index* ix, hipStream_t st)
{
    hipFree(ix->Pd);
    ix->Pd = nullptr;
    if (ix->dc == ix->dp) return ERQ_OK;
    ERQ_HIP(hipMalloc(&ix->Pd, sizeof(float) * ix->dp * ix->dc));
    ERQ_HIP(hipMemcpy2DAsync(ix->Pd, sizeof(float) * ix->dc, ix->P, sizeof(float) * ix->dp, sizeof(float) * ix->dc,
                             ix->dp, hipMemcpyDeviceToDevice, st));
    return ERQ_OK;
}

struct ProbePre {           // operands already split (and their norms), or null
    const unsigned short *qh = nullptr, *ql = nullptr; const float* qn = nullptr;
    const unsigned short *ch = nullptr, *cl = nullptr; const float* cn = nullptr;
};
int probe_impl(const float* q, int64_t nq, const float* cent, int64_t nlist, int dp, int nprobe,
               int32_t* probes, float* pdist, void* ws, size_t ws_bytes, hipStream_t st,
               const ProbePre& pre = ProbePre(), int metric = ERQ_METRIC_L2);

// distances nq x nlist, norms, and the BF16 hi/lo planes of both operands
size_t probe_ws(int64_t nq, int64_t nlist, int dp) {
    return align256(sizeof(float) * nq * nlist) + align256(sizeof(float) * nq) + align256(sizeof(float) * nlist) +
           2 * align256(sizeof(unsigned short) * nq * dp) + 2 * align256(sizeof(unsigned short) * nlist * dp);
}

// pre: the BF16 planes and norms of the queries and / or centroids when the
// caller has them (else computed here).  metric L2: ascending squared
// distances; inner product / cosine: ascending negated inner products.
int probe_impl(const float* q, int64_t nq, const float* cent, int64_t nlist, int dp, int nprobe,
               int32_t* probes, float* pdist, void* ws, size_t ws_bytes, hipStream_t st, const ProbePre& pre,
               int metric)
{
    if (ws_bytes < probe_ws(nq, nlist, dp)) return fail(ERQ_ENOMEM, "coarse probe: workspace too small");
    char* w = (char*)ws;
    float* D = (float*)w; w += align256(sizeof(float) * nq * nlist);
    float* qn = (float*)w; w += align256(sizeof(float) * nq);
    float* cn = (float*)w; w += align256(sizeof(float) * nlist);
    unsigned short* qh = (unsigned short*)w; w += align256(sizeof(unsigned short) * nq * dp);
    unsigned short* ql = (unsigned short*)w; w += align256(sizeof(unsigned short) * nq * dp);
    unsigned short* ch = (unsigned short*)w; w += align256(sizeof(unsigned short) * nlist * dp);
    unsigned short* cl = (unsigned short*)w;
    int pr = prof_begin(PK_PROBE, st);
    const unsigned short *uqh = qh, *uql = ql, *uch = ch, *ucl = cl;
    const float *uqn = qn, *ucn = cn;
    if (pre.qh && pre.ql && pre.qn) { uqh = pre.qh; uql = pre.ql; uqn = pre.qn; }
    else ERQ_HIP(launch_split_norm(q, nq, dp, qh, ql, qn, st));
    if (pre.ch && pre.cl && pre.cn) { uch = pre.ch; ucl = pre.cl; ucn = pre.cn; }
    else ERQ_HIP(launch_split_norm(cent, nlist, dp, ch, cl, cn, st));
    ERQ_HIP(launch_sqdist_pre(uqh, uql, nq, uch, ucl, nlist, dp, uqn, ucn, D, st, metric != ERQ_METRIC_L2));
    ERQ_HIP(launch_row_topk(D, nq, nlist, nprobe, probes, pdist, st));
    prof_end(pr, st);
    return ERQ_OK;
}

// ---- k-means (Sec. 4.1 builds the IVF lists with KMeans) -------------------------
// nearest centroid of every row (the probe with nprobe = 1: ties to the lower
// centroid id), in row chunks that keep the n x C distances small
int assign_rows(const float* x, int64_t n, int dp, const float* cent, int64_t C, int32_t* asg, hipStream_t st)
{
    if (n <= 0) return ERQ_OK;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(1LL << 28) / C));
    void* pws = nullptr;
    const size_t pb = probe_ws(chunk, C, dp);
    ERQ_HIP(hipMalloc(&pws, pb));
    struct Free { void* p; ~Free() { hipFree(p); } } fr{pws};
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t m = std::min(chunk, n - r0);
        if (int rc = probe_impl(x + r0 * dp, m, cent, C, dp, 1, asg + r0, nullptr, pws, pb, st)) return rc;
    }
    return ERQ_OK;
}

// per-list counts of an assignment -> host list offsets (ERQ_EINVAL for ids outside [0, C))
int list_offsets(const int32_t* asg, int64_t n, int64_t C, std::vector<int64_t>& off, hipStream_t st)
{
    int32_t* aux = nullptr;
    ERQ_HIP(hipMalloc(&aux, sizeof(int32_t) * (C + 1)));
    struct Free { void* p; ~Free() { hipFree(p); } } fr{aux};
    hipLaunchKernelGGL(fill_i32, dim3(blocks(C + 1)), dim3(256), 0, st, aux, C + 1, 0);
    ERQ_HIP(launch_count(asg, n, C, aux, aux + C, st));
    std::vector<int32_t> hc(C + 1);
    ERQ_HIP(hipMemcpyAsync(hc.data(), aux, sizeof(int32_t) * (C + 1), hipMemcpyDeviceToHost, st));
    ERQ_HIP(hipStreamSynchronize(st));
    if (hc[C] != 0) return fail(ERQ_EINVAL, "assignment outside [0, nlist)");
    off.assign(C + 1, 0);
    for (int64_t l = 0; l < C; ++l) off[l + 1] = off[l] + hc[l];
    return ERQ_OK;
}

// Lloyd's algorithm.  Readings: the initial centroids are C distinct rows
// chosen by Floyd's sampling with Philox random numbers of the seed (taken in
// ascending row order); `iters` rounds of assignment then per-list means; an
// empty list keeps its centroid; the returned assignment is to the final
// centroids.  Every sum has a fixed order, so a seed gives the same lists on
// every run.
int kmeans_impl(const float* x, int64_t n, int dp, int64_t C, int iters, uint64_t seed, float* cent, int32_t* asg_out,
                hipStream_t st)
{
    if (n < C) return fail(ERQ_EINVAL, "k-means: fewer rows than lists");
    std::unordered_set<int64_t> pick;
    pick.reserve((size_t)C * 2);
    for (int64_t j = n - C; j < n; ++j) {                 // Floyd: C distinct values of [0, n)
        const int64_t t = (int64_t)(philox_u64(seed, 0x4B4D4541u, (uint64_t)j) % (uint64_t)(j + 1));
        pick.insert(pick.count(t) ? j : t);
    }
    std::vector<int64_t> rows(pick.begin(), pick.end());
    std::sort(rows.begin(), rows.end());
    struct Bufs { std::vector<void*> p; ~Bufs() { for (void* q : p) hipFree(q); } } bufs;
    auto dalloc = [&](size_t b, void** out) -> int {
        ERQ_HIP(hipMalloc(out, std::max<size_t>(b, 256)));
        bufs.p.push_back(*out);
        return ERQ_OK;
    };
    int64_t* drows = nullptr; int32_t* asg = asg_out; int32_t* ids32 = nullptr; int64_t* doff = nullptr;
    void* bscr = nullptr;
    if (int rc = dalloc(sizeof(int64_t) * C, (void**)&drows)) return rc;
    if (!asg) {
        if (int rc = dalloc(sizeof(int32_t) * n, (void**)&asg)) return rc;
    }
    if (int rc = dalloc(sizeof(int32_t) * n, (void**)&ids32)) return rc;
    if (int rc = dalloc(sizeof(int64_t) * (C + 1), (void**)&doff)) return rc;
    if (int rc = dalloc(bucket_scratch_bytes(n, C), &bscr)) return rc;
    ERQ_HIP(hipMemcpyAsync(drows, rows.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, st));
    ERQ_HIP(launch_gather_rows(x, dp, drows, C, cent, st));
    ERQ_HIP(hipStreamSynchronize(st));                   // rows goes out of scope
    std::vector<int64_t> off;
    for (int it = 0; it < iters; ++it) {
        if (int rc = assign_rows(x, n, dp, cent, C, asg, st)) return rc;
        if (int rc = list_offsets(asg, n, C, off, st)) return rc;
        ERQ_HIP(hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, st));
        ERQ_HIP(launch_bucket_sort(asg, n, C, doff, ids32, bscr, st));
        void* mscr = nullptr;
        ERQ_HIP(hipMalloc(&mscr, list_mean_scratch_bytes(off, dp)));
        const hipError_t e = launch_list_mean(x, dp, ids32, off, doff, cent, mscr, st);   // synchronises
        hipFree(mscr);
        ERQ_HIP(e);
    }
    if (int rc = assign_rows(x, n, dp, cent, C, asg, st)) return rc;
    ERQ_HIP(hipStreamSynchronize(st));
    return ERQ_OK;
}

// ---- index files --------------------------------------------------------------
constexpr char kMagic[8] = {'E', 'R', 'Q', 'I', 'D', 'X', '\0', '\0'};
constexpr uint32_t kFileVersion = 2;
struct FileHeader {
    char magic[8];
    uint32_t version;
    int32_t dp, bits, has_raw, metric, dc;           // dc: code dimension (App. C projection when < dp)
    int64_t nlist, n, ntiles;
    int32_t tune[4];
    uint64_t seed;
    int32_t two_stage;                               // 1: the two-stage scan's data follow the codes
    float eps0;
    int32_t qplanes;                                 // int8 query planes of the scan (1 or 2)
    int32_t small_q;                                 // largest batch of the small-batch scan path
};

// bytes of every array of an index file after the header, in file order
std::vector<size_t> file_arrays(const FileHeader& h) {
    const size_t dp = (size_t)h.dp, C = (size_t)h.nlist, n = (size_t)h.n;
    return {sizeof(float) * dp * dp,              // P
            sizeof(float) * C * dp,               // raw centroids
            sizeof(float) * C * dp,               // rotated centroids
            sizeof(int64_t) * (C + 1),            // list offsets
            sizeof(int64_t) * n,                  // ids
            sizeof(float2) * n,                   // (f_add, f_rescale)
            sizeof(float2) * n,                   // scan factors
            (size_t)4 * (size_t)h.dc * h.bits * (size_t)h.ntiles,   // packed codes
            h.has_raw ? sizeof(float) * n * dp : 0,       // raw vectors
            h.two_stage ? (size_t)4 * (size_t)h.dc * (size_t)h.ntiles : 0,   // most significant bit planes
            h.two_stage ? sizeof(float4) * n : 0};        // 1-bit factors
}

// device <-> file through a host staging buffer, in chunks
int dev_to_file(FILE* f, const void* d, size_t bytes, std::vector<char>& buf, hipStream_t st) {
    for (size_t o = 0; o < bytes; o += buf.size()) {
        const size_t m = std::min(buf.size(), bytes - o);
        ERQ_HIP(hipMemcpyAsync(buf.data(), (const char*)d + o, m, hipMemcpyDeviceToHost, st));
        ERQ_HIP(hipStreamSynchronize(st));
        if (fwrite(buf.data(), 1, m, f) != m) return fail(ERQ_EINVAL, "erq_index_save: write failed");
    }
    return ERQ_OK;
}
int file_to_dev(FILE* f, void* d, size_t bytes, std::vector<char>& buf, hipStream_t st) {
    for (size_t o = 0; o < bytes; o += buf.size()) {
        const size_t m = std::min(buf.size(), bytes - o);
        if (fread(buf.data(), 1, m, f) != m) return fail(ERQ_EINVAL, "erq_index_load: file is truncated");
        ERQ_HIP(hipMemcpyAsync((char*)d + o, buf.data(), m, hipMemcpyHostToDevice, st));
        ERQ_HIP(hipStreamSynchronize(st));
    }
    return ERQ_OK;
}

}  // namespace
}  // namespace erq

using namespace erq;

struct erq_index_s : public Index {};

extern "C" {

const char* erq_last_error(void) { return g_err.c_str(); }
int erq_version(void) { return 200; }

int erq_rotate(const float* x, int64_t n, int32_t dp, const float* P, int32_t precision, float* out, void* stream)
{
    if (int rc = check_dp(dp, "erq_rotate")) return rc;
    if (n < 0 || (n > 0 && (!x || !P || !out))) return fail(ERQ_EINVAL, "erq_rotate: null pointer or n < 0");
    if (precision < 0 || precision > 2) return fail(ERQ_EUNSUPPORTED, "erq_rotate: precision must be 0, 1 or 2");
    if (x == out) return fail(ERQ_EINVAL, "erq_rotate: out must not alias x");
    hipStream_t st = (hipStream_t)stream;
    if (precision == 2) {
        // the search's rotation: BF16 hi/lo planes of x and of P^T, three products per K chunk
        if (n == 0) return ERQ_OK;
        struct Tmp { void* p[4] = {nullptr, nullptr, nullptr, nullptr}; ~Tmp() { for (void* q : p) hipFree(q); } } t;
        ERQ_HIP(hipMalloc(&t.p[0], sizeof(unsigned short) * n * dp));
        ERQ_HIP(hipMalloc(&t.p[1], sizeof(unsigned short) * n * dp));
        ERQ_HIP(hipMalloc(&t.p[2], sizeof(unsigned short) * dp * dp));
        ERQ_HIP(hipMalloc(&t.p[3], sizeof(unsigned short) * dp * dp));
        auto* xh = (unsigned short*)t.p[0]; auto* xl = (unsigned short*)t.p[1];
        auto* ph = (unsigned short*)t.p[2]; auto* pl = (unsigned short*)t.p[3];
        int pr = prof_begin(PK_ROTATE, st);
        ERQ_HIP(launch_split_bf16(x, n * dp, xh, xl, st));
        ERQ_HIP(launch_split_bf16_t(P, dp, dp, ph, pl, st));
        ERQ_HIP(launch_gemm_bf16x3(xh, xl, n, ph, pl, dp, dp, out, dp, st));
        prof_end(pr, st);
        ERQ_HIP(hipStreamSynchronize(st));          // before the scratch planes are freed
        return ERQ_OK;
    }
    int pr = prof_begin(PK_ROTATE, st);
    ERQ_HIP(launch_gemm(x, n, dp, P, dp, 0, precision, out, dp, st));
    prof_end(pr, st);
    return ERQ_OK;
}

int erq_quantize(const float* rrot, int64_t n, int32_t dp, int32_t bits, const float* norm2,
                 uint8_t* codes, float* f_add, float* f_rescale, float* cos_oo, void* stream)
{
    if (int rc = check_dp(dp, "erq_quantize")) return rc;
    if (dp > 3072) return fail(ERQ_EUNSUPPORTED, "erq_quantize: dp > 3072 exceeds the LDS window");
    if (bits < 1 || bits > 8) return fail(ERQ_EUNSUPPORTED, "erq_quantize: bits must be in [1, 8]");
    if (n < 0 || (n > 0 && (!rrot || !codes))) return fail(ERQ_EINVAL, "erq_quantize: null pointer or n < 0");
    int pr = prof_begin(PK_QUANTIZE, (hipStream_t)stream);
    ERQ_HIP(launch_quantize(rrot, n, dp, bits, norm2, codes, f_add, f_rescale, cos_oo, nullptr, (hipStream_t)stream));
    prof_end(pr, (hipStream_t)stream);
    return ERQ_OK;
}

int erq_probe_workspace_size(int64_t nq, int64_t nlist, int32_t dp, int32_t nprobe, size_t* bytes)
{
    if (!bytes || nq < 0 || nlist < 1 || nprobe < 1 || dp < 64 || dp % 64 != 0)
        return fail(ERQ_EINVAL, "erq_probe_workspace_size: bad arguments");
    *bytes = probe_ws(nq, nlist, dp);
    return ERQ_OK;
}

int erq_coarse_probe(const float* q, int64_t nq, const float* centroids, int64_t nlist, int32_t dp,
                     int32_t nprobe, int32_t metric, int32_t* probes, float* pdist, void* workspace, size_t ws_bytes,
                     void* stream)
{
    if (metric < ERQ_METRIC_L2 || metric > ERQ_METRIC_COSINE) return fail(ERQ_EINVAL, "erq_coarse_probe: bad metric");
    if (int rc = check_dp(dp, "erq_coarse_probe")) return rc;
    if (nq < 0 || nlist < 1 || nlist > (1LL << 31) - 1) return fail(ERQ_EINVAL, "erq_coarse_probe: bad sizes");
    if (nprobe < 1 || nprobe > 1024 || nprobe > nlist) return fail(ERQ_EUNSUPPORTED, "erq_coarse_probe: nprobe must be in [1, min(nlist, 1024)]");
    if (nq > 0 && (!q || !centroids || !probes || !workspace)) return fail(ERQ_EINVAL, "erq_coarse_probe: null pointer");
    return probe_impl(q, nq, centroids, nlist, dp, nprobe, probes, pdist, workspace, ws_bytes, (hipStream_t)stream,
                      ProbePre(), metric);
}

int erq_sample_rotation(int32_t dp, uint64_t seed, float* P_host)
{
    if (int rc = check_dp(dp, "erq_sample_rotation")) return rc;
    if (!P_host) return fail(ERQ_EINVAL, "erq_sample_rotation: null pointer");
    sample_rotation(dp, seed, P_host);
    return ERQ_OK;
}

int erq_index_create(int32_t dp, int32_t bits, int64_t nlist, const float* P, uint64_t seed, int32_t metric,
                     void* stream, erq_index* out)
{
    if (int rc = check_dp(dp, "erq_index_create")) return rc;
    if (metric < ERQ_METRIC_L2 || metric > ERQ_METRIC_COSINE) return fail(ERQ_EINVAL, "erq_index_create: bad metric");
    if (bits < 1 || bits > 8) return fail(ERQ_EUNSUPPORTED, "erq_index_create: bits must be in [1, 8]");
    if (nlist < 1 || nlist > (1 << 24)) return fail(ERQ_EINVAL, "erq_index_create: nlist must be in [1, 2^24]");
    if (!out) return fail(ERQ_EINVAL, "erq_index_create: null pointer");
    std::vector<float> hP;
    if (!P) {                                       // sample P (Haar) on the host
        hP.resize((size_t)dp * dp);
        sample_rotation(dp, seed, hP.data());
    }
    erq_index_s* ix = new (std::nothrow) erq_index_s();
    if (!ix) return fail(ERQ_ENOMEM, "erq_index_create: out of host memory");
    ix->dp = dp; ix->bits = bits; ix->nlist = nlist; ix->metric = metric; ix->dc = dp;
    ix->seed = P ? 0 : seed;
    hipGetDevice(&ix->device);
    if (hipMalloc(&ix->P, sizeof(float) * dp * dp) != hipSuccess) { delete ix; return fail(ERQ_ENOMEM, "erq_index_create: hipMalloc failed"); }
    hipError_t e = P ? hipMemcpyAsync(ix->P, P, sizeof(float) * dp * dp, hipMemcpyDeviceToDevice, (hipStream_t)stream)
                     : hipMemcpyAsync(ix->P, hP.data(), sizeof(float) * dp * dp, hipMemcpyHostToDevice,
                                      (hipStream_t)stream);
    if (e == hipSuccess) e = hipMalloc(&ix->pt_hi, sizeof(unsigned short) * dp * dp);
    if (e == hipSuccess) e = hipMalloc(&ix->pt_lo, sizeof(unsigned short) * dp * dp);
    if (e == hipSuccess) e = launch_split_bf16_t(ix->P, dp, dp, ix->pt_hi, ix->pt_lo, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        hipFree(ix->P); hipFree(ix->pt_hi); hipFree(ix->pt_lo); delete ix;
        return fail(ERQ_EDEVICE, std::string("erq_index_create: ") + hipGetErrorString(e));
    }
    *out = ix;
    return ERQ_OK;
}

int erq_index_save(erq_index ix, const char* path, void* stream)
{
    if (!ix || !path) return fail(ERQ_EINVAL, "erq_index_save: null pointer");
    if (!ix->list_off) return fail(ERQ_EINVAL, "erq_index_save: the index is empty");
    hipStream_t st = (hipStream_t)stream;
    FileHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = kFileVersion;
    h.dp = ix->dp; h.bits = ix->bits; h.has_raw = ix->raw ? 1 : 0; h.metric = ix->metric; h.dc = ix->dc;
    h.nlist = ix->nlist; h.n = ix->n; h.ntiles = ix->ntiles;
    h.tune[0] = ix->tune_nqt; h.tune[1] = ix->tune_pd; h.tune[2] = ix->tune_round1; h.tune[3] = ix->tune_round2;
    h.seed = ix->seed;
    h.two_stage = ix->msb ? 1 : 0;
    h.eps0 = ix->eps0;
    h.qplanes = ix->qplanes;
    h.small_q = ix->small_q;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(ERQ_EINVAL, std::string("erq_index_save: cannot open ") + path);
    struct Closer { FILE* f; ~Closer() { if (f) std::fclose(f); } } closer{f};
    if (fwrite(&h, sizeof(h), 1, f) != 1) return fail(ERQ_EINVAL, "erq_index_save: write failed");
    std::vector<char> buf((size_t)64 << 20);
    const void* src[11] = {ix->P, ix->cent, ix->cent_rot, ix->list_off, ix->ids, ix->fac, ix->sfac, ix->codes,
                           ix->raw, ix->msb, ix->fac1};
    const std::vector<size_t> sz = file_arrays(h);
    for (int a = 0; a < 11; ++a)
        if (sz[a]) { if (int rc = dev_to_file(f, src[a], sz[a], buf, st)) return rc; }
    if (std::fclose(f) != 0) { closer.f = nullptr; return fail(ERQ_EINVAL, "erq_index_save: close failed"); }
    closer.f = nullptr;
    return ERQ_OK;
}

int erq_index_load(const char* path, void* stream, erq_index* out)
{
    if (!path || !out) return fail(ERQ_EINVAL, "erq_index_load: null pointer");
    hipStream_t st = (hipStream_t)stream;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ERQ_EINVAL, std::string("erq_index_load: cannot open ") + path);
    struct Closer { FILE* f; ~Closer() { std::fclose(f); } } closer{f};
    FileHeader h{};
    if (fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kMagic, 8) != 0)
        return fail(ERQ_EINVAL, "erq_index_load: not an index file");
    if (h.version != kFileVersion) return fail(ERQ_EUNSUPPORTED, "erq_index_load: unknown file version");
    if (h.dp < 64 || h.dp > kMaxDp || h.dp % 64 || h.bits < 1 || h.bits > 8 || h.nlist < 1 ||
        h.nlist > (1 << 24) || h.n < 0 || h.n > (1LL << 31) - 1 || h.ntiles < 0 || (h.has_raw != 0 && h.has_raw != 1) ||
        h.metric < ERQ_METRIC_L2 || h.metric > ERQ_METRIC_COSINE || h.dc < 64 || h.dc > h.dp || h.dc % 64 ||
        (h.two_stage != 0 && h.two_stage != 1) || !(h.eps0 >= 0.0f) || !(h.eps0 < 1e30f) ||
        (h.qplanes != 1 && h.qplanes != 2) || (h.qplanes == 2 && (h.bits < 5 || h.two_stage)) ||
        h.small_q < 0 || h.small_q > kMaxSmallQ)
        return fail(ERQ_EINVAL, "erq_index_load: bad header");
    const std::vector<size_t> sz = file_arrays(h);
    size_t total = sizeof(h);
    for (size_t b : sz) total += b;
    if (std::fseek(f, 0, SEEK_END) != 0 || (size_t)std::ftell(f) != total)
        return fail(ERQ_EINVAL, "erq_index_load: file size does not match its header");
    std::fseek(f, (long)sizeof(h), SEEK_SET);
    // list offsets first (host): they fix the tiles and the list order
    const int64_t C = h.nlist, n = h.n;
    const int dp = h.dp;
    std::vector<int64_t> off(C + 1);
    {
        size_t skip = sz[0] + sz[1] + sz[2];
        std::fseek(f, (long)(sizeof(h) + skip), SEEK_SET);
        if (fread(off.data(), sizeof(int64_t), C + 1, f) != (size_t)(C + 1))
            return fail(ERQ_EINVAL, "erq_index_load: file is truncated");
        std::fseek(f, (long)sizeof(h), SEEK_SET);
    }
    if (off[0] != 0 || off[C] != n) return fail(ERQ_EINVAL, "erq_index_load: bad list offsets");
    erq_index_s* ix = new (std::nothrow) erq_index_s();
    if (!ix) return fail(ERQ_ENOMEM, "erq_index_load: out of host memory");
    struct Owner { erq_index_s* p; ~Owner() { if (p) erq_index_destroy(p); } } owner{ix};
    ix->dp = dp; ix->bits = h.bits; ix->nlist = C; ix->seed = h.seed; ix->metric = h.metric; ix->dc = h.dc;
    ix->two_stage = h.two_stage; ix->eps0 = h.eps0; ix->qplanes = h.qplanes; ix->small_q = h.small_q;
    ix->tune_nqt = h.tune[0]; ix->tune_pd = h.tune[1]; ix->tune_round1 = h.tune[2]; ix->tune_round2 = h.tune[3];
    hipGetDevice(&ix->device);
    if (int rc = set_list_meta(ix, off, st)) return rc;
    if (ix->ntiles != h.ntiles) return fail(ERQ_EINVAL, "erq_index_load: tile count does not match the lists");
    ix->n = n;
    ERQ_HIP(hipMalloc(&ix->P, sz[0]));
    ERQ_HIP(hipMalloc(&ix->cent, sz[1]));
    ERQ_HIP(hipMalloc(&ix->cent_rot, sz[2]));
    ERQ_HIP(hipMalloc(&ix->ids, std::max<size_t>(sz[4], 8)));
    ERQ_HIP(hipMalloc(&ix->fac, std::max<size_t>(sz[5], 8)));
    ERQ_HIP(hipMalloc(&ix->sfac, std::max<size_t>(sz[6], 8)));
    ERQ_HIP(hipMalloc(&ix->codes, std::max<size_t>(sz[7], 256)));
    if (h.has_raw) ERQ_HIP(hipMalloc(&ix->raw, std::max<size_t>(sz[8], 4)));
    if (h.two_stage) {
        ERQ_HIP(hipMalloc(&ix->msb, std::max<size_t>(sz[9], 256)));
        ERQ_HIP(hipMalloc(&ix->fac1, std::max<size_t>(sz[10], 16)));
    }
    void* dst[11] = {ix->P, ix->cent, ix->cent_rot, nullptr, ix->ids, ix->fac, ix->sfac, ix->codes, ix->raw,
                     ix->msb, ix->fac1};
    std::vector<char> buf((size_t)64 << 20);
    for (int a = 0; a < 11; ++a) {
        if (a == 3) { std::fseek(f, (long)sz[3], SEEK_CUR); continue; }   // list offsets: already uploaded
        if (sz[a]) { if (int rc = file_to_dev(f, dst[a], sz[a], buf, st)) return rc; }
    }
    ERQ_HIP(hipMalloc(&ix->pt_hi, sizeof(unsigned short) * dp * dp));
    ERQ_HIP(hipMalloc(&ix->pt_lo, sizeof(unsigned short) * dp * dp));
    ERQ_HIP(launch_split_bf16_t(ix->P, dp, dp, ix->pt_hi, ix->pt_lo, st));
    if (int rc = set_projection_matrix(ix, st)) return rc;
    ERQ_HIP(alloc_cent_planes(ix, st));
    ERQ_HIP(hipStreamSynchronize(st));
    owner.p = nullptr;
    *out = ix;
    return ERQ_OK;
}

int erq_index_set_projection(erq_index ix, int32_t dc, void* stream)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_set_projection: null index");
    if (ix->list_off) return fail(ERQ_EINVAL, "erq_index_set_projection: the index already holds vectors");
    if (ix->metric != ERQ_METRIC_L2) return fail(ERQ_EUNSUPPORTED, "erq_index_set_projection: L2 metric only");
    if (ix->two_stage && dc != ix->dp)
        return fail(ERQ_EUNSUPPORTED, "erq_index_set_projection: not with the two-stage scan");
    if (dc < 64 || dc > ix->dp || dc % 64 != 0)
        return fail(ERQ_ESHAPE, "erq_index_set_projection: dc must be a multiple of 64 in [64, dp]");
    ix->dc = dc;
    if (int rc = set_projection_matrix(ix, (hipStream_t)stream)) return rc;
    ERQ_HIP(hipStreamSynchronize((hipStream_t)stream));
    return ERQ_OK;
}

int erq_index_set_two_stage(erq_index ix, float eps0)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_set_two_stage: null index");
    if (!(eps0 >= 0.0f) || !(eps0 < 1e30f)) return fail(ERQ_EINVAL, "erq_index_set_two_stage: eps0 must be >= 0");
    if (eps0 > 0.0f && (ix->metric != ERQ_METRIC_L2 || ix->bits < 2 || ix->dc != ix->dp || ix->qplanes != 1))
        return fail(ERQ_EUNSUPPORTED,
                    "erq_index_set_two_stage: needs the L2 metric, bits >= 2, no projection, one query plane");
    if (!ix->list_off) {                             // empty: the build computes the 1-bit data
        ix->two_stage = eps0 > 0.0f ? 1 : 0;
        ix->eps0 = eps0;
        return ERQ_OK;
    }
    if (eps0 > 0.0f && !ix->msb)
        return fail(ERQ_EINVAL, "erq_index_set_two_stage: the index holds no 1-bit data (request it before the build)");
    ix->eps0 = eps0;
    return ERQ_OK;
}

int erq_index_set_query_planes(erq_index ix, int32_t planes)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_set_query_planes: null index");
    if (planes != 1 && planes != 2) return fail(ERQ_EINVAL, "erq_index_set_query_planes: planes must be 1 or 2");
    if (planes == 2 && (ix->bits < 5 || ix->two_stage))
        return fail(ERQ_EUNSUPPORTED, "erq_index_set_query_planes: two planes need bits >= 5 and no two-stage scan");
    ix->qplanes = planes;
    return ERQ_OK;
}

int erq_index_set_small_batch(erq_index ix, int32_t max_queries)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_set_small_batch: null index");
    if (max_queries < 0 || max_queries > kMaxSmallQ)
        return fail(ERQ_EINVAL, "erq_index_set_small_batch: max_queries must be in [0, 1024]");
    ix->small_q = max_queries;
    return ERQ_OK;
}

int erq_index_small_batch(erq_index ix, int32_t* max_queries)
{
    if (!ix || !max_queries) return fail(ERQ_EINVAL, "erq_index_small_batch: null pointer");
    *max_queries = ix->small_q;
    return ERQ_OK;
}

int erq_index_code_dim(erq_index ix, int32_t* dc)
{
    if (!ix || !dc) return fail(ERQ_EINVAL, "erq_index_code_dim: null pointer");
    *dc = ix->dc;
    return ERQ_OK;
}

int erq_index_get_rotation(erq_index ix, float* P_out, void* stream)
{
    if (!ix || !P_out) return fail(ERQ_EINVAL, "erq_index_get_rotation: null pointer");
    ERQ_HIP(hipMemcpyAsync(P_out, ix->P, sizeof(float) * ix->dp * ix->dp, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return ERQ_OK;
}

int erq_index_destroy(erq_index ix)
{
    if (!ix) return ERQ_OK;
    hipDeviceSynchronize();
    free_index_storage(ix);
    hipFree(ix->P);
    hipFree(ix->Pd);
    hipFree(ix->pt_hi);
    hipFree(ix->pt_lo);
    hipFree(ix->raw);
    delete ix;
    return ERQ_OK;
}

int erq_index_import(erq_index ix, int64_t n, const int64_t* list_off, const int64_t* ids,
                     const uint8_t* codes, const float* f_add, const float* f_rescale,
                     const float* centroids, const float* centroids_rot, void* stream)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_import: null index");
    if (n < 0 || n > (1LL << 31) - 1) return fail(ERQ_EINVAL, "erq_index_import: n out of range");
    if (!list_off || !centroids || (n > 0 && (!ids || !codes || !f_add || !f_rescale)))
        return fail(ERQ_EINVAL, "erq_index_import: null pointer");
    if (ix->two_stage) return fail(ERQ_EUNSUPPORTED, "erq_index_import: the two-stage data need erq_index_build");
    hipStream_t st = (hipStream_t)stream;
    const int64_t C = ix->nlist;
    const int dp = ix->dp;
    std::vector<int64_t> off(C + 1);
    ERQ_HIP(hipMemcpyAsync(off.data(), list_off, sizeof(int64_t) * (C + 1), hipMemcpyDeviceToHost, st));
    ERQ_HIP(hipStreamSynchronize(st));
    if (off[0] != 0 || off[C] != n) return fail(ERQ_EINVAL, "erq_index_import: list_off must start at 0 and end at n");
    free_index_storage(ix);
    if (int rc = set_list_meta(ix, off, st)) return rc;
    ix->n = n;
    ERQ_HIP(hipMalloc(&ix->ids, sizeof(int64_t) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->fac, sizeof(float2) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->sfac, sizeof(float2) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->codes, std::max<int64_t>((int64_t)4 * ix->dc * ix->bits * ix->ntiles, 256)));
    ERQ_HIP(hipMalloc(&ix->cent, sizeof(float) * C * dp));
    ERQ_HIP(hipMalloc(&ix->cent_rot, sizeof(float) * C * dp));
    ERQ_HIP(hipMemcpyAsync(ix->cent, centroids, sizeof(float) * C * dp, hipMemcpyDeviceToDevice, st));
    ERQ_HIP(alloc_cent_planes(ix, st));
    if (centroids_rot)
        ERQ_HIP(hipMemcpyAsync(ix->cent_rot, centroids_rot, sizeof(float) * C * dp, hipMemcpyDeviceToDevice, st));
    else
        ERQ_HIP(launch_gemm(ix->cent, C, dp, ix->P, dp, 0, 0, ix->cent_rot, dp, st));
    if (n > 0) {
        // ids are row numbers: in [0, n) (the scan keeps them as int32, the re-rank indexes raw rows by them)
        int32_t* bad = nullptr;
        ERQ_HIP(hipMalloc(&bad, sizeof(int32_t)));
        int32_t hbad = 0;
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, bad, 1, 0);
        hipLaunchKernelGGL(check_ids_kernel, dim3(blocks(n)), dim3(256), 0, st, ids, n, bad);
        hipError_t ce = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (ce == hipSuccess) ce = hipStreamSynchronize(st);
        hipFree(bad);
        ERQ_HIP(ce);
        if (hbad) {
            free_index_storage(ix);
            return fail(ERQ_EINVAL, "erq_index_import: ids must lie in [0, n)");
        }
        ERQ_HIP(hipMemcpyAsync(ix->ids, ids, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(interleave_fac_kernel, dim3(blocks(n)), dim3(256), 0, st, f_add, f_rescale, n, ix->fac);
        ERQ_HIP(hipGetLastError());
        ERQ_HIP(launch_pack_n(codes, ix->list_off, ix->tile_off, C, ix->dc, ix->bits, ix->ntiles, ix->codes, st));
        ERQ_HIP(launch_scan_fac(codes, ix->list_off, C, ix->cent_rot, ix->fac, n, ix->dc, dp, ix->bits, ix->metric,
                                ix->sfac, st));
    }
    ERQ_HIP(hipStreamSynchronize(st));
    return ERQ_OK;
}

int erq_index_set_raw(erq_index ix, const float* x, int64_t n, void* stream)
{
    if (!ix || !x) return fail(ERQ_EINVAL, "erq_index_set_raw: null pointer");
    if (n != ix->n) return fail(ERQ_ESHAPE, "erq_index_set_raw: n differs from the index size");
    hipFree(ix->raw);
    ix->raw = nullptr;
    ERQ_HIP(hipMalloc(&ix->raw, sizeof(float) * std::max<int64_t>(n, 1) * ix->dp));
    if (ix->metric == ERQ_METRIC_COSINE)
        ERQ_HIP(launch_normalize(x, n, ix->dp, ix->raw, (hipStream_t)stream));
    else
        ERQ_HIP(hipMemcpyAsync(ix->raw, x, sizeof(float) * n * ix->dp, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    ERQ_HIP(hipStreamSynchronize((hipStream_t)stream));
    return ERQ_OK;
}

int erq_kmeans(const float* x, int64_t n, int32_t dp, int64_t nlist, int32_t iters, uint64_t seed,
               float* centroids, int32_t* assign, void* stream)
{
    if (int rc = check_dp(dp, "erq_kmeans")) return rc;
    if (nlist < 1 || nlist > (1 << 24) || n < nlist || n > (1LL << 31) - 1)
        return fail(ERQ_EINVAL, "erq_kmeans: need 1 <= nlist <= n < 2^31");
    if (iters < 0 || iters > 1000) return fail(ERQ_EINVAL, "erq_kmeans: iters must be in [0, 1000]");
    if (!x || !centroids) return fail(ERQ_EINVAL, "erq_kmeans: null pointer");
    return kmeans_impl(x, n, dp, nlist, iters, seed, centroids, assign, (hipStream_t)stream);
}

int erq_index_build(erq_index ix, const float* x, int64_t n, const float* centroids, const int32_t* assign,
                    int32_t precision, int32_t keep_raw, void* stream)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_build: null index");
    if (n < 0 || n > (1LL << 31) - 1) return fail(ERQ_EINVAL, "erq_index_build: n out of range");
    if (n > 0 && !x) return fail(ERQ_EINVAL, "erq_index_build: null pointer");
    float* own_cent = nullptr;                      // centroids of the library's k-means
    float* xnorm = nullptr;                         // cosine: the rows scaled to unit length
    struct FreeC { float** p; float** q; ~FreeC() { hipFree(*p); hipFree(*q); } } free_cent{&own_cent, &xnorm};
    if (ix->metric == ERQ_METRIC_COSINE && n > 0) {
        ERQ_HIP(hipMalloc(&xnorm, sizeof(float) * n * ix->dp));
        ERQ_HIP(launch_normalize(x, n, ix->dp, xnorm, (hipStream_t)stream));
        x = xnorm;
    }
    if (!centroids) {
        if (assign) return fail(ERQ_EINVAL, "erq_index_build: an assignment needs its centroids");
        if (n < ix->nlist) return fail(ERQ_EINVAL, "erq_index_build: k-means needs at least nlist rows");
        ERQ_HIP(hipMalloc(&own_cent, sizeof(float) * ix->nlist * ix->dp));
        if (int rc = kmeans_impl(x, n, ix->dp, ix->nlist, kBuildKmeansIters, ix->seed ^ 0x6B6D65616E73ull, own_cent,
                                 nullptr, (hipStream_t)stream))
            return rc;
        centroids = own_cent;
    }
    if (precision != 0 && precision != 1) return fail(ERQ_EUNSUPPORTED, "erq_index_build: precision must be 0 or 1");
    if (ix->dp > 3072) return fail(ERQ_EUNSUPPORTED, "erq_index_build: dp > 3072 exceeds the LDS window");
    hipStream_t st = (hipStream_t)stream;
    const int64_t C = ix->nlist;
    const int dp = ix->dp, dc = ix->dc;
    free_index_storage(ix);
    hipFree(ix->raw);
    ix->raw = nullptr;
    ERQ_HIP(hipMalloc(&ix->cent, sizeof(float) * C * dp));
    ERQ_HIP(hipMalloc(&ix->cent_rot, sizeof(float) * C * dp));
    ERQ_HIP(hipMemcpyAsync(ix->cent, centroids, sizeof(float) * C * dp, hipMemcpyDeviceToDevice, st));
    ERQ_HIP(alloc_cent_planes(ix, st));
    ERQ_HIP(launch_gemm(ix->cent, C, dp, ix->P, dp, 0, 0, ix->cent_rot, dp, st));

    // assignment (nearest centroid when not given)
    int32_t* asg = nullptr;
    int32_t* aux = nullptr;     // cnt | (unused) | bad
    ERQ_HIP(hipMalloc(&asg, sizeof(int32_t) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&aux, sizeof(int32_t) * (2 * C + 1)));
    struct Guard { std::vector<void*> p; ~Guard() { for (void* q : p) hipFree(q); } } guard;
    guard.p.push_back(asg); guard.p.push_back(aux);
    if (assign) {
        ERQ_HIP(hipMemcpyAsync(asg, assign, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    } else if (n > 0) {
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(1LL << 28) / C));
        void* pws = nullptr;
        size_t pb = probe_ws(chunk, C, dp);
        ERQ_HIP(hipMalloc(&pws, pb));
        guard.p.push_back(pws);
        for (int64_t r0 = 0; r0 < n; r0 += chunk) {
            int64_t m = std::min(chunk, n - r0);
            if (int rc = probe_impl(x + r0 * dp, m, ix->cent, C, dp, 1, asg + r0, nullptr, pws, pb, st, ProbePre(),
                                    ix->metric))
                return rc;
        }
    }
    int32_t* cnt = aux;
    int32_t* bad = aux + 2 * C;
    hipLaunchKernelGGL(fill_i32, dim3(blocks(2 * C + 1)), dim3(256), 0, st, aux, 2 * C + 1, 0);
    ERQ_HIP(launch_count(asg, n, C, cnt, bad, st));
    std::vector<int32_t> hc(C);
    int32_t hbad = 0;
    ERQ_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * C, hipMemcpyDeviceToHost, st));
    ERQ_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ERQ_HIP(hipStreamSynchronize(st));
    if (hbad != 0) return fail(ERQ_EINVAL, "erq_index_build: assignment outside [0, nlist)");
    std::vector<int64_t> off(C + 1, 0);
    for (int64_t l = 0; l < C; ++l) off[l + 1] = off[l] + hc[l];
    if (int rc = set_list_meta(ix, off, st)) return rc;
    ix->n = n;
    int32_t* ids32 = nullptr;
    ERQ_HIP(hipMalloc(&ids32, sizeof(int32_t) * std::max<int64_t>(n, 1)));
    guard.p.push_back(ids32);
    ERQ_HIP(hipMalloc(&ix->ids, sizeof(int64_t) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->fac, sizeof(float2) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->sfac, sizeof(float2) * std::max<int64_t>(n, 1)));
    ERQ_HIP(hipMalloc(&ix->codes, std::max<int64_t>((int64_t)4 * dc * ix->bits * ix->ntiles, 256)));
    // members in list order, ids ascending within each list: a stable bucket
    // sort of the rows by list, so the layout is the same on every build
    if (n > 0) {
        void* bs = nullptr;
        ERQ_HIP(hipMalloc(&bs, bucket_scratch_bytes(n, C)));
        guard.p.push_back(bs);
        ERQ_HIP(launch_bucket_sort(asg, n, C, ix->list_off, ids32, bs, st));
        hipLaunchKernelGGL(widen_i32, dim3(blocks(n)), dim3(256), 0, st, ids32, n, ix->ids);
        ERQ_HIP(hipGetLastError());
    }

    // residual -> rotate -> quantise, in batches, list order
    uint8_t* codes_u = nullptr;
    ERQ_HIP(hipMalloc(&codes_u, std::max<int64_t>(n, 1) * dc));
    guard.p.push_back(codes_u);
    const int64_t bt = std::max<int64_t>(1, std::min<int64_t>(n, 131072));
    float *res = nullptr, *rot = nullptr, *nrm = nullptr;
    ERQ_HIP(hipMalloc(&res, sizeof(float) * bt * dp));
    ERQ_HIP(hipMalloc(&rot, sizeof(float) * bt * dc));
    ERQ_HIP(hipMalloc(&nrm, sizeof(float) * bt));
    guard.p.push_back(res); guard.p.push_back(rot); guard.p.push_back(nrm);
    float* l1 = nullptr;                            // ||r'||_1 per member (two-stage scan)
    if (ix->two_stage) {
        ERQ_HIP(hipMalloc(&l1, sizeof(float) * std::max<int64_t>(n, 1)));
        guard.p.push_back(l1);
    }
    for (int64_t v0 = 0; v0 < n; v0 += bt) {
        int64_t m = std::min(bt, n - v0);
        ERQ_HIP(launch_residual(x, ix->ids + v0, asg, ix->cent, m, dp, res, nrm, st));
        int pr = prof_begin(PK_ROTATE, st);
        ERQ_HIP(launch_gemm(res, m, dp, dc < dp ? ix->Pd : ix->P, dc, 0, precision, rot, dc, st));
        prof_end(pr, st);
        pr = prof_begin(PK_QUANTIZE, st);
        // projection (App. C): the codes and <y, r'_d> from the first dc
        // coordinates, ||r'_d||^2 from them too; the fix-up then takes
        // f_add = ||r||^2 and scales f_rescale by dp / dc
        ERQ_HIP(launch_quantize(rot, m, dc, ix->bits, dc < dp ? nullptr : nrm, codes_u + v0 * dc, nullptr, nullptr,
                                nullptr, ix->fac + v0, st));
        if (dc < dp) {
            hipLaunchKernelGGL(proj_fac_kernel, dim3(blocks(m)), dim3(256), 0, st, nrm, m, (float)dp / (float)dc,
                               ix->fac + v0);
            ERQ_HIP(hipGetLastError());
        }
        if (l1) {
            hipLaunchKernelGGL(row_l1_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, rot, m, dc, l1 + v0);
            ERQ_HIP(hipGetLastError());
        }
        prof_end(pr, st);
    }
    ERQ_HIP(launch_pack_n(codes_u, ix->list_off, ix->tile_off, C, dc, ix->bits, ix->ntiles, ix->codes, st));
    ERQ_HIP(launch_scan_fac(codes_u, ix->list_off, C, ix->cent_rot, ix->fac, n, dc, dp, ix->bits, ix->metric,
                            ix->sfac, st));
    if (ix->two_stage) {
        // the most significant bit planes in the 1-bit tile layout, and the 1-bit factors
        uint8_t* mu = nullptr;
        ERQ_HIP(hipMalloc(&mu, std::max<int64_t>(n, 1) * dc));
        guard.p.push_back(mu);
        ERQ_HIP(hipMalloc(&ix->msb, std::max<int64_t>((int64_t)4 * dc * ix->ntiles, 256)));
        ERQ_HIP(hipMalloc(&ix->fac1, sizeof(float4) * std::max<int64_t>(n, 1)));
        if (n > 0) {
            hipLaunchKernelGGL(msb_kernel, dim3(blocks(n * dc)), dim3(256), 0, st, codes_u, n * dc, ix->bits - 1, mu);
            ERQ_HIP(hipGetLastError());
        }
        ERQ_HIP(launch_pack_n(mu, ix->list_off, ix->tile_off, C, dc, 1, ix->ntiles, ix->msb, st));
        ERQ_HIP(launch_scan1_fac(codes_u, ix->list_off, C, ix->cent_rot, dp, ix->fac, l1, n, dc, ix->bits, ix->fac1,
                                 st));
    }
    if (keep_raw && n > 0) {
        ERQ_HIP(hipMalloc(&ix->raw, sizeof(float) * n * dp));
        ERQ_HIP(hipMemcpyAsync(ix->raw, x, sizeof(float) * n * dp, hipMemcpyDeviceToDevice, st));
    }
    ERQ_HIP(hipStreamSynchronize(st));
    return ERQ_OK;
}

int erq_index_info(erq_index ix, int64_t* n, int32_t* dp, int32_t* bits, int64_t* nlist, int64_t* code_bytes)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_info: null index");
    if (n) *n = ix->n;
    if (dp) *dp = ix->dp;
    if (bits) *bits = ix->bits;
    if (nlist) *nlist = ix->nlist;
    if (code_bytes) *code_bytes = (int64_t)4 * ix->dc * ix->bits * ix->ntiles;
    return ERQ_OK;
}

int erq_index_export(erq_index ix, int64_t* list_off, int64_t* ids, uint8_t* codes, float* f_add,
                     float* f_rescale, float* centroids_rot, void* stream)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_export: null index");
    if (!ix->list_off) return fail(ERQ_EINVAL, "erq_index_export: empty index");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = ix->n, C = ix->nlist;
    if (list_off) ERQ_HIP(hipMemcpyAsync(list_off, ix->list_off, sizeof(int64_t) * (C + 1), hipMemcpyDeviceToDevice, st));
    if (ids && n) ERQ_HIP(hipMemcpyAsync(ids, ix->ids, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, st));
    if (codes && n) ERQ_HIP(launch_unpack_n(ix->codes, ix->list_off, ix->tile_off, C, ix->dc, ix->bits, ix->ntiles, codes, st));
    if ((f_add || f_rescale) && n) {
        hipLaunchKernelGGL(split_fac_kernel, dim3(blocks(n)), dim3(256), 0, st, ix->fac, n, f_add, f_rescale);
        ERQ_HIP(hipGetLastError());
    }
    if (centroids_rot) ERQ_HIP(hipMemcpyAsync(centroids_rot, ix->cent_rot, sizeof(float) * C * ix->dp, hipMemcpyDeviceToDevice, st));
    return ERQ_OK;
}

int erq_scan_workspace_size(erq_index ix, int64_t nq, int32_t nprobe, int32_t kk, size_t* bytes)
{
    if (!ix || !bytes || nq < 0 || nprobe < 1 || kk < 1) return fail(ERQ_EINVAL, "erq_scan_workspace_size: bad arguments");
    *bytes = scan_workspace_bytes(nq, nprobe, ix->nlist, kk, ix->dc, ix->max_list);
    return ERQ_OK;
}

int erq_scan(erq_index ix, const float* qrot, int64_t nq, const int32_t* probes, int32_t nprobe, int32_t kk,
             int64_t* out_ids, float* out_est, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ix || !ix->codes) return fail(ERQ_EINVAL, "erq_scan: index is empty");
    if (nq < 0 || nq * (int64_t)std::max(nprobe, 1) > (1LL << 31) - 1) return fail(ERQ_EINVAL, "erq_scan: nq out of range");
    if (nprobe < 1 || nprobe > 1024) return fail(ERQ_EUNSUPPORTED, "erq_scan: nprobe must be in [1, 1024]");
    if (kk < 1 || kk > kMaxK) return fail(ERQ_EUNSUPPORTED, "erq_scan: kk must be in [1, 1024]");
    if (nq > 0 && (!qrot || !probes || !out_ids || !out_est || !workspace)) return fail(ERQ_EINVAL, "erq_scan: null pointer");
    if (ix->nlist > 1000000) return fail(ERQ_EUNSUPPORTED, "erq_scan: more than 10^6 lists");
    return run_scan(ix, qrot, ix->dp, nq, probes, nullptr, nprobe, kk, out_ids, out_est, workspace, ws_bytes,
                    (hipStream_t)stream);
}

int erq_rerank(erq_index ix, const float* q, int64_t nq, const int64_t* cand, int32_t kc, int32_t k,
               int64_t* out_ids, float* out_dist, void* stream)
{
    if (!ix || !ix->raw) return fail(ERQ_EINVAL, "erq_rerank: the index holds no raw vectors");
    if (kc < 1 || kc > kMaxK || k < 1 || k > kc) return fail(ERQ_EUNSUPPORTED, "erq_rerank: need 1 <= k <= kc <= 1024");
    if (nq < 0 || (nq > 0 && (!q || !cand || !out_ids || !out_dist))) return fail(ERQ_EINVAL, "erq_rerank: bad arguments");
    int pr = prof_begin(PK_RERANK, (hipStream_t)stream);
    const float* qq = q;
    float* qnorm = nullptr;
    if (ix->metric == ERQ_METRIC_COSINE && nq > 0) {      // the rows are stored normalised; so is the query
        ERQ_HIP(hipMalloc(&qnorm, sizeof(float) * nq * ix->dp));
        ERQ_HIP(launch_normalize(q, nq, ix->dp, qnorm, (hipStream_t)stream));
        qq = qnorm;
    }
    hipError_t re = launch_rerank(ix->raw, ix->n, ix->dp, qq, nq, cand, nullptr, kc, k, nullptr, nullptr, out_ids,
                                  out_dist, (hipStream_t)stream, ix->metric);
    if (qnorm) {
        if (re == hipSuccess) re = hipStreamSynchronize((hipStream_t)stream);
        hipFree(qnorm);
    }
    ERQ_HIP(re);
    prof_end(pr, (hipStream_t)stream);
    return ERQ_OK;
}

static size_t search_ws(Index* ix, int64_t nq, int nprobe, int k, int rerank_k) {
    const int kk = rerank_k > 0 ? rerank_k : k;
    size_t b = 0;
    b += align256(sizeof(float) * nq * ix->dc);           // qrot (the coordinates the codes use)
    b += align256(sizeof(int32_t) * nq * nprobe);         // probes
    b += align256(sizeof(float) * nq * nprobe);           // probe distances ||q - c||^2
    b += align256(sizeof(int64_t) * nq * kk);             // candidate ids
    b += align256(sizeof(float) * nq * kk);               // candidate estimates
    b += 2 * align256(sizeof(unsigned short) * nq * ix->dp);   // BF16 hi/lo planes of the queries
    b += align256(sizeof(float) * nq);                          // ||q||^2
    b += 2 * align256(sizeof(int32_t) * nq);                    // per-query k and re-rank depth
    if (ix->metric == ERQ_METRIC_COSINE) b += align256(sizeof(float) * nq * ix->dp);   // unit-length queries
    b += std::max(probe_ws(nq, ix->nlist, ix->dp), scan_workspace_bytes(nq, nprobe, ix->nlist, kk, ix->dc, ix->max_list));
    return b;
}

int erq_search_workspace_size(erq_index ix, int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k, size_t* bytes)
{
    if (!ix || !bytes || nq < 0 || nprobe < 1 || k < 1 || rerank_k < 0) return fail(ERQ_EINVAL, "erq_search_workspace_size: bad arguments");
    *bytes = search_ws(ix, nq, nprobe, k, rerank_k);
    return ERQ_OK;
}

// argument checks of erq_search (and of its no-allocation variant)
static int search_check(Index* ix, const float* q, int64_t nq, int nprobe, int k, int rerank_k, int64_t* out_ids,
                        float* out_dist, const char* who)
{
    const std::string w(who);
    if (!ix || !ix->codes) return fail(ERQ_EINVAL, w + ": index is empty");
    if (k < 1 || k > kMaxK) return fail(ERQ_EUNSUPPORTED, w + ": k must be in [1, 1024]");
    if (rerank_k < 0 || rerank_k > kMaxK || (rerank_k > 0 && rerank_k < k))
        return fail(ERQ_EUNSUPPORTED, w + ": rerank_k must be 0 or in [k, 1024]");
    if (rerank_k > 0 && !ix->raw) return fail(ERQ_EINVAL, w + ": re-rank needs raw vectors in the index");
    if (nprobe < 1 || nprobe > 1024 || nprobe > ix->nlist)
        return fail(ERQ_EUNSUPPORTED, w + ": nprobe must be in [1, min(nlist, 1024)]");
    if (nq < 0 || nq * (int64_t)nprobe > (1LL << 31) - 1) return fail(ERQ_EINVAL, w + ": nq out of range");
    if (nq > 0 && (!q || !out_ids || !out_dist)) return fail(ERQ_EINVAL, w + ": null pointer");
    return ERQ_OK;
}

// The query path on a checked call: rotate, probe, per-query parameters,
// scan, re-rank or copy, all on `st` inside the workspace ws.
static int search_run(Index* ix, const float* q, int64_t nq, int nprobe, int k, int rerank_k, const int32_t* nprobe_q,
                      const int32_t* k_q, const int32_t* rerank_q, int64_t* out_ids, float* out_dist, void* workspace,
                      size_t ws_bytes, hipStream_t st)
{
    const int kk = rerank_k > 0 ? rerank_k : k;
    char* w = (char*)workspace;
    float* qrot = (float*)w; w += align256(sizeof(float) * nq * ix->dc);
    int32_t* probes = (int32_t*)w; w += align256(sizeof(int32_t) * nq * nprobe);
    float* pdist = (float*)w; w += align256(sizeof(float) * nq * nprobe);
    int64_t* cid = (int64_t*)w; w += align256(sizeof(int64_t) * nq * kk);
    float* cest = (float*)w; w += align256(sizeof(float) * nq * kk);
    unsigned short* qh = (unsigned short*)w; w += align256(sizeof(unsigned short) * nq * ix->dp);
    unsigned short* ql = (unsigned short*)w; w += align256(sizeof(unsigned short) * nq * ix->dp);
    float* qn = (float*)w; w += align256(sizeof(float) * nq);
    int32_t* kq = (int32_t*)w; w += align256(sizeof(int32_t) * nq);
    int32_t* rq = (int32_t*)w; w += align256(sizeof(int32_t) * nq);
    if (ix->metric == ERQ_METRIC_COSINE) {          // unit-length queries for every later step
        float* qn_rows = (float*)w; w += align256(sizeof(float) * nq * ix->dp);
        ERQ_HIP(launch_normalize(q, nq, ix->dp, qn_rows, st));
        q = qn_rows;
    }
    size_t rest = ws_bytes - (size_t)(w - (char*)workspace);
    // q' = q P on the BF16 matrix cores from hi/lo planes (the probe's
    // products and error bound); the planes serve the probe too
    int pr = prof_begin(PK_ROTATE, st);
    ERQ_HIP(launch_split_norm(q, nq, ix->dp, qh, ql, qn, st));
    // (with the projection, the first dc coordinates of q' only)
    ERQ_HIP(launch_gemm_bf16x3(qh, ql, nq, ix->pt_hi, ix->pt_lo, ix->dc, ix->dp, qrot, ix->dc, st));
    prof_end(pr, st);
    // the probe's ||q - c||^2 = ||q' - c'||^2 (P orthogonal) is the scan's ||s||^2 (L2), its
    // -<q, c> = -<q', c'> the scan's per-pair term (inner-product metrics)
    ProbePre pre;
    pre.qh = qh; pre.ql = ql; pre.qn = qn;
    pre.ch = ix->cent_hi; pre.cl = ix->cent_lo; pre.cn = ix->cent_n2;
    if (int rc = probe_impl(q, nq, ix->cent, ix->nlist, ix->dp, nprobe, probes, pdist, w, rest, st, pre, ix->metric))
        return rc;
    const bool per_query = nprobe_q || k_q || rerank_q;
    if (per_query) {
        hipLaunchKernelGGL(query_params_kernel, dim3(blocks(nq)), dim3(256), 0, st, nq, nprobe, k, rerank_k, nprobe_q,
                           k_q, rerank_q, kq, rq, probes);
        ERQ_HIP(hipGetLastError());
    }
    if (int rc = run_scan(ix, qrot, ix->dc, nq, probes, pdist, nprobe, kk, cid, cest, w, rest, st)) return rc;
    if (rerank_k > 0) {
        int pr2 = prof_begin(PK_RERANK, st);
        ERQ_HIP(launch_rerank(ix->raw, ix->n, ix->dp, q, nq, cid, cest, kk, k, per_query ? rq : nullptr,
                              per_query ? kq : nullptr, out_ids, out_dist, st, ix->metric));
        prof_end(pr2, st);
    } else {
        hipLaunchKernelGGL(copy_cols_kernel, dim3(blocks(nq * k)), dim3(256), 0, st, cid, cest, nq, kk, k,
                           per_query ? kq : nullptr, out_ids, out_dist);
        ERQ_HIP(hipGetLastError());
    }
    return ERQ_OK;
}

// ---- erq_search_static: the search with the library's own device scratch ----
// A file-scope device array, one copy per GPU, used as the search workspace
// by callers that cannot allocate.  Host code never passes the array's name
// to a kernel: its device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call there)
int scratch_ptr(void** out)
{
    int d = 0;
    ERQ_HIP(hipGetDevice(&d));
    if (d < 0 || d >= kMaxDevices) return fail(ERQ_EUNSUPPORTED, "erq_search_static: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[d]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ERQ_EDEVICE, std::string("erq_search_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[d] = p;
    }
    *out = g_scratch_ptr[d];
    return ERQ_OK;
}
}  // namespace

int erq_search_static(erq_index ix, const float* q, int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k,
                      const int32_t* nprobe_q, const int32_t* k_q, const int32_t* rerank_q, int64_t* out_ids,
                      float* out_dist, void* stream)
{
    if (int rc = search_check(ix, q, nq, nprobe, k, rerank_k, out_ids, out_dist, "erq_search_static")) return rc;
    if (nq == 0) return ERQ_OK;
    const size_t need = search_ws(ix, nq, nprobe, k, rerank_k);
    if (need > kScratchBytes)
        return fail(ERQ_ENOMEM, "erq_search_static: the call needs " + std::to_string(need) +
                                    " bytes of workspace, more than the library's 64 MiB scratch");
    void* ws = nullptr;
    if (int rc = scratch_ptr(&ws)) return rc;
    return search_run(ix, q, nq, nprobe, k, rerank_k, nprobe_q, k_q, rerank_q, out_ids, out_dist, ws, kScratchBytes,
                      (hipStream_t)stream);
}

int erq_static_scratch_bytes(size_t* bytes)
{
    if (!bytes) return fail(ERQ_EINVAL, "erq_static_scratch_bytes: null pointer");
    *bytes = kScratchBytes;
    return ERQ_OK;
}

int erq_search(erq_index ix, const float* q, int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k,
               const int32_t* nprobe_q, const int32_t* k_q, const int32_t* rerank_q, int64_t* out_ids,
               float* out_dist, void* workspace, size_t ws_bytes, void* stream)
{
    if (int rc = search_check(ix, q, nq, nprobe, k, rerank_k, out_ids, out_dist, "erq_search")) return rc;
    if (nq == 0) return ERQ_OK;
    if (!workspace) return fail(ERQ_EINVAL, "erq_search: null workspace");
    if (ws_bytes < search_ws(ix, nq, nprobe, k, rerank_k)) return fail(ERQ_ENOMEM, "erq_search: workspace too small");
    return search_run(ix, q, nq, nprobe, k, rerank_k, nprobe_q, k_q, rerank_q, out_ids, out_dist, workspace, ws_bytes,
                      (hipStream_t)stream);
}

int erq_index_set_tune(erq_index ix, int32_t nqt, int32_t pd, int32_t round1, int32_t round2)
{
    if (!ix) return fail(ERQ_EINVAL, "erq_index_set_tune: null index");
    if (nqt < 0 || nqt > 2 || (nqt == 2 && ix->dc > kMaxDpNqt2))
        return fail(ERQ_EINVAL, "erq_index_set_tune: nqt must be 0, 1 or 2 (2 needs dp <= 1536)");
    if (pd < 0 || (pd > 0 && !scan_pd_valid(pd, ix->dc, ix->bits)))
        return fail(ERQ_EINVAL, "erq_index_set_tune: pd must be 0 or one of 1, 2, 3, 4, 6 dividing dp/64 (6 for bits <= 4)");
    if (round1 < 0 || round1 > 1024) return fail(ERQ_EINVAL, "erq_index_set_tune: round1 must be in [0, 1024]");
    if (round2 < 0 || round2 > 1024) return fail(ERQ_EINVAL, "erq_index_set_tune: round2 must be in [0, 1024]");
    ix->tune_nqt = nqt; ix->tune_pd = pd; ix->tune_round1 = round1; ix->tune_round2 = round2;
    return ERQ_OK;
}

int erq_index_get_tune(erq_index ix, int32_t* nqt, int32_t* pd, int32_t* round1, int32_t* round2)
{
    if (!ix || !nqt || !pd || !round1 || !round2) return fail(ERQ_EINVAL, "erq_index_get_tune: null pointer");
    *nqt = ix->tune_nqt; *pd = ix->tune_pd; *round1 = ix->tune_round1; *round2 = ix->tune_round2;
    return ERQ_OK;
}

// Coordinate search over the scan schedule: first (nqt, pd) with the stored
// round1 and round2, then round1, then round2 (none or a multiple of round1);
// each candidate is timed with
// HIP events over `reps` calls of erq_search after one untimed call.
int erq_index_tune(erq_index ix, const float* q, int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k,
                   int32_t reps, int64_t* out_ids, float* out_dist, void* workspace, size_t ws_bytes, void* stream,
                   int32_t* choice, double* best_ms)
{
    if (!ix || !choice) return fail(ERQ_EINVAL, "erq_index_tune: null pointer");
    if (reps < 1 || reps > 100) return fail(ERQ_EINVAL, "erq_index_tune: reps must be in [1, 100]");
    if (nq < 1) return fail(ERQ_EINVAL, "erq_index_tune: needs at least one query");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        if (ea) hipEventDestroy(ea);
        return fail(ERQ_EDEVICE, "erq_index_tune: hipEventCreate failed");
    }
    const int saved[4] = {ix->tune_nqt, ix->tune_pd, ix->tune_round1, ix->tune_round2};
    int rc = ERQ_OK;
    double best = -1.0;
    int bq = scan_nqt(ix), bp = scan_pd(ix), br = scan_round1(ix), b2 = scan_round2(ix);
    auto time_one = [&](int nqt, int pd, int r1, int r2, double* ms) -> int {
        ix->tune_nqt = nqt; ix->tune_pd = pd; ix->tune_round1 = r1; ix->tune_round2 = r2;
        if (int r = erq_search(ix, q, nq, nprobe, k, rerank_k, nullptr, nullptr, nullptr, out_ids, out_dist, workspace,
                               ws_bytes, stream))
            return r;
        if (hipEventRecord(ea, st) != hipSuccess) return fail(ERQ_EDEVICE, "erq_index_tune: event record failed");
        for (int i = 0; i < reps; ++i)
            if (int r = erq_search(ix, q, nq, nprobe, k, rerank_k, nullptr, nullptr, nullptr, out_ids, out_dist,
                                   workspace, ws_bytes, stream))
                return r;
        float t = 0.0f;
        if (hipEventRecord(eb, st) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
            hipEventElapsedTime(&t, ea, eb) != hipSuccess)
            return fail(ERQ_EDEVICE, "erq_index_tune: event timing failed");
        *ms = (double)t / reps;
        return ERQ_OK;
    };
    for (int nqt = 1; nqt <= 2 && rc == ERQ_OK; ++nqt) {
        if (nqt == 2 && ix->dc > kMaxDpNqt2) continue;
        for (int pd : {6, 4, 3, 2, 1}) {
            if (!scan_pd_valid(pd, ix->dc, ix->bits)) continue;
            double ms = 0.0;
            rc = time_one(nqt, pd, br, b2, &ms);
            if (rc != ERQ_OK) break;
            if (best < 0.0 || ms < best) { best = ms; bq = nqt; bp = pd; }
        }
    }
    for (int r1 : {2, 4, 8, 16, 32}) {
        if (rc != ERQ_OK) break;
        if (r1 >= nprobe || r1 == br) continue;
        double ms = 0.0;
        rc = time_one(bq, bp, r1, b2, &ms);
        if (rc == ERQ_OK && ms < best) { best = ms; br = r1; }
    }
    for (int f : {0, 2, 4, 8, 16}) {
        if (rc != ERQ_OK) break;
        const int r2 = f * br;
        if ((f > 0 && r2 >= nprobe) || r2 == b2) continue;
        double ms = 0.0;
        rc = time_one(bq, bp, br, r2, &ms);
        if (rc == ERQ_OK && ms < best) { best = ms; b2 = r2; }
    }
    hipEventDestroy(ea);
    hipEventDestroy(eb);
    if (rc != ERQ_OK) {
        ix->tune_nqt = saved[0]; ix->tune_pd = saved[1]; ix->tune_round1 = saved[2]; ix->tune_round2 = saved[3];
        return rc;
    }
    ix->tune_nqt = bq; ix->tune_pd = bp; ix->tune_round1 = br; ix->tune_round2 = b2;
    choice[0] = bq; choice[1] = bp; choice[2] = br; choice[3] = b2;
    if (best_ms) *best_ms = best;
    return ERQ_OK;
}

int erq_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    g_prof_stats = on >= 2;
    return ERQ_OK;
}

int erq_profile_read(const char* kernel, double* total_ms, int64_t* launches, int32_t reset)
{
    if (!kernel) return fail(ERQ_EINVAL, "erq_profile_read: null name");
    if (std::strcmp(kernel, "scan_redo_pairs") == 0) {        // pairs sent to pass C, summed over scans
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (total_ms) *total_ms = (double)g_redo_total;
        if (launches) *launches = g_redo_calls;
        if (reset) { g_redo_total = 0; g_redo_calls = 0; }
        return ERQ_OK;
    }
    if (std::strcmp(kernel, "scan2_groups") == 0) {           // two-stage scan: groups skipped / scanned
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (total_ms) *total_ms = (double)g_groups_skipped;
        if (launches) *launches = g_groups_total;
        if (reset) { g_groups_total = 0; g_groups_skipped = 0; }
        return ERQ_OK;
    }
    int kid = -1;
    for (int i = 0; i < PK_COUNT; ++i) if (std::strcmp(kernel, kProfNames[i]) == 0) kid = i;
    if (kid < 0) return fail(ERQ_EINVAL, std::string("erq_profile_read: unknown kernel ") + kernel);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& r : g_prof) {
        if (r.kernel != kid) continue;
        ERQ_HIP(hipEventSynchronize(r.b));
        float ms = 0.0f;
        ERQ_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
        ++cnt;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    if (reset) {
        for (auto& r : g_prof) {
            hipEventSynchronize(r.b);
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        g_prof.clear();
    }
    return ERQ_OK;
}

}  // extern "C"
