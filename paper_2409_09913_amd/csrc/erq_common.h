// Internal declarations shared by the HIP translation units of liberq.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/erq.h"

namespace erq {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kWave = 64;
constexpr int kTileV = 32;      // vectors per packed code tile (rows of one 32x32 MFMA tile)
constexpr int kMaxDp = 4096;
constexpr int kMaxDpNqt2 = 1536;  // largest dp whose two-tile query block fits the LDS
constexpr int kMaxK = 1024;       // largest top-k / re-rank depth of a scan

// ---- status plumbing -------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define ERQ_HIP(call)                                                              \
    do {                                                                           \
        hipError_t _e = (call);                                                    \
        if (_e != hipSuccess)                                                      \
            return ::erq::fail(ERQ_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

// ---- packed code layout -----------------------------------------------------
// Codes of one list are stored in tiles of 32 vectors.  A tile holds dp/64
// K-blocks of 64 dimensions; a K-block holds, for each power-of-two part of
// the code (see parts_of), 64 lanes x (4*w) bytes, where lane L covers
// vector (L % 32) and dimensions kb*64 + s*32 + (L/32)*16 + j, s in {0,1},
// j in [0,16).  Total bytes per tile: 4 * dp * B.
struct Parts {
    int n;            // number of parts
    int w[3];         // width in bits of each part
    int pos[3];       // bit position of each part inside y_u
};
__host__ __device__ inline Parts parts_of(int bits) {
    Parts p{};
    switch (bits) {
        case 1: p.n = 1; p.w[0] = 1; p.pos[0] = 0; break;
        case 2: p.n = 1; p.w[0] = 2; p.pos[0] = 0; break;
        case 3: p.n = 2; p.w[0] = 2; p.pos[0] = 0; p.w[1] = 1; p.pos[1] = 2; break;
        case 4: p.n = 1; p.w[0] = 4; p.pos[0] = 0; break;
        case 5: p.n = 2; p.w[0] = 4; p.pos[0] = 0; p.w[1] = 1; p.pos[1] = 4; break;
        case 6: p.n = 2; p.w[0] = 4; p.pos[0] = 0; p.w[1] = 2; p.pos[1] = 4; break;
        case 7: p.n = 3; p.w[0] = 4; p.pos[0] = 0; p.w[1] = 2; p.pos[1] = 4; p.w[2] = 1; p.pos[2] = 6; break;
        default: p.n = 1; p.w[0] = 8; p.pos[0] = 0; break;
    }
    return p;
}
// Stored byte value is y_u for B <= 7 and y_u - 128 (two's complement) for B = 8,
// so that it is a valid signed int8 for the matrix cores.
__host__ __device__ inline int stored_offset(int bits) { return bits == 8 ? 128 : 0; }

// ---- the index ---------------------------------------------------------------
struct Index {
    int dp = 0, bits = 0;
    int dc = 0;                    // code dimension: dp, or d < dp with the projection of App. C
    int metric = ERQ_METRIC_L2;    // erq_metric
    int64_t nlist = 0, n = 0;
    int device = 0;
    uint64_t seed = 0;             // seed P was sampled from (0 when the caller gave P)
    float* P = nullptr;            // dp x dp
    float* Pd = nullptr;           // dp x dc, the first dc columns of P (only when dc < dp)
    unsigned short* pt_hi = nullptr;   // BF16 hi/lo planes of P^T (dp x dp each): the search's rotation
    unsigned short* pt_lo = nullptr;
    float* cent = nullptr;         // nlist x dp raw centroids
    float* cent_rot = nullptr;     // nlist x dp rotated centroids
    unsigned short* cent_hi = nullptr;   // BF16 hi/lo planes of the raw centroids and their squared
    unsigned short* cent_lo = nullptr;   // norms: the probe's B operand, fixed per index
    float* cent_n2 = nullptr;
    int64_t* list_off = nullptr;   // nlist + 1 (device)
    int64_t* tile_off = nullptr;   // nlist + 1, offset of each list's first tile (device)
    int32_t* list_order = nullptr; // lists by decreasing size (device)
    int tune_nqt = 0, tune_pd = 0, tune_round1 = 0;   // scan schedule; 0 = built-in rule
    int tune_round2 = 0;                               // end of a middle round of probe ranks; 0 = none
    int64_t* ids = nullptr;        // n, list order
    float2* fac = nullptr;         // n, (f_add, f_rescale), list order
    float2* sfac = nullptr;        // n, (f_add - f_rescale <y_bar, c'>, f_rescale): the scan's factors
    uint8_t* codes = nullptr;      // ntiles * 4 * dc * bits bytes
    // two-stage scan (Sec. 4.2): requested before the build; its data are the
    // most significant bit planes (ntiles * 4 * dc bytes, the 1-bit tile
    // layout) and the 1-bit factors (g1, f1, e1, 0) per member
    int small_q = 128;             // batches of at most this many queries take the scan's small-batch path
    int qplanes = 1;               // int8 query planes of the scan: 1, or 2 (q' ~ delta (q_hi + q_lo / 254), B >= 5)
    int two_stage = 0;
    float eps0 = 0.0f;             // > 0: the scan prunes with the 1-bit bound at this eps0
    uint8_t* msb = nullptr;
    float4* fac1 = nullptr;
    float* raw = nullptr;          // n x dp raw vectors (id order) or null
    int64_t ntiles = 0;
    std::vector<int64_t> h_list_off;
    int64_t max_list = 0;
};

void free_index_storage(Index* ix);

// ---- kernel timing (see erq_profile_enable) ---------------------------------
enum ProfKernel { PK_SCAN = 0, PK_QUANTIZE, PK_ROTATE, PK_PROBE, PK_RERANK, PK_SCAN_A, PK_SCAN_B,
                  PK_SCAN_C, PK_COUNT };
// diagnostics of the last scan while profiling is on (pairs scanned by the exact fallback)
void prof_note_redo(const int32_t* dev_count, hipStream_t st);
// profiling with counters (erq_profile_enable(2)) is on
bool prof_stats_on();
// returns a started record (or -1 when profiling is off); prof_end closes it
int prof_begin(int kernel, hipStream_t st);
void prof_end(int rec, hipStream_t st);

// ---- launchers (each returns hipError_t of the launch) ------------------------
// out[n x N] = A[n x K] * B where B is K x N row-major (b_trans = 0) or N x K
// row-major (b_trans = 1).  precision 0 = FP32 MFMA, 1 = BF16 MFMA.
hipError_t launch_gemm(const float* A, int64_t n, int K, const float* B, int N, int b_trans,
                       int precision, float* out, int64_t ldo, hipStream_t st);
// per-row k smallest of a n x N FP32 matrix, ascending by (value, column).
hipError_t launch_row_topk(const float* D, int64_t n, int64_t N, int k, int32_t* idx,
                           float* val, hipStream_t st);
hipError_t launch_quantize(const float* rrot, int64_t n, int dp, int bits, const float* norm2,
                           uint8_t* codes, float* f_add, float* f_rescale, float* cos_oo,
                           float2* fac, hipStream_t st);

// scan pipeline
size_t scan_workspace_bytes(int64_t nq, int nprobe, int64_t nlist, int kk, int dp, int64_t max_list);
// scan schedule in effect for an index (stored value if valid, else the rule)
int scan_nqt(const Index* ix);
int scan_pd(const Index* ix);
int scan_round1(const Index* ix);
int scan_round2(const Index* ix);
bool scan_pd_valid(int pd, int dp, int bits);
// pdist: the per-pair term (nq x nprobe) or null to compute it: ||q' - c'||^2
// for L2, -<q', c'> for the inner-product metrics (ix->metric)
// qrot: nq rows qld apart; the codes use their first dc coordinates; without
// pdist the per-pair term is computed from all dp (then qld must be dp)
int run_scan(Index* ix, const float* qrot, int64_t qld, int64_t nq, const int32_t* probes, const float* pdist,
             int nprobe, int kk, int64_t* out_ids, float* out_est, void* ws, size_t ws_bytes, hipStream_t st);
// scan factors from unpacked codes (list order) and (f_add, f_rescale):
// L2 (g_add, f_rescale) with g_add = f_add - f_rescale <y_bar, c'>; the
// inner-product metrics (0, f_rescale / 2)
// codes_u: n x dc; cent_rot: nlist x ld (its first dc coordinates are used)
// 1-bit factors of the two-stage scan (codes_u: n x dp; cent_rot rows ld apart)
hipError_t launch_scan1_fac(const uint8_t* codes_u, const int64_t* list_off, int64_t nlist, const float* cent_rot,
                            int ld, const float2* fac, const float* l1, int64_t n, int dp, int bits, float4* fac1,
                            hipStream_t st);
hipError_t launch_scan_fac(const uint8_t* codes_u, const int64_t* list_off, int64_t nlist, const float* cent_rot,
                           const float2* fac, int64_t n, int dc, int ld, int bits, int metric, float2* sfac,
                           hipStream_t st);
// rows scaled to unit length (FP32, IEEE sqrt and division; zero rows stay zero)
hipError_t launch_normalize(const float* x, int64_t n, int dp, float* out, hipStream_t st);
// exact re-rank of each query's first kc_q[i] (all kc when null) candidates
// (ids outside [0, n) skipped), keeping its k_q[i] (else k) best; a query
// with kc_q[i] == 0 gets its first candidates and their estimates copied
hipError_t launch_rerank(const float* raw, int64_t n, int dp, const float* q, int64_t nq, const int64_t* cand,
                         const float* cand_est, int kc, int k, const int32_t* kc_q, const int32_t* k_q,
                         int64_t* out_ids, float* out_d, hipStream_t st, int metric = ERQ_METRIC_L2);

// Haar orthogonal dp x dp matrix of the seed, row-major FP32, host memory (host code)
void sample_rotation(int dp, uint64_t seed, float* P);
// 64 random bits of Philox4x32-10 for (seed, stream tag, counter) (host code)
uint64_t philox_u64(uint64_t seed, uint32_t tag, uint64_t counter);

// Stable bucket sort of row ids by list: ids32[list_off[l] + j] = the j-th
// row (ascending) with assign[row] == l.  list_off (device, nlist + 1) must
// hold the exclusive prefix of the per-list counts.  Scratch: bucket_scratch_bytes.
size_t bucket_scratch_bytes(int64_t n, int64_t nlist);
hipError_t launch_bucket_sort(const int32_t* assign, int64_t n, int64_t nlist, const int64_t* list_off,
                              int32_t* ids32, void* scratch, hipStream_t st);
// Per-list means of x over the members of each list (rows ids32 in list
// order, FP64 sums in member order), into cent (FP32); empty lists keep
// their row of cent.  Scratch: list_mean_scratch_bytes.
size_t list_mean_scratch_bytes(const std::vector<int64_t>& off, int dp);
hipError_t launch_list_mean(const float* x, int dp, const int32_t* ids32, const std::vector<int64_t>& off,
                            const int64_t* list_off, float* cent, void* scratch, hipStream_t st);
hipError_t launch_gather_rows(const float* x, int dp, const int64_t* rows, int64_t m, float* out, hipStream_t st);

// list building
hipError_t launch_residual(const float* x, const int64_t* ids, const int32_t* assign, const float* cent,
                           int64_t n, int dp, float* res, float* norm2, hipStream_t st);

}  // namespace erq
