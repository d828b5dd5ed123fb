/*
 * erq.h -- C ABI of the MI355X (gfx950) implementation of Extended RaBitQ
 * (Gao et al., arXiv 2409.09913): B-bit quantisation of rotated vectors and
 * IVF search on the codes with an int8 x int8 -> int32 matrix-core scan.
 *
 * Conventions for every call:
 *  - All array arguments are DEVICE pointers (memory of the current HIP
 *    device, e.g. from torch tensors) unless the comment says "host".
 *    Arrays are dense and row-major.  Vectors live in dp dimensions, where dp
 *    is the data dimension zero-padded to a multiple of 64 (Sec. 5.1); the
 *    caller pads.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued asynchronously on it; arguments are validated synchronously
 *    before anything is enqueued.  Device faults surface at the next
 *    synchronising call.
 *  - The caller owns every input, output and workspace buffer; no call keeps
 *    a caller pointer after it returns.  An erq_index owns the copies it
 *    makes and frees them in erq_index_destroy.
 *  - Every call returns an erq_status; on a non-zero status nothing was
 *    enqueued and erq_last_error() (thread-local) describes the problem.
 *  - Sizes: dp in [64, 4096] and a multiple of 64; bits (B) in [1, 8];
 *    n, nq < 2^31.
 */
#ifndef ERQ_H
#define ERQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ERQ_OK = 0,
    ERQ_EINVAL = 1,        /* null pointer, negative or inconsistent size */
    ERQ_ESHAPE = 2,        /* dp not a multiple of 64, out of range, ... */
    ERQ_ENOMEM = 3,        /* allocation failed or workspace too small */
    ERQ_EUNSUPPORTED = 4,  /* parameter outside what the kernels implement */
    ERQ_EDEVICE = 5        /* HIP runtime error (message has the HIP text) */
} erq_status;

/* Distance of an index.  L2: squared Euclidean distance (the paper's
   setting).  IP: inner product, results ordered by the negated inner
   product (largest first); the estimate is <c, q> + <r, q> with
   <r, q> = ||r|| <o, q'> estimated as <o_bar, q'>/<o_bar, o> (Lemma 2.1),
   which the stored factors give as -(f_rescale / 2) <y_bar, q'>.  COSINE:
   the inner product of rows and queries normalised to unit length by the
   library (the paper's conclusion names both adaptations). */
typedef enum { ERQ_METRIC_L2 = 0, ERQ_METRIC_IP = 1, ERQ_METRIC_COSINE = 2 } erq_metric;

/* Thread-local description of the last non-zero status of this thread. */
const char* erq_last_error(void);

/* ABI version (major*100 + minor). */
int erq_version(void);

/* ------------------------------------------------------------------------ */
/* Rotation (Sec. 3.2.1, Sec. 3.4): out = x * P, i.e. every row r of x is    */
/* replaced by P^T r = P^{-1} r for the random orthogonal P.                 */
/* x: n x dp, P: dp x dp, out: n x dp (FP32).  precision 0 = FP32 matrix     */
/* cores; 1 = BF16 inputs with FP32 accumulation; 2 = the rotation of       */
/* erq_search: both operands split into BF16 hi/lo planes (x = hi + lo to   */
/* 2^-17 relative), three products per K chunk (lo*hi, hi*lo, hi*hi) with   */
/* FP32 accumulation, error <= 2^-14 sum_k |x_k P_kj| plus the FP32          */
/* accumulation bound; bit-identical to the rotation inside erq_search.    */
/* Precision 2 allocates its scratch planes and synchronises `stream`.     */
/* out must not alias x.                                                     */
/* ------------------------------------------------------------------------ */
int erq_rotate(const float* x, int64_t n, int32_t dp, const float* P,
               int32_t precision, float* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Quantisation, Algorithm 1 (Sec. 3.2.2) and the per-vector factors       */
/* (Sec. 3.3, Sec. 5.1).  rrot: n x dp rotated residuals r' = P^T (o_r - c). */
/* norm2: n values ||o_r - c||^2, or NULL to use ||r'||^2.                   */
/* Outputs: codes n x dp uint8 holding y_u in [0, 2^B) (unpacked),            */
/*   f_add[n] = ||r||^2, f_rescale[n] = -2 ||r||^2 / <y_bar, r'>, so that     */
/*   est = f_add + ||s||^2 + f_rescale * <y_bar, s'> (Eq. eq:dis to ip with  */
/*   Eq. eq 3.3: represent); cos_oo[n] = <o_bar, o> (may be NULL).           */
/* The codeword is the exact maximiser of <y/||y||, r'> over the grid G    */
/* found by enumerating the critical values in ascending order; equal        */
/* critical values are taken in ascending dimension order and the first     */
/* strict maximum wins.  A zero residual gives y_u = 2^{B-1} and zero        */
/* factors.                                                                  */
/* ------------------------------------------------------------------------ */
int erq_quantize(const float* rrot, int64_t n, int32_t dp, int32_t bits,
                 const float* norm2, uint8_t* codes, float* f_add,
                 float* f_rescale, float* cos_oo, void* stream);

/* ------------------------------------------------------------------------ */
/* Coarse probe of IVF (Sec. 4.1): for every query the nprobe nearest list   */
/* centroids by squared Euclidean distance ||q||^2 + ||c||^2 - 2 q.c,        */
/* ascending by (distance, list id); metric IP or COSINE: by the negated     */
/* inner product -q.c (largest inner products first; the caller normalises  */
/* for cosine).  q.c is taken on the BF16 matrix cores */
/* from a hi/lo split of both FP32 operands (three products, FP32 sums):    */
/* error <= 2^-14 sum|q_i c_i| plus FP32 accumulation, so only near-ties   */
/* may order differently from exact arithmetic.                             */
/* q: nq x dp raw queries, centroids: nlist x dp.                           */
/* probes: nq x nprobe int32 (output), pdist: nq x nprobe FP32 or NULL.       */
/* nprobe in [1, min(nlist, 1024)].  workspace: erq_probe_workspace_size     */
/* (it holds the nq x nlist distances and the BF16 hi/lo planes of q and    */
/* the centroids, so it depends on dp).                                      */
/* ------------------------------------------------------------------------ */
int erq_probe_workspace_size(int64_t nq, int64_t nlist, int32_t dp, int32_t nprobe, size_t* bytes);
int erq_coarse_probe(const float* q, int64_t nq, const float* centroids, int64_t nlist,
                     int32_t dp, int32_t nprobe, int32_t metric, int32_t* probes, float* pdist,
                     void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Index: the IVF lists of Sec. 4.1 with the quantisation codes of every     */
/* member, stored packed for the int8 matrix-core scan, plus the rotation P, */
/* raw and rotated centroids, ids and factors.  Optionally the raw vectors   */
/* for an exact re-rank (the paper's setting keeps none, Sec. 2.1).          */
/* ------------------------------------------------------------------------ */
typedef struct erq_index_s* erq_index;

/* The random orthogonal matrix of Sec. 3.2.1 (the codebook is fixed by P
   alone), sampled from the seed: Haar-distributed, the Q factor of the QR
   decomposition of a dp x dp standard-normal matrix with the signs of R's
   diagonal folded into Q.  Normals from Philox4x32-10 (counter-based, keyed
   by the seed) and Box-Muller; QR by Householder reflections in FP64 on the
   host.  P_host: dp x dp FP32, row-major, HOST memory.  Deterministic in
   (dp, seed).  No device work. */
int erq_sample_rotation(int32_t dp, uint64_t seed, float* P_host);

/* Empty index for dp-dimensional vectors, B = bits, nlist lists, distance
   `metric` (erq_metric).  P (device, dp x dp FP32) is copied; P = NULL
   samples it with erq_sample_rotation(dp, seed).  Synchronises `stream`. */
int erq_index_create(int32_t dp, int32_t bits, int64_t nlist, const float* P,
                     uint64_t seed, int32_t metric, void* stream, erq_index* out);
/* Frees everything the index owns.  No work that uses the index may still be
   in flight (freeing device memory waits for the device). */
int erq_index_destroy(erq_index idx);

/* Random projection to dc < dp dimensions before quantising (App. C): the
   codes keep the first dc coordinates of the rotated residual r' (a random
   dc-dimensional projection, P being Haar), with f_add = ||r||^2 over all dp
   coordinates and f_rescale = -(2 dp/dc) ||r'_d||^2 / <y_bar, r'_d> from the
   kept ones, so that <y_bar, s'_d> f_rescale estimates -2 <r, s>; ||s||^2
   stays exact over all dp.  Queries are rotated to their first dc
   coordinates only.  dc: a multiple of 64 in [64, dp] (dp = no projection,
   the default).  Only on an empty index (ERQ_EINVAL after a build or
   import) with the L2 metric (ERQ_EUNSUPPORTED otherwise).  Synchronises
   `stream`. */
int erq_index_set_projection(erq_index idx, int32_t dc, void* stream);
/* MSB-first two-stage scan (Sec. 4.2).  The most significant bit of every
   coordinate of y_u is RaBitQ's 1-bit code of the same residual; the scan
   first estimates every (member, query) pair from those bits alone,
     est1 = f_add + ||s||^2 + f1 <x, s'>,  x = x_b - 1/2, f1 = -4 f_add / ||r'||_1,
   drops a pair whose Lemma 2.1 lower bound
     est1 - eps0 * 2 ||r|| ||s|| sqrt(1 - c^2) / c / sqrt(D - 1),
     c = ||r'||_1 / (sqrt(D) ||r||),
   exceeds the query's current bound (an upper bound of its kk-th estimate),
   and reads the full codes only for groups of 64 members in which some pair
   is left; those pairs get the one-stage estimate.  A member of the one-stage
   top-kk is lost only when its 1-bit bound fails (probability decreasing
   like exp(-eps0^2 / 2)).  On an empty index, eps0 > 0 makes erq_index_build
   store the 1-bit data (bit planes: dp/8 bytes, factors: 16 bytes per
   member); on a built index it sets eps0 (0 = the one-stage scan; ERQ_EINVAL
   when the index has no 1-bit data).  ERQ_EUNSUPPORTED for the
   inner-product metrics, B = 1 and a projection; erq_index_import refuses an
   index that requested it.  The 1-bit data and eps0 are saved with the
   index. */
int erq_index_set_two_stage(erq_index idx, float eps0);

/* Query planes of the scan.  1 (default): q' is quantised to int8 once,
   q' ~= delta * q_int (reading C-13), whose rounding error (delta/2 per
   coordinate) is as large as the estimator's own error at large B.  2:
   a second int8 plane of the rounding remainder,
     q_lo = rint((q' / delta - q_int) * 254),  q' ~= delta * (q_int + q_lo / 254),
   products <y_u, q_int> and <y_u, q_lo> both exact in int32 on the matrix
   cores, the error 254 times smaller, at twice the matrix-core work per
   query (32 queries per work item instead of 64).  planes = 2 needs
   bits >= 5 and no two-stage scan (ERQ_EUNSUPPORTED).  A query-time setting:
   the codes do not change; saved with the index. */
int erq_index_set_query_planes(erq_index idx, int32_t planes);

/* Batches of at most max_queries queries (default 128; 0 = never) take the
   scan's small-batch path: the member tiles of each query's probed lists
   are split evenly over up to 64 workgroups that keep exact top-kk lists,
   merged by one final select, instead of the pair-grouped pipeline of large
   batches (first bound, rounds of bounded scans, selects: about 35
   launches).  Both give the exact top-kk by (estimate, id), bit for bit the
   same; the small path reads each probed list once per query rather than
   once per tile of its queries, so it suits batches whose queries share few
   lists.  It always scans in one stage (a two-stage setting applies to the
   pipeline only), and it is not used when kk > 256 at nprobe >= 16 (fewer
   than 16 workgroups per query).  max_queries in [0, 1024]; saved with the
   index. */
int erq_index_set_small_batch(erq_index idx, int32_t max_queries);

/* The index's current small-batch threshold (see erq_index_set_small_batch). */
int erq_index_small_batch(erq_index idx, int32_t* max_queries);

/* The code dimension dc (dp without a projection). */
int erq_index_code_dim(erq_index idx, int32_t* dc);

/* Copies the index's rotation P (dp x dp FP32, row-major) to P_out (device). */
int erq_index_get_rotation(erq_index idx, float* P_out, void* stream);

/* Writes the whole index to a file (host path): a versioned header (magic
   "ERQIDX", version 2, dp, bits, raw kept, metric, code dimension, nlist,
   n, tiles, scan schedule, seed, two-stage flag and eps0, query planes,
   small-batch threshold),
   then P, raw and rotated centroids, list offsets, ids, factors, scan
   factors, packed codes, when kept the raw vectors, and with the two-stage
   scan its bit planes and 1-bit factors, in native byte order.
   Synchronises `stream`. */
int erq_index_save(erq_index idx, const char* path, void* stream);
/* Reads a file of erq_index_save into a new index on the current device.
   ERQ_EINVAL for a file that is not an index, whose size does not match its
   header, or whose lists are inconsistent (checked before any device work);
   ERQ_EUNSUPPORTED for another file version.  Synchronises `stream`. */
int erq_index_load(const char* path, void* stream, erq_index* out);

/* Fills the index from caller-made contents (no quantisation on the device):
   list_off: nlist+1 int64 offsets into the list-ordered arrays; ids: n int64
   row ids, each in [0, n) (row numbers of the vectors given to
   erq_index_set_raw; ERQ_EINVAL otherwise, checked on the device before the
   call returns); codes: n x dc uint8 y_u in list order (dc = the code
   dimension, dp without a projection); f_add, f_rescale: n FP32;
   centroids, centroids_rot: nlist x dp FP32 (centroids_rot = P^T c;
   NULL -> computed with erq_rotate in FP32).  Replaces previous contents.
   Synchronises `stream`. */
int erq_index_import(erq_index idx, int64_t n, const int64_t* list_off, const int64_t* ids,
                     const uint8_t* codes, const float* f_add, const float* f_rescale,
                     const float* centroids, const float* centroids_rot, void* stream);

/* k-means for the IVF lists (Sec. 4.1 partitions the data with KMeans),
   Lloyd's algorithm on the device.  Readings of what the paper leaves open:
   the initial centroids are nlist distinct rows picked by Floyd's sampling
   with Philox4x32-10 numbers of the seed (in ascending row order); each of
   `iters` rounds assigns every row to its nearest centroid (the coarse
   probe's distances, ties to the lower id) and replaces each centroid by its
   list's mean (FP64 sums in ascending row order); an empty list keeps its
   centroid.  x: n x dp; centroids: nlist x dp output; assign: n int32 output
   (the nearest final centroid of each row) or NULL.  Every sum has a fixed
   order, so a seed gives the same result on every run.  1 <= nlist <= n,
   iters in [0, 1000].  Allocates its scratch; synchronises `stream`. */
int erq_kmeans(const float* x, int64_t n, int32_t dp, int64_t nlist, int32_t iters, uint64_t seed,
               float* centroids, int32_t* assign, void* stream);

/* Index phase on the device (Sec. 3.4 with IVF centring, Sec. 4.1, 5.1):
   x: n x dp raw vectors (row i has id i); centroids: nlist x dp, or NULL to
   build the lists with erq_kmeans (10 rounds, seeded from the index's
   seed); assign: n list ids, or NULL to assign every row to its nearest
   centroid (must be NULL when centroids is).  Per row:
   r = x - c, ||r||^2, r' = P^T r (precision as in erq_rotate), Algorithm 1,
   factors, packing.  Members are stored list by list, ids ascending
   within each list, so the same input always gives the same index.
   keep_raw != 0 keeps a copy of x for erq_rerank.
   Synchronises `stream` before returning. */
int erq_index_build(erq_index idx, const float* x, int64_t n, const float* centroids,
                    const int32_t* assign, int32_t precision, int32_t keep_raw, void* stream);

/* Copies raw vectors (n x dp, id order) into the index for erq_rerank. */
int erq_index_set_raw(erq_index idx, const float* x, int64_t n, void* stream);

/* Sizes of the index (host outputs; any may be NULL). */
int erq_index_info(erq_index idx, int64_t* n, int32_t* dp, int32_t* bits, int64_t* nlist,
                   int64_t* code_bytes);

/* Reads the contents back in list order: list_off (nlist+1), ids (n),
   codes (n x dc, y_u unpacked from the packed layout), f_add, f_rescale (n),
   centroids_rot (nlist x dp).  Any output may be NULL. */
int erq_index_export(erq_index idx, int64_t* list_off, int64_t* ids, uint8_t* codes,
                     float* f_add, float* f_rescale, float* centroids_rot, void* stream);

/* ------------------------------------------------------------------------ */
/* Scan (Sec. 3.3, Sec. 4.1): estimated squared distances of every member of */
/* the probed lists, kept as the kk smallest per query.                     */
/* qrot: nq x dp rotated queries q' = P^T q_r (with a projection the codes */
/* use the first dc coordinates, ||s'||^2 all dp); probes: nq x nprobe ids    */
/* (entries < 0 are skipped, so queries may probe fewer lists).  Every query */
/* is quantised to int8 once, symmetrically: delta = max|q'|/127,           */
/* q_i = rint(q'_i * 127/max|q'|).  For a probed list with rotated centroid */
/* c', s' = q' - c' and <y_bar, s'> = <y_bar, q'> - <y_bar, c'> (linear), so  */
/* est = f_add + ||s'||^2 + f_rescale * (delta/2 * (2 <y_u, q_int> -        */
/*       (2^B - 1) sum q_int) - <y_bar, c'>)                                 */
/* with <y_u, q_int> exact in int32 on the matrix cores, <y_bar, c'> held  */
/* per member in the index (FP64 accumulate), ||s'||^2 per pair in FP32,     */
/* the rest in FP32.                                                         */
/* Output: out_ids, out_est nq x kk ascending by (est, id); missing entries  */
/* are (-1, +inf).  kk in [1, 1024].  workspace: erq_scan_workspace_size.    */
/* ------------------------------------------------------------------------ */
int erq_scan_workspace_size(erq_index idx, int64_t nq, int32_t nprobe, int32_t kk, size_t* bytes);
int erq_scan(erq_index idx, const float* qrot, int64_t nq, const int32_t* probes,
             int32_t nprobe, int32_t kk, int64_t* out_ids, float* out_est,
             void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Exact re-rank: squared Euclidean distance (FP32) between each raw query   */
/* and its kc candidate rows (ids outside [0, n) are skipped), the k         */
/* smallest ascending by (distance, id).  Needs raw vectors in the index.    */
/* q: nq x dp, cand: nq x kc int64; out: nq x k (-1, +inf padded).  kc in    */
/* [1, 1024], k <= kc.                                                       */
/* ------------------------------------------------------------------------ */
int erq_rerank(erq_index idx, const float* q, int64_t nq, const int64_t* cand, int32_t kc,
               int32_t k, int64_t* out_ids, float* out_dist, void* stream);

/* ------------------------------------------------------------------------ */
/* With the inner-product metrics (erq_metric) the per-pair term is -<c', q'> */
/* (from the probe in erq_search, computed per pair in erq_scan), the member */
/* factors are (0, f_rescale / 2), and the results are the negated estimated */
/* inner products; the rest is the same.                                     */
/* Whole query path (Sec. 2.1 K-NN, Sec. 4.1 IVF): rotate, coarse probe,     */
/* scan, and exact re-rank of the best estimates.  The rotation q' = q P is  */
/* erq_rotate's precision 2 (error <= 2^-14 sum_k |q_k P_kj| per output,     */
/* about the FP32 accumulation bound at dp = 768).  The scan's ||s||^2 per   */
/* pair is the probe's ||q||^2 + ||c||^2 - 2 q.c, clamped at 0.              */
/* nprobe, k, rerank_k are the batch's largest values: nprobe in            */
/* [1, min(nlist, 1024)], k in [1, 1024], rerank_k 0 or in [k, 1024]        */
/* (re-rank needs raw vectors).  Per-query values (device int32 arrays of nq, */
/* each may be NULL = the batch value for every query): nprobe_q clamped to */
/* [1, nprobe]; k_q clamped to [1, k]; rerank_q 0 (estimates) or clamped to */
/* [k_q, rerank_k] (0 for all when rerank_k is 0).  A query's result does   */
/* not depend on the other queries of the batch.  Output nq x k ascending by */
/* (distance, id): estimated squared distances for a query without re-rank, */
/* exact FP32 ones with it; columns past the query's k_q are (-1, +inf).     */
/* Inner-product metrics: negated (estimated or exact) inner products; the   */
/* cosine metric normalises the queries first (rows were normalised at      */
/* build, and raw rows kept for re-rank are stored normalised).             */
/* workspace: erq_search_workspace_size(nq, nprobe, k, rerank_k).           */
/* ------------------------------------------------------------------------ */
int erq_search_workspace_size(erq_index idx, int64_t nq, int32_t nprobe, int32_t k,
                              int32_t rerank_k, size_t* bytes);
int erq_search(erq_index idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
               int32_t rerank_k, const int32_t* nprobe_q, const int32_t* k_q,
               const int32_t* rerank_q, int64_t* out_ids, float* out_dist,
               void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* erq_search without a workspace argument, for callers that cannot         */
/* allocate device memory (code under HIP graph capture, tight serving      */
/* loops, harnesses that forbid hipMalloc).  Same arguments, checks and     */
/* results as erq_search; the workspace is the library's own static device  */
/* scratch of 64 MiB (erq_static_scratch_bytes), one copy per GPU, held from */
/* the library's load until the process ends; its address is looked up on   */
/* the first call on each device.  The call makes no allocation.  Calls     */
/* whose workspace (erq_search_workspace_size) exceeds the scratch return   */
/* ERQ_ENOMEM before any device work.  Every call on a GPU uses that GPU's   */
/* one scratch: calls that may overlap on the same GPU (other streams, other */
/* host threads) race and must be serialised by the caller.                */
/* ------------------------------------------------------------------------ */
int erq_search_static(erq_index idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                      int32_t rerank_k, const int32_t* nprobe_q, const int32_t* k_q,
                      const int32_t* rerank_q, int64_t* out_ids, float* out_dist, void* stream);
int erq_static_scratch_bytes(size_t* bytes);

/* ------------------------------------------------------------------------ */
/* Scan schedule (tuning, not part of the method).  Four knobs of the        */
/* bounded scan; 0 selects the built-in rule:                                */
/*   nqt    query tiles of 32 per work item, 1 or 2 (2 needs dp <= 1536;     */
/*          rule: 2 for dp <= 768);                                          */
/*   pd     K-steps of packed codes in flight per wave, one of 1, 2, 3, 4, 6 */
/*          dividing dp/64 (6 only for bits <= 4; rule: the largest);        */
/*   round1 end of the first bounded rounds, in [1, 1024] (rule: 4): the    */
/*          first round always covers the first bound's 4 nearest ranks     */
/*          (their first 256 members are not scanned again), and round1 > 4  */
/*          adds a round [4, round1);                                        */
/*   round2 end of a middle round [round1, round2), in [0, 1024]; it takes  */
/*          effect only when round1 < round2 < nprobe (rule: no middle      */
/*          round; then, while kk times the ranks left over the ranks       */
/*          scanned exceeds 3/4 of (4096 - kk), the rest is cut at g times   */
/*          the ranks scanned, g = 16 halved while kk * (g - 1) > 1024:      */
/*          nprobe 1024 and kk 200 give [0, 4), [4, 16), [16, 64), [64, 256),*/
/*          [256, 1024)).                                                    */
/*          Each round ends with a select that lowers the bound.            */
/* No value changes a result: estimates are computed pair by pair in the    */
/* same arithmetic and the output is the exact top-kk by (estimate, id)      */
/* under every schedule.  set_tune rejects invalid values (ERQ_EINVAL) and   */
/* leaves the schedule unchanged; get_tune writes the four stored values.   */
/* erq_index_tune searches the schedule on the caller's queries and         */
/* erq_search arguments, every query with the batch values (outputs and     */
/* workspace as for erq_search; they hold                                   */
/* the last call's result on return): first (nqt, pd) over every valid pair */
/* with round1 and round2 fixed, then round1 in {2, 4, 8, 16, 32}          */
/* (< nprobe), then round2 in {0, 2, 4, 8, 16} x round1 (< nprobe); each     */
/* candidate is timed with HIP events over `reps` calls after one untimed   */
/* call, on `stream`.  It keeps the fastest, writes it to choice[0..3]       */
/* (host) and its mean milliseconds per call to *best_ms (host, may be      */
/* NULL).  It synchronises the stream and must not run concurrently with    */
/* other calls on the same index.  reps in [1, 100].  On an error the       */
/* previous schedule is restored.                                            */
/* ------------------------------------------------------------------------ */
int erq_index_set_tune(erq_index idx, int32_t nqt, int32_t pd, int32_t round1, int32_t round2);
int erq_index_get_tune(erq_index idx, int32_t* nqt, int32_t* pd, int32_t* round1, int32_t* round2);
int erq_index_tune(erq_index idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                   int32_t rerank_k, int32_t reps, int64_t* out_ids, float* out_dist,
                   void* workspace, size_t ws_bytes, void* stream, int32_t* choice, double* best_ms);

/* ------------------------------------------------------------------------ */
/* Kernel timing (measurement support, not part of the method).  While       */
/* enabled, every launch of the named kernels is bracketed by two HIP events */
/* recorded on the stream it is launched on.  Names: "scan" (the int8 matrix- */
/* core scan, all passes), "scan_a" (its first bound), "scan_b" (each launch */
/* of the bounded scan), "scan_c" (final selection and exact fallback),     */
/* "quantize", "rotate", "probe", "rerank".  "scan_redo_pairs"              */
/* returns in total_ms the number of pairs re-scanned by the exact fallback,*/
/* "scan2_groups" the groups of 64 members whose full codes the two-stage   */
/* scan did not read (total_ms) and all its groups (launches); both are     */
/* counted only with on == 2, which synchronises after each scan.           */
/* erq_profile_read waits for the recorded events and returns the summed     */
/* duration (ms) and launch count of one kernel (host outputs); reset != 0   */
/* drops the records of every kernel.                                        */
/* ------------------------------------------------------------------------ */
int erq_profile_enable(int32_t on);
int erq_profile_read(const char* kernel, double* total_ms, int64_t* launches, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* ERQ_H */
