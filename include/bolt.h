/*
 * bolt.h -- C ABI of the MI355X (gfx950) Bolt hot path.
 *
 * Bolt (Blalock & Guttag, KDD 2017) approximates a distance or similarity
 * that is a sum over dimensions (Sec. 1.1) with three functions: h encodes
 * database vectors to M 4-bit codes, g turns a query into M lookup tables of
 * 16 entries quantised to uint8, and d_hat sums one entry per table for each
 * encoded vector (Sec. 3.1, Sec. 3.2).  This library implements h, g and
 * d_hat, plus top-k retrieval (Sec. 1.2), as HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers: every array argument is a caller-owned DEVICE pointer unless the
 *   entry point says "host".  The library never takes ownership.  Outputs
 *   must not alias inputs.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  Calls validate their arguments on the host, then enqueue work
 *   on the stream and return without waiting.  A kernel fault is reported by
 *   the HIP runtime at the next synchronisation or call (BOLT_ERR_DEVICE).
 * Workspace: entry points that need scratch memory take `ws`/`ws_bytes`
 *   (device memory owned by the caller); the matching *_ws_bytes() function
 *   gives the size.  Too small a workspace returns BOLT_ERR_NOMEM.
 * Shapes: J % M == 0, M even and 2 <= M <= 256 (codes pack two 4-bit codes
 *   per byte, and M <= 256 keeps every sum below 65536).  N and Q may be 0
 *   (nothing is enqueued).  N <= 2^31 - 1 per database.
 * Inputs must be finite (NaN and Inf are not supported).
 * Errors: every call returns a bolt_status; bolt_last_error() gives a
 *   message for the calling thread's last failure.
 *
 * Layouts (canonical; the paper fixes none of them)
 *   X, Qv      fp32 [rows][ld], the first J columns used
 *   centroids  fp32 [M][16][J/M]: codebook m, centroid i, sub-dimension.
 *              Subspace m covers dimensions [m*J/M, (m+1)*J/M) (Sec. 3.1:
 *              consecutive indices).
 *   codes      uint8 [N][M/2]: byte t holds the code of subspace 2t in bits
 *              0-3 and of subspace 2t+1 in bits 4-7.
 *   luts       [Q][M][16]: table m of query q, entry i.
 */
#ifndef BOLT_H
#define BOLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bolt_status {
    BOLT_OK = 0,
    BOLT_ERR_INVALID = -1,     /* null pointer with size > 0, bad k, bad ld, misalignment */
    BOLT_ERR_SHAPE = -2,       /* J % M != 0, M odd, M outside [2, 256], N too large */
    BOLT_ERR_UNSUPPORTED = -3, /* a valid request the library does not handle (e.g. k > 2048) */
    BOLT_ERR_DEVICE = -4,      /* the HIP runtime reported an error */
    BOLT_ERR_NOMEM = -5        /* workspace too small */
} bolt_status;

/* Table metrics (Sec. 1.1, eq. distFuncForm: a sum over dimensions of a
 * per-dimension term; Sec. 1.1 also names cosine similarity):
 *   BOLT_METRIC_L2      squared L2, (q - c)^2
 *   BOLT_METRIC_DOT     dot product, q * c
 *   BOLT_METRIC_L1      L1, |q - c| (the same tables as BOLT_METRIC_LP(1))
 *   BOLT_METRIC_LP(p)   the L_p distance to the p, |q - c|^p, integer
 *                       1 <= p <= 16 (BOLT_METRIC_LP(2) gives the L2 tables)
 *   BOLT_METRIC_COSINE  cosine similarity: the dot product of the unit query
 *                       q / |q| with codebooks learned on unit database rows
 *                       (bolt_normalize_rows before bolt_encode)
 * Distances (L2, L1, L_p) retrieve the smallest sums, similarities (dot,
 * cosine) the largest.  Encoding uses squared L2 for all of them. */
enum { BOLT_METRIC_L2 = 0, BOLT_METRIC_DOT = 1, BOLT_METRIC_L1 = 2, BOLT_METRIC_COSINE = 4 };
#define BOLT_METRIC_LP(p) (3 + 256 * (p))

enum { BOLT_TOPK_MAX_K = 2048 };

/* Message describing the calling thread's most recent failure ("" if none). */
const char *bolt_last_error(void);

/* Library version string. */
const char *bolt_version(void);

/*
 * Data encoding h (Sec. 3.1, definition of h; K = 16 centroids per
 * codebook, Sec. 3.2).  For each row n and subspace m, codes receives the
 * index of the centroid of codebook m nearest to x_n^(m) in squared
 * Euclidean distance (whatever the task metric), ties to the lowest index.
 * Distances are computed in fp32 in the order
 *     acc = 0; for j ascending: t = x_j - c_j; acc = fma(t, t, acc).
 *
 *   X          device fp32 [N][ldx], ldx >= J
 *   N          rows (0 allowed)
 *   J          dimensions, J % M == 0
 *   ldx        row stride of X in elements
 *   centroids  device fp32 [M][16][J/M]
 *   M          subspaces (even, 2..256)
 *   codes      device uint8 [N][M/2], written completely
 */
int bolt_encode(const float *X, int64_t N, int32_t J, int64_t ldx,
                const float *centroids, int32_t M, uint8_t *codes, void *stream);

/*
 * Unit rows for cosine similarity (Sec. 1.1): Y[r] = X[r] / |X[r]| in fp32,
 *     s = 0; for j ascending: s = fma(x_j, x_j, s);  n = sqrt(s);  y_j = x_j / n
 * with a correctly rounded square root and division; a zero row stays zero.
 * The database side of cosine search encodes these rows (bolt_encode) with
 * codebooks learned on unit rows.
 *
 *   X   device fp32 [N][ldx], ldx >= J;   Y  device fp32 [N][ldy], ldy >= J
 *   (Y may equal X with ldy == ldx: in place)
 */
int bolt_normalize_rows(const float *X, int64_t N, int32_t J, int64_t ldx, float *Y, int64_t ldy,
                        void *stream);

/*
 * Query encoding g with the learned uint8 quantisation (Sec. 3.1,
 * definition of D; Sec. 3.2, beta_m).  For query q, table m, entry i:
 *     D = sum over j in subspace m of delta(q_j, c_ij), in fp32, j ascending,
 *         squared L2: t = q_j - c_ij; acc = fma(t, t, acc)
 *         dot:        acc = fma(q_j, c_ij, acc)
 *         L1:         acc = acc + |q_j - c_ij|
 *         L_p:        t = |q_j - c_ij|; p = 1: acc = acc + t; else
 *                     w = t, p - 2 times w = w * t, then acc = fma(w, t, acc)
 *         cosine:     u = q / |q| as bolt_normalize_rows computes it, then
 *                     acc = fma(u_j, c_ij, acc)
 *     beta = clamp(floor(fma(a, D, -offsets[m])), 0, 255)
 * offsets[m] is the table offset in quantised units, b'_m = a * F_m^-1(alpha),
 * so that the learned lower quantile maps to 0 (Sec. 3.2).
 *
 *   Qv         device fp32 [Q][ldq]
 *   metric     any of the metric codes above
 *   a          shared scale (> 0), host scalar
 *   offsets    device fp32 [M]
 *   luts_f32   device fp32 [Q][M][16] or NULL (the unquantised D)
 *   luts_u8    device uint8 [Q][M][16] or NULL
 */
int bolt_build_luts(const float *Qv, int64_t Q, int32_t J, int64_t ldq,
                    const float *centroids, int32_t M, int32_t metric, float a,
                    const float *offsets, float *luts_f32, uint8_t *luts_u8,
                    void *stream);

/*
 * The scan d_hat (Sec. 3.1, approximate distance as the sum of the table
 * entries selected by the codes; vectorised lookups, Sec. 3.2):
 *     out[q][n] = sum over m of luts_u8[q][m][code(n, m)]
 * an exact integer (below 65536 since M <= 256).  The monotone outer f of
 * the distance form (Sec. 1.1) is not applied.  The two entry points do the
 * same arithmetic; they exist so that callers name the metric the tables
 * were built for.
 *
 *   codes      device uint8 [N][M/2]
 *   luts_u8    device uint8 [Q][M][16]
 *   out        device uint16 [Q][ldo], ldo >= N
 */
int bolt_scan_l2(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                 int64_t Q, uint16_t *out, int64_t ldo, void *stream);
int bolt_scan_dot(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                  int64_t Q, uint16_t *out, int64_t ldo, void *stream);

/*
 * Top-k retrieval (Sec. 1.2, the k closest vectors; Sec. 4.5 ranks by the
 * smallest approximate distance).  For each of the Q rows of dists, the k
 * smallest values (largest = 0, squared L2) or the k largest (largest = 1,
 * dot product / maximum inner product search), ordered by value and, among
 * equal values, by ascending index.  If k > N the tail is padded with
 * vals = 65535 (largest = 0) or 0 (largest = 1) and idx = -1.
 *
 *   dists      device uint16 [Q][ldd]
 *   k          1 .. BOLT_TOPK_MAX_K
 *   vals       device uint16 [Q][k]
 *   idx        device int32 [Q][k]
 *   ws         device workspace of bolt_topk_ws_bytes(Q, N, k) bytes
 */
size_t bolt_topk_ws_bytes(int64_t Q, int64_t N, int32_t k);
int bolt_topk(const uint16_t *dists, int64_t Q, int64_t N, int64_t ldd, int32_t k,
              int32_t largest, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
              void *stream);

/*
 * Scan followed by top-k without materialising the [Q][N] sums: the same
 * result as bolt_scan_* then bolt_topk with largest = (metric == DOT).
 *
 *   codes      device uint8 [N][M/2], 16-byte aligned
 *   luts_u8    device uint8 [Q][M][16], 16-byte aligned
 *   metric     a distance metric (k smallest) or a similarity (dot, cosine:
 *              k largest); only the direction depends on it
 *   ws         device workspace of bolt_scan_topk_ws_bytes(N, M, Q, k) bytes,
 *              256-byte aligned.  M in {8, 16, 32, 64} with k <= 256 takes the
 *              fused path (workspace about Q * N * k / 2048 bytes); other M
 *              or k scan into a [Q][N] sum matrix in the workspace (Q * N * 2
 *              bytes) and select from it.
 * Errors: BOLT_ERR_INVALID for misaligned codes or tables (N > 0), a null
 * pointer, a bad metric or k; BOLT_ERR_NOMEM, naming the size, for a smaller
 * workspace.
 */
size_t bolt_scan_topk_ws_bytes(int64_t N, int32_t M, int64_t Q, int32_t k);
int bolt_scan_topk(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                   int64_t Q, int32_t metric, int32_t k, uint16_t *vals, int32_t *idx,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * bolt_scan_topk for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and result, with the workspace taken from a static
 * device array of BOLT_NOALLOC_SCRATCH_BYTES bytes that the library holds on
 * every GPU it runs on until the process ends.  The call allocates nothing.
 * Inputs and outputs are as for bolt_scan_topk and are still the caller's.
 * Errors: as bolt_scan_topk, and BOLT_ERR_UNSUPPORTED (naming the size) when
 * bolt_scan_topk_ws_bytes(N, M, Q, k) exceeds BOLT_NOALLOC_SCRATCH_BYTES.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (several streams or threads) race and must be serialised by the
 * caller.
 */
#define BOLT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int bolt_scan_topk_noalloc(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                           int64_t Q, int32_t metric, int32_t k, uint16_t *vals, int32_t *idx,
                           void *stream);

/*
 * Scan + top-k over a subset of the rows, as an index produces it (Sec. 1.2:
 * the k closest among the vectors a search visits): the union of n_ranges
 * row ranges [ranges[2r], ranges[2r+1]).  The result is that of
 * bolt_scan_topk over the rows in the ranges, with row indices into the
 * whole code matrix.  All queries of the call scan the same ranges.
 *
 *   ranges     HOST int64 [n_ranges][2], ascending, disjoint, inside [0, N]
 *   ws         device workspace of bolt_scan_topk_ranges_ws_bytes(ranges,
 *              n_ranges, M, Q, k) bytes, 256-byte aligned (0 bytes when the
 *              ranges hold no row: then every result is padding)
 * Needs the fused kernels: M in {8, 16, 32, 64}, k <= 256, codes and tables
 * 16-byte aligned, else BOLT_ERR_UNSUPPORTED.  The tile list is copied from
 * host memory on the stream (the call may wait for that copy).
 */
size_t bolt_scan_topk_ranges_ws_bytes(const int64_t *ranges, int32_t n_ranges, int32_t M,
                                      int64_t Q, int32_t k);
int bolt_scan_topk_ranges(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                          int64_t Q, int32_t metric, int32_t k, const int64_t *ranges,
                          int32_t n_ranges, uint16_t *vals, int32_t *idx, void *ws,
                          size_t ws_bytes, void *stream);

/*
 * Scan + top-k of queries under two metrics in one call (Sec. 3.1 scan,
 * Sec. 1.2 retrieval; Sec. 4.5 ranks by the smallest distance and the inner
 * product search by the largest): queries [0, q_split) are ranked as
 * bolt_scan_topk ranks them under metric_lo, and queries [q_split, Q) as
 * under metric_hi.  Every result equals that of bolt_scan_topk over the
 * query's own tables and metric.  Where the two metrics rank in opposite
 * directions and the shape runs on the matrix-core tiles, one set of
 * launches serves both sides (a distance and a similarity over the same
 * database scan together); otherwise the call runs the two sides one after
 * the other on the stream, with the same workspace.
 *
 *   luts_u8    device uint8 [Q][M][16], 16-byte aligned: rows [0, q_split)
 *              built for metric_lo, rows [q_split, Q) for metric_hi
 *   q_split    0 .. Q
 *   ws         device workspace of bolt_scan_topk_split_ws_bytes(N, M, Q,
 *              q_split, k) bytes, 256-byte aligned
 * Other arguments, results and errors as for bolt_scan_topk
 * (BOLT_ERR_INVALID also for q_split outside [0, Q]).
 */
size_t bolt_scan_topk_split_ws_bytes(int64_t N, int32_t M, int64_t Q, int64_t q_split, int32_t k);
int bolt_scan_topk_split(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                         int64_t Q, int64_t q_split, int32_t metric_lo, int32_t metric_hi,
                         int32_t k, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Approximate matrix product (Sec. 4.4: rows of the first matrix are the
 * database, columns of the second are the queries).  With dot-product
 * tables for the K query columns, the product entry is the scan sum S
 * rescaled to the original units (Sec. 3.2: y_hat = (beta + b) / a, the
 * per-table offsets adding up to one bias):
 *     out = fp32( fp32(S + bias) * scale ),  bias = sum_m offsets[m], scale = 1/a
 * with both roundings as written.
 *
 *   codes      device uint8 [N][M/2]   (the encoded first matrix, N rows)
 *   luts_u8    device uint8 [K][M][16] (dot tables of the K columns)
 *   bias       host fp32 scalar
 *   scale      host fp32 scalar
 *   out        device fp32; transpose = 0: [K][ldo] (ldo >= N),
 *              transpose = 1: [N][ldo] (ldo >= K)
 */
int bolt_amm(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
             int64_t K, float bias, float scale, float *out, int64_t ldo,
             int32_t transpose, void *stream);

/*
 * Bolt No Quantize (Sec. 4.2: Bolt's encoding with the float tables instead
 * of their uint8 quantisation, the control for what the quantiser costs in
 * accuracy).  out[q][n] is the fp32 sum of the float table entries selected
 * by the codes, in one fixed order: acc = 0, then acc = acc + luts_f32[q][m]
 * [code(n, m)] for m = 0 .. M-1, each add rounded to nearest (no fused
 * operations), so the result is the same bit for bit on any device.
 *
 *   codes      device uint8 [N][M/2], any even M in [2, 256]
 *   luts_f32   device fp32 [Q][M][16] (the luts_f32 of bolt_build_luts)
 *   out        device fp32 [Q][ldo], ldo >= N
 * Errors: BOLT_ERR_SHAPE for a bad M, N or Q; BOLT_ERR_INVALID for null
 * pointers or ldo < N; BOLT_ERR_UNSUPPORTED above 524280 queries per call.
 */
int bolt_scan_f32(const uint8_t *codes, int64_t N, int32_t M, const float *luts_f32,
                  int64_t Q, float *out, int64_t ldo, void *stream);

/*
 * Top-k of fp32 rows (the float-table scan's retrieval, Sec. 1.2): per row
 * of dists the k smallest values (largest = 0) or the k largest (largest =
 * 1), ordered by value and, among equal values, by ascending index.  Inputs
 * must be finite.  If k > N the tail holds +inf (largest = 0) or -inf
 * (largest = 1) with idx = -1.
 *
 *   dists      device fp32 [Q][ldd], ldd >= N
 *   k          1 .. BOLT_TOPK_MAX_K
 *   vals       device fp32 [Q][k];  idx  device int32 [Q][k]
 */
int bolt_topk_f32(const float *dists, int64_t Q, int64_t N, int64_t ldd, int32_t k,
                  int32_t largest, float *vals, int32_t *idx, void *stream);

/*
 * Batched scan + top-k over many encoded databases of uneven size in one
 * persistent launch: the scan + top-k of bolt_scan_topk (Sec. 3.1 scan,
 * Sec. 1.2 the k closest vectors) for every (database, query) of the batch,
 * with bit-identical results.
 *
 * bolt_batch_db describes one database and its queries (all DEVICE pointers):
 *   codes [N][M/2], luts [Q][M][16] (16-byte aligned), vals [Q][k] and idx
 *   [Q][k] receive the sorted top k as in bolt_scan_topk (k smallest sums for
 *   BOLT_METRIC_L2, k largest for BOLT_METRIC_DOT).  M in {8, 16, 32, 64},
 *   1 <= k <= 256.  Q = 0 databases are ignored; N = 0 gives padding.
 * bolt_batch_tuning (may be NULL for defaults): rows_per_tile (multiple of
 *   1024 in [1024, 65536], default 16384), few_max_q (databases with at most
 *   this many queries use the pair-table path, 0..7, default 2), blocks_per_cu
 *   (persistent workgroups per CU, 1..8, default 3).
 * bolt_batch_plan_create builds the tile list on the host, uploads it into
 *   the caller-owned DEVICE workspace ws (bolt_batch_ws_bytes bytes, 256-byte
 *   aligned; it also holds the candidate lists) and synchronises the stream.
 *   The plan (a host object) and ws must outlive every run.
 * bolt_batch_run enqueues one batched pass on the stream: it reads the
 *   current contents of every luts buffer, so new queries can be written in
 *   place between runs.  Runs sharing a plan must not overlap.
 * bolt_batch_graph_create captures one run in a HIP graph (instantiated,
 *   returned as void*); bolt_batch_graph_launch replays it on a stream.
 */
typedef struct bolt_batch_db {
    const uint8_t *codes;
    int64_t N;
    int32_t M;
    int32_t metric;
    const uint8_t *luts;
    int32_t Q;
    int32_t k;
    uint16_t *vals;
    int32_t *idx;
} bolt_batch_db;

typedef struct bolt_batch_tuning {
    int32_t rows_per_tile;
    int32_t few_max_q;
    int32_t blocks_per_cu;
} bolt_batch_tuning;

typedef struct bolt_batch_plan bolt_batch_plan;

size_t bolt_batch_ws_bytes(const bolt_batch_db *dbs, int32_t n_db, const bolt_batch_tuning *tuning);
int bolt_batch_plan_create(const bolt_batch_db *dbs, int32_t n_db, const bolt_batch_tuning *tuning,
                           void *ws, size_t ws_bytes, void *stream, bolt_batch_plan **plan);
int bolt_batch_run(const bolt_batch_plan *plan, void *stream);
int bolt_batch_plan_info(const bolt_batch_plan *plan, int64_t *n_tiles, int64_t *n_queries,
                         int32_t *grid);
int bolt_batch_plan_destroy(bolt_batch_plan *plan);
int bolt_batch_graph_create(const bolt_batch_plan *plan, void **graph_exec);
int bolt_batch_graph_launch(void *graph_exec, void *stream);
int bolt_batch_graph_destroy(void *graph_exec);

/*
 * Offline phase (Sec. 1.2), on the HOST: codebooks by k-means with K = 16
 * per subspace (Sec. 3.1, 3.2), then the quantiser of Sec. 3.2 for one
 * metric.  All pointers are HOST pointers.  Random choices are inputs:
 * init_rows holds the 16 training rows that seed every codebook.
 *
 *   X          host fp32 [n][ldx] training vectors
 *   iters      Lloyd iterations (assignment ties to the lowest index; an empty
 *              cluster keeps its centroid)
 *   init_rows  host int64 [16], distinct rows of X
 *   Qt         host fp32 [nq][ldq] training queries
 *   metric     metric the tables will be built for
 *   alphas     host fp64 [nalpha] grid of tail fractions
 *   centroids  host fp32 [M][16][J/M] (output)
 *   a          host fp32 (output): shared scale
 *   offsets    host fp32 [M] (output): b'_m = a * F_m^-1(alpha)
 *   alpha_idx  host int32 (output, may be NULL): the chosen grid index
 * The distribution of table m is the multiset of D_m[h(x)_m](q) over all
 * (training query, training vector) pairs; b_m is its alpha-quantile, a =
 * 255 / (1-alpha)-quantile of (y - b_m) pooled over all tables (1 if that
 * is not positive), quantiles by linear interpolation between order
 * statistics; the alpha with the smallest mean squared reconstruction error
 * wins, ties to the smaller alpha.
 */
/*
 * Codebook learning on the GPU: the k-means of bolt_train_host (K = 16 per
 * subspace, Sec. 3.1, 3.2) with its data and centroids in device memory.
 * Lloyd iterations: every (row, subspace) goes to the centroid at the
 * smallest fp64 squared distance (ascending dimension order, ties to the
 * lowest index), each centroid becomes the fp64 mean of its rows rounded to
 * fp32, and an empty cluster keeps its centroid.  The fp64 means are summed
 * in parallel order: bit-identical to ascending-row sums whenever those are
 * exact (integer-valued data), else within the last bit of the fp32 result.
 *
 *   X          device fp32 [n][ldx] training vectors, n >= 16
 *   iters      Lloyd iterations, 0 .. 10000
 *   init_rows  HOST int64 [16]: centroid i of every subspace starts at row
 *              init_rows[i] (the random choice is an input)
 *   centroids  device fp32 [M][16][J/M] (output)
 *   objective  HOST fp64 [iters + 1] (output, may be NULL): total squared
 *              error of the assignment before each update and after the last
 *   ws         device workspace of bolt_kmeans_ws_bytes(J, M, iters) bytes,
 *              256-byte aligned
 * The call synchronises the stream before it returns.  J * 16 fp64 sums are
 * kept in LDS: BOLT_ERR_UNSUPPORTED for J above about 1100.
 */
size_t bolt_kmeans_ws_bytes(int32_t J, int32_t M, int32_t iters);
int bolt_kmeans(const float *X, int64_t n, int32_t J, int64_t ldx, int32_t M, int32_t iters,
                const int64_t *init_rows, float *centroids, double *objective, void *ws,
                size_t ws_bytes, void *stream);

/*
 * Learning the quantiser on the GPU (Sec. 3.2): the search of
 * bolt_learn_quantizer_host with the training queries, training codes and
 * centroids in device memory.  For each alpha of the grid, b_m is the
 * alpha-quantile of table m's distribution (D_m[i](q) over the training
 * queries q, weighted by the number of training vectors with code i in
 * subspace m; fp64 tables), a = 255 / the (1 - alpha)-quantile of y - b_m
 * pooled over all tables (a = 1 if not positive), b'_m = fp32(fp32(a) b_m),
 * and the loss is the weighted mean squared reconstruction error; the
 * smallest loss wins, ties to the smaller alpha.  Quantiles interpolate
 * linearly between order statistics.  For the chosen alpha, a and b' are the
 * fp64 operations of the definition in its order (bit-identical to a
 * sequential evaluation); the losses are summed in parallel order.  L_p
 * tables take |q - c|^p as repeated fp64 products.
 *
 *   Qt         device fp32 [nq][ldq] training queries, 1 <= nq <= 1024
 *   codes      device uint8 [n][M/2] codes of the n training vectors
 *   centroids  device fp32 [M][16][J/M]
 *   alphas     HOST fp64 [nalpha], each in [0, 0.5), 1 <= nalpha <= 64
 *   a          HOST fp32 (output): the shared scale
 *   offsets    device fp32 [M] (output): b'_m
 *   alpha_idx  HOST int32 (output, may be NULL): the chosen grid index
 *   losses     HOST fp64 [nalpha] (output, may be NULL)
 *   ws         device workspace of bolt_learn_quantizer_ws_bytes(nq, M, nalpha)
 *              bytes, 256-byte aligned (0 for unsupported sizes)
 * The call synchronises the stream before it returns.
 */
size_t bolt_learn_quantizer_ws_bytes(int64_t nq, int32_t M, int32_t nalpha);
int bolt_learn_quantizer(const float *Qt, int64_t nq, int32_t J, int64_t ldq, const uint8_t *codes,
                         int64_t n, const float *centroids, int32_t M, int32_t metric,
                         const double *alphas, int32_t nalpha, float *a, float *offsets,
                         int32_t *alpha_idx, double *losses, void *ws, size_t ws_bytes, void *stream);

int bolt_train_host(const float *X, int64_t n, int32_t J, int64_t ldx, int32_t M,
                    int32_t iters, const int64_t *init_rows, const float *Qt, int64_t nq,
                    int64_t ldq, int32_t metric, const double *alphas, int32_t nalpha,
                    float *centroids, float *a, float *offsets, int32_t *alpha_idx);

/*
 * Quantiser only (the second half of bolt_train_host) for already learned
 * centroids: lets one set of codebooks serve both metrics.  HOST pointers;
 * codes are the packed codes of the n training vectors.
 */
int bolt_learn_quantizer_host(const float *Qt, int64_t nq, int32_t J, int64_t ldq,
                              const uint8_t *codes, int64_t n, const float *centroids,
                              int32_t M, int32_t metric, const double *alphas,
                              int32_t nalpha, float *a, float *offsets, int32_t *alpha_idx);

/*
 * Kernel timing: with bolt_prof_enable(1), every library kernel launch is
 * bracketed by HIP events recorded on its own stream (not inside graph
 * capture).  bolt_prof_only(prefix) restricts that to the launches whose
 * name starts with prefix (a HOST string, copied; NULL or "" times every
 * launch), so that a timed loop pays the events' stream time only for the
 * kernels it measures.  bolt_prof_read waits for the recorded events and
 * writes "name=launches:milliseconds;" for every kernel name into names (a
 * HOST buffer of cap bytes, NUL-terminated, truncated if short); it returns
 * the full length and, with reset != 0, clears the totals.
 */
int bolt_prof_enable(int32_t on);
int bolt_prof_only(const char *prefix);
int bolt_prof_read(char *names, size_t cap, int32_t reset);

/*
 * Test hooks (not part of the hot path): pin the scan kernel (-1 automatic,
 * 0 plain loop, 1 pair tables for few queries, 2 grouped, 3 int8 matrix
 * cores for M in {8, 16, 32, 64}), route
 * bolt_scan_topk through the unfused scan-then-select path (on != 0), and
 * pin the kernel of fused scans with many queries (-1 automatic, 2 grouped
 * LDS tables, 3 int8 matrix cores; 3 applies only where k <= 128, otherwise
 * the grouped kernel runs).  Process-wide settings, not thread-safe.
 */
int bolt_debug_force_scan_kernel(int32_t kind);
int bolt_debug_force_unfused_topk(int32_t on);
int bolt_debug_force_fused_kind(int32_t kind);
/*
 * Test hook: speculative starting bounds of fused scans with many queries
 * over a whole database (-1 automatic and 1 on, both from 2^16 rows, also
 * for the databases of a batched plan; 0 off; 2 as 1 with every bound made
 * to fail, so that every query takes the exact recomputation).  Results are
 * the same in every mode.
 */
int bolt_debug_speculation(int32_t mode);
/*
 * Test hook: the int8 matrix-core tiles contract the one-hot codes with the
 * sparse instruction (on != 0, the default: four subspaces per instruction
 * from a 4:2-structured operand) or the dense one (two subspaces per
 * instruction).  Results are the same either way.
 */
int bolt_debug_sparse_mfma(int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* BOLT_H */
