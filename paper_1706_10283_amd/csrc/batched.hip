// Many queries against many encoded databases of uneven size in one
// persistent launch (the batched form of the scan + top-k of Sec. 3.1 and
// Sec. 1.2).
//
// Plan (host): every database is cut into tiles (query block x row block):
// query blocks of 32 on the int8 matrix cores (M = 16, 32 or 64, 8 or more
// queries, k <= 128), of 16 (8 for M = 64) on the grouped path, or all of a
// database's queries on the pair-table path when they are few; row blocks
// of `rows_per_tile` rows.  Tiles are sorted by decreasing work so that the
// dynamic schedule hands out the longest tiles first.  The descriptors, the
// per-database candidate lists and per-query bounds live in one caller-owned
// workspace.
//
// Run (device): a fill kernel resets the tile counters and the bounds; a
// persistent kernel (a few workgroups per CU) pulls the matrix-core tiles
// from one counter and a second one the other tiles from another, each
// until it passes its tile count, so every wave exits; a merge kernel then
// turns each query's candidate lists into its sorted top k, and a
// persistent recomputation kernel redoes, on the whole GPU, any query whose
// sampled bound failed (its workgroups exit at once when none did).  The launches
// depend only on the plan, so they can be captured once in a HIP graph and
// replayed with new query tables in place.  Results are
// bit-identical to bolt_scan_topk on each database alone: the sums are exact
// integers and the keys totally ordered.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "scan_common.hpp"
#include "tiles.hpp"

namespace {

struct DevDb {
    const uint8_t *codes;
    const uint8_t *luts;
    uint64_t *cand;
    uint32_t *gthr;
    uint16_t *vals;
    int32_t *idx;
    int64_t N;
    int64_t n_rb;
    int32_t M;
    int32_t Q;
    int32_t k;
    int32_t largest;
    // speculative starting bounds (matrix-core databases from kSpecMinRows rows)
    uint16_t *sdist;   // sample group minima [Q][G], or null: no speculation
    int64_t G;         // group minima per query: G / kSpecGroups chunks at a stride of `stride` rows
    int64_t stride;
    int32_t spec_r;    // rank of the sample group minimum taken as the bound
    int32_t pad;
    uint32_t *fail;    // per query: a barrier-free tile overflowed, recompute exactly
    uint32_t *lcnt;    // speculative databases: per-query dense candidate lists (count of cand[q])
};

// One sample work item: queries [q0, q0 + 32) of a database over one chunk.
struct DevSample {
    int32_t db;
    int32_t q0;
    int32_t chunk;
    int32_t pad;
};

struct DevTile {
    int32_t db;
    int32_t kind;   // 1 pair tables (few queries), 2 grouped, 3 matrix cores
    int32_t q0;
    int32_t nq;
    int64_t rb;
};

struct DevQuery {
    int32_t db;
    int32_t q;
};

// Largest LDS footprint of any tile: GroupedLds<32, 2>, MfmaLds<1> or a
// few-query tile of at most this many bytes.
constexpr size_t kBatchLds = 49664;

// Workgroups of the persistent recomputation launch (the number of listed
// queries is known only on the device).
constexpr int64_t kRedoGrid = 1024;
constexpr int64_t kRedoMergeGrid = 64;

__global__ void batch_reset_kernel(uint32_t *counter, uint32_t *gthr, uint32_t *fail, uint32_t *lcnt, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < 4)   // matrix-core tiles (M = 16, 32), other tiles, matrix-core tiles (M = 64), recomputation list
        counter[i] = 0;
    if (i < n) {
        gthr[i] = 0xFFFFu;
        fail[i] = 0u;
        lcnt[i] = 0u;
    }
}

template <int MM, bool MF>
__device__ void run_tile(const DevDb &db, const DevTile &t, int64_t rows_per_tile, char *lds)
{
    bolt::TileJob job;
    job.codes = db.codes;
    job.luts = db.luts;
    job.cand = db.cand;
    job.gthr = db.gthr;
    job.rb = t.rb;
    job.r0 = t.rb * rows_per_tile;
    job.r1 = (job.r0 + rows_per_tile) < db.N ? (job.r0 + rows_per_tile) : db.N;
    job.n_rb = db.n_rb;
    job.q0 = t.q0;
    job.nq = t.nq;
    job.k = (uint32_t)db.k;
    job.order = bolt::one_order(db.largest != 0);
    job.fail = db.fail;
    job.lcnt = MF && db.sdist ? db.lcnt : nullptr;
    if (MF) {
        // sampled bounds: barrier-free passes (overflow flags the query)
        if (db.sdist)
            bolt::mfma_tile<MM, 1, true, true>(job, *reinterpret_cast<bolt::MfmaLds<1> *>(lds));
        else
            bolt::mfma_tile<MM, 1, false, true>(job, *reinterpret_cast<bolt::MfmaLds<1> *>(lds));
    } else if (t.kind == 1) {
        bolt::few_tile<MM, false>(job, lds);
    } else {
        constexpr int NG = MM <= 32 ? 2 : 1;
        bolt::grouped_tile<MM, NG>(job, *reinterpret_cast<bolt::GroupedLds<MM, NG> *>(lds));
    }
}

// F = 1: the matrix-core tiles of M = 16 and 32, F = 2: those of M = 64,
// F = 0: the pair-table and grouped tiles.  Each family is a launch of its
// own, so that each keeps its own register budget (at M = 64 the tables
// alone take 128 registers: two waves per SIMD).
template <int F>
__global__ __launch_bounds__(256) void batch_scan_kernel(const DevDb *__restrict__ dbs,
                                                         const DevTile *__restrict__ tiles,
                                                         int32_t n_tiles, int64_t rows_per_tile,
                                                         uint32_t *counter)
{
    static_assert(sizeof(bolt::GroupedLds<32, 2>) <= kBatchLds, "grouped tile LDS");
    static_assert(sizeof(bolt::GroupedLds<64, 1>) <= kBatchLds, "grouped tile LDS");
    static_assert(sizeof(bolt::GroupedLds<16, 2>) <= kBatchLds, "grouped tile LDS");
    static_assert(sizeof(bolt::GroupedLds<8, 2>) <= kBatchLds, "grouped tile LDS");
    static_assert(sizeof(bolt::MfmaLds<1>) <= kBatchLds, "matrix-core tile LDS");
    __shared__ __attribute__((aligned(16))) char lds[F ? sizeof(bolt::MfmaLds<1>) : kBatchLds];
    __shared__ int32_t sh_tile;
    for (;;) {
        if (threadIdx.x == 0)
            sh_tile = (int32_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int32_t ti = sh_tile;
        __syncthreads();   // everyone has read sh_tile; the previous tile is done with LDS
        if (ti >= n_tiles)
            break;
        const DevTile t = tiles[ti];
        const DevDb db = dbs[t.db];
        if (F == 2) {   // M = 64 only
            run_tile<64, true>(db, t, rows_per_tile, lds);
            continue;
        }
        if (F == 1) {   // M = 16 or 32 only (see tile_kind)
            if (db.M == 16)
                run_tile<16, true>(db, t, rows_per_tile, lds);
            else
                run_tile<32, true>(db, t, rows_per_tile, lds);
            continue;
        }
        switch (db.M) {
        case 8: run_tile<8, false>(db, t, rows_per_tile, lds); break;
        case 16: run_tile<16, false>(db, t, rows_per_tile, lds); break;
        case 32: run_tile<32, false>(db, t, rows_per_tile, lds); break;
        default: run_tile<64, false>(db, t, rows_per_tile, lds); break;
        }
    }
}

// Sample group minima of the speculative bounds (as in the one-database
// path): one workgroup per work item.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batch_sample_kernel(
    const DevDb *__restrict__ dbs, const DevSample *__restrict__ items)
{
    __shared__ bolt::OneHot onehot;
    __shared__ __attribute__((aligned(16))) uint16_t gmin[32 * bolt::kSpecGminStride];
    const DevSample it = items[blockIdx.x];
    const DevDb db = dbs[it.db];
    const int nq = (db.Q - it.q0) < 32 ? (db.Q - it.q0) : 32;
    const int64_t r0 = (int64_t)it.chunk * db.stride, g0 = (int64_t)it.chunk * bolt::kSpecGroups;
    const bolt::RankOrder order = bolt::one_order(db.largest != 0);
    if (db.M == 16)
        bolt::mfma_sample_tile<16, 1, true>(db.codes, db.luts, it.q0, nq, order, r0, db.sdist, db.G, g0, onehot,
                                            gmin);
    else if (db.M == 32)
        bolt::mfma_sample_tile<32, 1, true>(db.codes, db.luts, it.q0, nq, order, r0, db.sdist, db.G, g0, onehot,
                                            gmin);
    else
        bolt::mfma_sample_tile<64, 1, true>(db.codes, db.luts, it.q0, nq, order, r0, db.sdist, db.G, g0, onehot,
                                            gmin);
}

// Starting bound of each query of a speculative database: the r-th smallest
// of its sample group minima (0 when a test forces the recomputation); other
// queries keep the open bound.
__global__ __launch_bounds__(256) void batch_select_kernel(const DevDb *__restrict__ dbs,
                                                           const DevQuery *__restrict__ queries, int force_fail)
{
    __shared__ __attribute__((aligned(16))) uint32_t h[bolt::kHistBins];
    const DevQuery qq = queries[blockIdx.x];
    const DevDb db = dbs[qq.db];
    if (!db.sdist)
        return;
    const uint32_t b = bolt::select_rank_u16(db.sdist + (int64_t)qq.q * db.G, db.G, (uint32_t)db.spec_r,
                                             bolt::hist_shift(db.M), h);
    if (threadIdx.x == 0)
        db.gthr[qq.q] = force_fail ? 0u : b;
}

// Top k of one query from its candidate lists.  A query of a speculative
// database with fewer than k candidates, or flagged by an overflowing
// barrier-free tile, is listed for the exact recomputation instead: its
// bound is opened and its index into `queries` is appended to redo (count
// in *redo_cnt).
__global__ __launch_bounds__(256) void batch_merge_kernel(const DevDb *__restrict__ dbs,
                                                          const DevQuery *__restrict__ queries,
                                                          uint32_t *__restrict__ redo_cnt,
                                                          uint32_t *__restrict__ redo)
{
    __shared__ bolt::MergeLds L;
    __shared__ __attribute__((aligned(16))) uint32_t h[bolt::kHistBins];
    const DevQuery qq = queries[blockIdx.x];
    const DevDb db = dbs[qq.db];
    const int64_t per_query = db.n_rb * db.k;
    const uint32_t k = (uint32_t)db.k;
    // speculative databases: the dense list of the barrier-free tiles; others: padded slots
    const uint64_t *src = db.cand + (int64_t)qq.q * per_query;
    const uint32_t n =
        db.sdist ? bolt::merge_collect_list(L, h, src,
                                            (int64_t)db.lcnt[qq.q] < per_query ? (int64_t)db.lcnt[qq.q] : per_query, k,
                                            bolt::hist_shift(db.M), db.gthr[qq.q], false)
                 : bolt::merge_collect(L, src, 0, per_query, k, db.gthr[qq.q], false);
    if (db.sdist && (n < k || db.fail[qq.q])) {
        if (threadIdx.x == 0) {
            db.gthr[qq.q] = 0xFFFFu;
            redo[atomicAdd(redo_cnt, 1u)] = blockIdx.x;
        }
        return;
    }
    bolt::merge_finish(L, n, k, db.largest, 255u * (uint32_t)db.M, db.vals + (int64_t)qq.q * db.k,
                       db.idx + (int64_t)qq.q * db.k);
}

// Exact recomputation of the listed queries on the whole GPU: item i of the
// persistent loop is (listed query i / max_rb, row block i % max_rb), a
// one-query tile from the open bound over that row block of the query's
// database (items past the database's row blocks are skipped), writing its
// local top k to the query's own candidate slot (free since the merge).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_redo_scan_kernel(
    const DevDb *__restrict__ dbs, const DevQuery *__restrict__ queries, const uint32_t *__restrict__ redo_cnt,
    const uint32_t *__restrict__ redo, int64_t max_rb, int64_t rows_per_tile)
{
    constexpr size_t kL8 = bolt::one_query_lds_bytes(8), kL16 = bolt::one_query_lds_bytes(16),
                     kL32 = bolt::one_query_lds_bytes(32), kL64 = bolt::one_query_lds_bytes(64);
    constexpr size_t kA = kL8 > kL16 ? kL8 : kL16, kB = kL32 > kL64 ? kL32 : kL64;
    __shared__ __attribute__((aligned(16))) char lds[kA > kB ? kA : kB];   // one buffer for every code size
    const int64_t items = (int64_t)*redo_cnt * max_rb;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const DevQuery qq = queries[redo[it / max_rb]];
        const DevDb db = dbs[qq.db];
        const int64_t rb = it % max_rb;
        if (rb >= db.n_rb)
            continue;   // uniform across the workgroup
        const int64_t r0 = rb * rows_per_tile;
        const int64_t r1 = (r0 + rows_per_tile) < db.N ? (r0 + rows_per_tile) : db.N;
        const uint8_t *lq = db.luts + (int64_t)qq.q * db.M * 16;
        uint64_t *dst = db.cand + ((int64_t)qq.q * db.n_rb + rb) * db.k;
        uint32_t *g = db.gthr + qq.q;
        switch (db.M) {
        case 8: bolt::one_query_tile<8>(db.codes, r0, r1, lq, (uint32_t)db.k, db.largest, dst, nullptr, nullptr, g, lds); break;
        case 16: bolt::one_query_tile<16>(db.codes, r0, r1, lq, (uint32_t)db.k, db.largest, dst, nullptr, nullptr, g, lds); break;
        case 32: bolt::one_query_tile<32>(db.codes, r0, r1, lq, (uint32_t)db.k, db.largest, dst, nullptr, nullptr, g, lds); break;
        default: bolt::one_query_tile<64>(db.codes, r0, r1, lq, (uint32_t)db.k, db.largest, dst, nullptr, nullptr, g, lds); break;
        }
        __syncthreads();   // the tile's writer is done with lds
    }
}

// Merge of the recomputed queries: workgroup w takes listed queries w,
// w + grid, ...: the exact k smallest keys of the query's padded slots at or
// below its published bound, sorted.
__global__ __launch_bounds__(256) void batch_redo_merge_kernel(const DevDb *__restrict__ dbs,
                                                               const DevQuery *__restrict__ queries,
                                                               const uint32_t *__restrict__ redo_cnt,
                                                               const uint32_t *__restrict__ redo)
{
    __shared__ bolt::MergeLds L;
    const uint32_t n_redo = *redo_cnt;
    for (uint32_t j = blockIdx.x; j < n_redo; j += gridDim.x) {
        const DevQuery qq = queries[redo[j]];
        const DevDb db = dbs[qq.db];
        const int64_t per_query = db.n_rb * db.k;
        const uint32_t k = (uint32_t)db.k;
        const uint32_t n = bolt::merge_collect(L, db.cand + (int64_t)qq.q * per_query, 0, per_query, k,
                                               db.gthr[qq.q], false);
        bolt::merge_finish(L, n, k, db.largest, 255u * (uint32_t)db.M, db.vals + (int64_t)qq.q * db.k,
                           db.idx + (int64_t)qq.q * db.k);
        __syncthreads();
    }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    size_t dbs_off, tiles_off, queries_off, gthr_off, fail_off, redo_off, lcnt_off, counter_off, samples_off, cand_off,
        total;
    int64_t n_tiles, n_queries, n_samples, max_rb;
};

// Speculative bounds of a matrix-core database (as the one-database path
// decides them): the number of sample chunks, or 0 for none.
int64_t spec_chunks(const bolt_batch_db &d, int kind)
{
    const int mode = bolt::g_spec_mode;
    if (kind != 3 || mode == 0 || d.N < (mode > 0 ? bolt::kSpecMinRowsForced : bolt::kSpecMinRows))
        return 0;
    int64_t nsc = d.N / 32 / bolt::kSpecSpan;
    nsc = nsc < 16 ? 16 : (nsc > 256 ? 256 : nsc);
    while (nsc > 16 && (int64_t)d.Q * nsc * bolt::kSpecSpan > bolt::kSpecMaxDists)
        nsc /= 2;
    return (int64_t)d.Q * nsc * bolt::kSpecSpan > bolt::kSpecMaxDists ? 0 : nsc;
}

int resolve(const bolt_batch_tuning *tuning, int32_t &rows, int32_t &few_max, int32_t &per_cu)
{
    rows = tuning && tuning->rows_per_tile ? tuning->rows_per_tile : 16384;
    few_max = tuning && tuning->few_max_q ? tuning->few_max_q : 2;
    per_cu = tuning && tuning->blocks_per_cu ? tuning->blocks_per_cu : 3;
    if (rows < 1024 || rows > bolt::kTileRowsMax || rows % 1024)
        return bolt::fail(BOLT_ERR_INVALID, "rows_per_tile must be a multiple of 1024 in [1024, 65536]");
    if (few_max < 0 || few_max > 7)
        return bolt::fail(BOLT_ERR_INVALID, "few_max_q must be in [0, 7]");
    if (per_cu < 1 || per_cu > 8)
        return bolt::fail(BOLT_ERR_INVALID, "blocks_per_cu must be in [1, 8]");
    return BOLT_OK;
}

// Pair-table tiles need their LDS to fit the persistent kernel's buffer.
bool few_fits(int M, int nq) { return bolt::few_tile_lds_bytes(M, nq) <= kBatchLds; }

// Tile kind of a database: 1 pair tables (at most few_max queries), 3
// matrix cores (M = 16, 32 or 64, three or more queries: a part-filled
// 32-query tile costs about what a full one costs and beats the pair-table
// and grouped kernels from three; k within the tile's candidate buffer),
// else 2 grouped.
int tile_kind(const bolt_batch_db &d, int few_max)
{
    if (d.Q <= few_max && few_fits(d.M, d.Q))
        return 1;
    if (d.M >= 16 && d.Q >= 3 && d.k <= bolt::kMfmaCap - bolt::kMfmaPass)
        return 3;
    return 2;
}

int validate(const bolt_batch_db *dbs, int32_t n_db)
{
    if (n_db < 0 || (n_db > 0 && !dbs))
        return bolt::fail(BOLT_ERR_INVALID, "bad database list");
    for (int i = 0; i < n_db; ++i) {
        const bolt_batch_db &d = dbs[i];
        if (!(d.M == 8 || d.M == 16 || d.M == 32 || d.M == 64))
            return bolt::fail(BOLT_ERR_UNSUPPORTED, "database %d: M must be 8, 16, 32 or 64", i);
        if (d.N < 0 || d.N > INT32_MAX || d.Q < 0)
            return bolt::fail(BOLT_ERR_SHAPE, "database %d: bad N or Q", i);
        if (d.k < 1 || d.k > 256)
            return bolt::fail(BOLT_ERR_UNSUPPORTED, "database %d: k must be in [1, 256]", i);
        bolt::Metric mt;
        if (bolt::decode_metric(d.metric, &mt) != BOLT_OK)
            return bolt::fail(BOLT_ERR_INVALID, "database %d: bad metric %d", i, d.metric);
        if (d.Q > 0 && (!d.luts || !d.vals || !d.idx || (d.N > 0 && !d.codes)))
            return bolt::fail(BOLT_ERR_INVALID, "database %d: null pointer", i);
        if (!bolt::aligned(d.codes, 16) || !bolt::aligned(d.luts, 16))
            return bolt::fail(BOLT_ERR_INVALID, "database %d: codes and tables must be 16-byte aligned", i);
    }
    return BOLT_OK;
}

Layout layout_of(const bolt_batch_db *dbs, int32_t n_db, int32_t rows, int32_t few_max)
{
    Layout L{};
    int64_t tiles = 0, queries = 0, samples = 0, max_rb = 0;
    size_t cand = 0;
    for (int i = 0; i < n_db; ++i) {
        const bolt_batch_db &d = dbs[i];
        if (d.Q == 0)
            continue;
        const int64_t n_rb = (d.N + rows - 1) / rows;   // 0 for an empty database: padding only
        const int kind = tile_kind(d, few_max);
        const int qb = kind == 3 ? 32 : (d.M <= 32 ? 16 : 8);
        const int64_t n_qb = kind == 1 ? 1 : (d.Q + qb - 1) / qb;
        tiles += n_rb * n_qb;
        queries += d.Q;
        cand += align256((size_t)d.Q * n_rb * d.k * sizeof(uint64_t));
        const int64_t nsc = spec_chunks(d, kind);
        if (nsc) {
            max_rb = n_rb > max_rb ? n_rb : max_rb;
            samples += (d.Q + 31) / 32 * nsc;
            cand += align256((size_t)d.Q * nsc * bolt::kSpecGroups * sizeof(uint16_t));
        }
    }
    L.n_tiles = tiles;
    L.n_queries = queries;
    L.n_samples = samples;
    L.max_rb = max_rb;
    size_t off = 0;
    L.dbs_off = off;
    off += align256(sizeof(DevDb) * (size_t)(n_db > 0 ? n_db : 1));
    L.tiles_off = off;
    off += align256(sizeof(DevTile) * (size_t)(tiles > 0 ? tiles : 1));
    L.queries_off = off;
    off += align256(sizeof(DevQuery) * (size_t)(queries > 0 ? queries : 1));
    L.gthr_off = off;
    off += align256(sizeof(uint32_t) * (size_t)(queries > 0 ? queries : 1));
    L.fail_off = off;
    off += align256(sizeof(uint32_t) * (size_t)(queries > 0 ? queries : 1));
    L.redo_off = off;
    off += align256(sizeof(uint32_t) * (size_t)(queries > 0 ? queries : 1));
    L.lcnt_off = off;
    off += align256(sizeof(uint32_t) * (size_t)(queries > 0 ? queries : 1));
    L.counter_off = off;
    off += 256;
    L.samples_off = off;
    off += align256(sizeof(DevSample) * (size_t)(samples > 0 ? samples : 1));
    L.cand_off = off;
    off += cand;
    L.total = off;
    return L;
}

}  // namespace

struct bolt_batch_plan {
    char *ws = nullptr;
    int64_t n_tiles = 0, n_queries = 0;
    int64_t n_mfma = 0;     // the first n_mfma tiles are matrix-core tiles of M = 16 and 32,
    int64_t n_mfma64 = 0;   // the next n_mfma64 those of M = 64
    int64_t n_samples = 0;
    int64_t max_rb = 0;     // most row blocks of a speculative database (recomputation items per query)
    int32_t rows_per_tile = 0, grid = 0;
    std::vector<char> host;   // staged descriptors (kept until the plan is destroyed)
    DevDb *dbs = nullptr;
    DevTile *tiles = nullptr;
    DevQuery *queries = nullptr;
    uint32_t *gthr = nullptr;
    uint32_t *fail = nullptr;
    uint32_t *redo = nullptr;      // queries listed for the recomputation (count in counter[3])
    uint32_t *lcnt = nullptr;      // dense candidate list counts per query
    uint32_t *counter = nullptr;
    DevSample *samples = nullptr;
};

extern "C" size_t bolt_batch_ws_bytes(const bolt_batch_db *dbs, int32_t n_db, const bolt_batch_tuning *tuning)
{
    int32_t rows, few_max, per_cu;
    if (resolve(tuning, rows, few_max, per_cu) || validate(dbs, n_db))
        return 0;
    return layout_of(dbs, n_db, rows, few_max).total;
}

extern "C" int bolt_batch_plan_create(const bolt_batch_db *dbs, int32_t n_db,
                                      const bolt_batch_tuning *tuning, void *ws, size_t ws_bytes,
                                      void *stream, bolt_batch_plan **plan_out)
{
    using namespace bolt;
    if (!plan_out)
        return fail(BOLT_ERR_INVALID, "plan pointer is null");
    *plan_out = nullptr;
    int32_t rows, few_max, per_cu;
    BOLT_TRY(resolve(tuning, rows, few_max, per_cu));
    BOLT_TRY(validate(dbs, n_db));
    const Layout L = layout_of(dbs, n_db, rows, few_max);
    if (L.n_tiles > INT32_MAX)
        return fail(BOLT_ERR_UNSUPPORTED, "too many tiles");
    if (ws_bytes < L.total || !ws || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "batch workspace of %zu bytes (256-byte aligned) needed", L.total);

    bolt_batch_plan *p = new bolt_batch_plan();
    p->ws = reinterpret_cast<char *>(ws);
    p->n_tiles = L.n_tiles;
    p->n_queries = L.n_queries;
    p->rows_per_tile = rows;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;   // the persistent grid's size only: MI355X has 256 CUs
    p->grid = per_cu * cus;
    p->dbs = reinterpret_cast<DevDb *>(p->ws + L.dbs_off);
    p->tiles = reinterpret_cast<DevTile *>(p->ws + L.tiles_off);
    p->queries = reinterpret_cast<DevQuery *>(p->ws + L.queries_off);
    p->gthr = reinterpret_cast<uint32_t *>(p->ws + L.gthr_off);
    p->fail = reinterpret_cast<uint32_t *>(p->ws + L.fail_off);
    p->redo = reinterpret_cast<uint32_t *>(p->ws + L.redo_off);
    p->lcnt = reinterpret_cast<uint32_t *>(p->ws + L.lcnt_off);
    p->max_rb = L.max_rb;
    p->counter = reinterpret_cast<uint32_t *>(p->ws + L.counter_off);
    p->samples = reinterpret_cast<DevSample *>(p->ws + L.samples_off);
    p->n_samples = L.n_samples;

    std::vector<DevDb> hd(n_db);
    std::vector<DevTile> ht;
    std::vector<double> cost;
    std::vector<DevQuery> hq;
    std::vector<DevSample> hs;
    hs.reserve(L.n_samples);
    ht.reserve(L.n_tiles);
    cost.reserve(L.n_tiles);
    hq.reserve(L.n_queries);
    size_t cand_off = L.cand_off;
    int64_t qbase = 0;
    for (int i = 0; i < n_db; ++i) {
        const bolt_batch_db &d = dbs[i];
        DevDb &o = hd[i];
        std::memset(&o, 0, sizeof(o));
        o.codes = d.codes;
        o.luts = d.luts;
        o.vals = d.vals;
        o.idx = d.idx;
        o.N = d.N;
        o.M = d.M;
        o.Q = d.Q;
        o.k = d.k;
        bolt::Metric mt;
        bolt::decode_metric(d.metric, &mt);   // validated when the plan was made
        o.largest = mt.largest;
        if (d.Q == 0)
            continue;
        o.n_rb = (d.N + rows - 1) / rows;
        o.cand = reinterpret_cast<uint64_t *>(p->ws + cand_off);
        cand_off += align256((size_t)d.Q * o.n_rb * d.k * sizeof(uint64_t));
        o.gthr = p->gthr + qbase;
        o.fail = p->fail + qbase;
        o.lcnt = p->lcnt + qbase;
        qbase += d.Q;
        const int kind = tile_kind(d, few_max);
        const int64_t nsc = spec_chunks(d, kind);
        if (nsc) {
            o.sdist = reinterpret_cast<uint16_t *>(p->ws + cand_off);
            cand_off += align256((size_t)d.Q * nsc * bolt::kSpecGroups * sizeof(uint16_t));
            o.G = nsc * bolt::kSpecGroups;
            o.stride = d.N / nsc;
            o.spec_r = bolt::spec_rank(d.k, (double)(nsc * bolt::kSpecSpan) / (double)d.N);
            for (int q0 = 0; q0 < d.Q; q0 += 32)
                for (int64_t c = 0; c < nsc; ++c)
                    hs.push_back({i, q0, (int32_t)c, 0});
        }
        const int qb = kind == 1 ? d.Q : (kind == 3 ? 32 : (d.M <= 32 ? 16 : 8));
        for (int64_t rb = 0; rb < o.n_rb; ++rb) {
            const int64_t r = std::min<int64_t>(rows, d.N - rb * rows);
            for (int q0 = 0; q0 < d.Q; q0 += qb) {
                DevTile t;
                t.db = i;
                t.kind = kind;
                t.q0 = q0;
                t.nq = std::min(qb, d.Q - q0);
                t.rb = rb;
                ht.push_back(t);
                // grouped and matrix-core tiles pay for a full query block
                // whatever nq is; a matrix-core lookup costs about 1/4 of a
                // grouped one
                const double w = kind == 3 ? 0.25 : 1.0;
                cost.push_back(w * (double)r * d.M * (kind == 1 ? t.nq : qb));
            }
        }
        for (int q = 0; q < d.Q; ++q)
            hq.push_back({i, q});
    }
    // matrix-core tiles of M = 16 and 32, then of M = 64, then the others
    // (a launch each), each family longest first
    auto family = [&](const DevTile &t) { return t.kind != 3 ? 2 : (hd[t.db].M == 64 ? 1 : 0); };
    std::vector<int64_t> order(ht.size());
    for (size_t e = 0; e < order.size(); ++e)
        order[e] = (int64_t)e;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const int fa = family(ht[a]), fb = family(ht[b]);
        return fa != fb ? fa < fb : cost[a] > cost[b];
    });
    p->n_mfma = 0;
    p->n_mfma64 = 0;
    for (const DevTile &t : ht) {
        p->n_mfma += family(t) == 0;
        p->n_mfma64 += family(t) == 1;
    }
    const size_t nb_db = sizeof(DevDb) * hd.size(), nb_t = sizeof(DevTile) * ht.size(),
                 nb_q = sizeof(DevQuery) * hq.size(), nb_s = sizeof(DevSample) * hs.size();
    p->host.resize(nb_db + nb_t + nb_q + nb_s + 1);
    std::memcpy(p->host.data(), hd.data(), nb_db);
    DevTile *st = reinterpret_cast<DevTile *>(p->host.data() + nb_db);
    for (size_t e = 0; e < order.size(); ++e)
        st[e] = ht[order[e]];
    std::memcpy(p->host.data() + nb_db + nb_t, hq.data(), nb_q);
    if (nb_s)
        std::memcpy(p->host.data() + nb_db + nb_t + nb_q, hs.data(), nb_s);
    hipStream_t s = as_stream(stream);
    hipError_t e1 = hipMemcpyAsync(p->dbs, p->host.data(), nb_db, hipMemcpyHostToDevice, s);
    hipError_t e2 = hipMemcpyAsync(p->tiles, p->host.data() + nb_db, nb_t, hipMemcpyHostToDevice, s);
    hipError_t e3 = hipMemcpyAsync(p->queries, p->host.data() + nb_db + nb_t, nb_q, hipMemcpyHostToDevice, s);
    hipError_t e5 = nb_s ? hipMemcpyAsync(p->samples, p->host.data() + nb_db + nb_t + nb_q, nb_s,
                                          hipMemcpyHostToDevice, s)
                         : hipSuccess;
    hipError_t e4 = hipStreamSynchronize(s);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess) {
        delete p;
        return fail(BOLT_ERR_DEVICE, "uploading the batch plan failed");
    }
    *plan_out = p;
    return BOLT_OK;
}

extern "C" int bolt_batch_run(const bolt_batch_plan *p, void *stream)
{
    using namespace bolt;
    if (!p)
        return fail(BOLT_ERR_INVALID, "plan is null");
    if (p->n_queries == 0)
        return BOLT_OK;
    hipStream_t s = as_stream(stream);
    const int64_t nz = p->n_queries;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, p->counter,
                       p->gthr, p->fail, p->lcnt, nz);
    if (p->n_samples > 0) {   // speculative starting bounds
        bolt::ProfScope prof_("batch_spec", s);
        hipLaunchKernelGGL(batch_sample_kernel, dim3((unsigned)p->n_samples), dim3(256), 0, s, p->dbs, p->samples);
        hipLaunchKernelGGL(batch_select_kernel, dim3((unsigned)p->n_queries), dim3(256), 0, s, p->dbs, p->queries,
                           bolt::g_spec_mode == 2 ? 1 : 0);
    }
    {
        bolt::ProfScope prof_("batch_scan", s);
        const int64_t n_mf = p->n_mfma + p->n_mfma64;
        if (p->n_mfma > 0)
            hipLaunchKernelGGL(batch_scan_kernel<1>, dim3((unsigned)p->grid), dim3(256), 0, s, p->dbs, p->tiles,
                               (int32_t)p->n_mfma, (int64_t)p->rows_per_tile, p->counter);
        if (p->n_mfma64 > 0)
            hipLaunchKernelGGL(batch_scan_kernel<2>, dim3((unsigned)p->grid), dim3(256), 0, s, p->dbs,
                               p->tiles + p->n_mfma, (int32_t)p->n_mfma64, (int64_t)p->rows_per_tile,
                               p->counter + 2);
        if (p->n_tiles > n_mf)
            hipLaunchKernelGGL(batch_scan_kernel<0>, dim3((unsigned)p->grid), dim3(256), 0, s, p->dbs,
                               p->tiles + n_mf, (int32_t)(p->n_tiles - n_mf), (int64_t)p->rows_per_tile,
                               p->counter + 1);
    }
    {
        bolt::ProfScope prof_("batch_merge", s);
        hipLaunchKernelGGL(batch_merge_kernel, dim3((unsigned)p->n_queries), dim3(256), 0, s, p->dbs,
                           p->queries, p->counter + 3, p->redo);
    }
    if (p->n_samples > 0) {   // recomputation of failed sampled bounds (none: every workgroup exits at once)
        bolt::ProfScope prof_("batch_redo", s);
        const int64_t items = p->max_rb * p->n_queries;
        hipLaunchKernelGGL(batch_redo_scan_kernel, dim3((unsigned)(items < kRedoGrid ? items : kRedoGrid)),
                           dim3(256), 0, s, p->dbs, p->queries, p->counter + 3, p->redo, p->max_rb,
                           (int64_t)p->rows_per_tile);
        hipLaunchKernelGGL(batch_redo_merge_kernel,
                           dim3((unsigned)(p->n_queries < kRedoMergeGrid ? p->n_queries : kRedoMergeGrid)), dim3(256),
                           0, s, p->dbs, p->queries, p->counter + 3, p->redo);
    }
    return check_launch("bolt_batch_run");
}

extern "C" int bolt_batch_plan_info(const bolt_batch_plan *p, int64_t *n_tiles, int64_t *n_queries,
                                    int32_t *grid)
{
    if (!p)
        return bolt::fail(BOLT_ERR_INVALID, "plan is null");
    if (n_tiles)
        *n_tiles = p->n_tiles;
    if (n_queries)
        *n_queries = p->n_queries;
    if (grid)
        *grid = p->grid;
    return BOLT_OK;
}

extern "C" int bolt_batch_plan_destroy(bolt_batch_plan *p)
{
    delete p;
    return BOLT_OK;
}

// HIP graph of one run: captured on a private stream, replayable on any.
extern "C" int bolt_batch_graph_create(const bolt_batch_plan *p, void **graph_exec)
{
    using namespace bolt;
    if (!p || !graph_exec)
        return fail(BOLT_ERR_INVALID, "null argument");
    *graph_exec = nullptr;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(BOLT_ERR_DEVICE, "stream creation failed");
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    int st = BOLT_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(BOLT_ERR_DEVICE, "hipStreamBeginCapture failed");
    } else {
        const int rs = bolt_batch_run(p, cs);
        const hipError_t ee = hipStreamEndCapture(cs, &g);
        if (rs != BOLT_OK)
            st = rs;
        else if (ee != hipSuccess || !g)
            st = fail(BOLT_ERR_DEVICE, "hipStreamEndCapture failed");
        else if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
            st = fail(BOLT_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    if (g)
        (void)hipGraphDestroy(g);   // cleanup: nothing to do on failure
    (void)hipStreamDestroy(cs);
    if (st == BOLT_OK)
        *graph_exec = ge;
    return st;
}

extern "C" int bolt_batch_graph_launch(void *graph_exec, void *stream)
{
    using namespace bolt;
    if (!graph_exec)
        return fail(BOLT_ERR_INVALID, "graph is null");
    if (hipGraphLaunch(reinterpret_cast<hipGraphExec_t>(graph_exec), as_stream(stream)) != hipSuccess)
        return fail(BOLT_ERR_DEVICE, "hipGraphLaunch failed");
    return BOLT_OK;
}

extern "C" int bolt_batch_graph_destroy(void *graph_exec)
{
    if (graph_exec && hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(graph_exec)) != hipSuccess)
        return bolt::fail(BOLT_ERR_DEVICE, "hipGraphExecDestroy failed");
    return BOLT_OK;
}
