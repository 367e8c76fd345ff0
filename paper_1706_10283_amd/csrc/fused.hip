// Scan fused with top-k selection (Sec. 3.1 scan; Sec. 1.2 the k closest
// vectors) for gfx950: the [Q][N] sums are never written to memory.
//
// Stage 0 (a whole database of 2^16 rows or more): sampled starting bounds.
// A sample launch takes the d of every query over chunks of rows at a
// regular stride on the matrix cores and keeps one minimum per 16 rows; a
// selection launch gives each query the exact r-th smallest of its minima
// as its starting bound.
//
// Stage 1, one workgroup per (row block, query block): the scan computes
// the sums (one or two queries, or up to seven at M = 8 or for k > 128:
// pair tables in LDS; otherwise, with k <= 128, the one-hot codes times the
// tables on the int8 matrix cores; for k > 128: query-interleaved tables in
// LDS); each sum is compared with
// its query's bound and the survivors are appended to that query's LDS
// buffer.  Without sampled bounds the buffers that could overflow are pruned
// between passes and a pruned bound is published to the other workgroups
// with a global atomicMin (any row whose d exceeds a workgroup's k-th
// smallest d cannot be in the global top-k); with them the matrix-core
// passes run with no barriers and no atomics (see tiles.hpp).  The bounds
// only decide which rows are kept as candidates, never the result.  Each
// workgroup finally writes its exact local top-k per query as packed 48-bit
// keys (d << 32 | row) with their count, and counts them into a per-query
// histogram of d.
//
// Stage 2: the merge takes per query the keys at or below the bound the
// histogram gives (the first bin where the count reaches k), in one or two
// levels, keeps the exact k smallest and sorts them.  A query whose sampled
// bound failed (fewer than k candidates, or a tile's buffer overflowed) is
// put on a list instead, and stage 3 recomputes it exactly on the whole GPU,
// so results never depend on the sample, the schedule or the row order.
//
// Stage 3 (with sampled bounds; always launched, its workgroups exit at
// once when the list is empty): every (listed query, tile) pair is scanned
// again from an open bound by a one-query tile, over the workgroups of one
// persistent grid, and the workgroup that finishes a query's last tile
// merges that query's tiles and writes its result.
//
// Workgroups of one row block are placed on one XCD (consecutive workgroup
// ids are dispatched round-robin to the 8 XCDs), so each XCD's L2 holds only
// its share of the codes while all query blocks reuse them.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "scan_common.hpp"
#include "tiles.hpp"

namespace {

using bolt::code_at;
using bolt::load_row;
using bolt::PruneResult;
using bolt::hist_bound;

constexpr int kRowsPerBlock = 16384;      // rows per workgroup (<= 65536: 16-bit local rows)
// Queries from which the matrix-core tiles are used.  A part-filled 32-query
// tile costs about what a full one costs, while the few-query kernel's time
// grows with every query: over 2.5e8 rows the tiles win from three queries
// at M = 16, 32 and 64 (M = 32: 1.7 against 2.1 ms at three queries, 1.9
// against 7.2 ms at seven).  M = 8 keeps the few-query kernel below eight.
constexpr int64_t mfma_min_q(int M) { return M == 8 ? 8 : 3; }
// 32-query tiles per matrix-core workgroup: with one, the tables take half
// the registers of two and four waves per SIMD fit (beside 33 KB of LDS),
// which more than pays for reading the one-hot operand once per instruction
constexpr int kMfmaNT = 1;

// Decode the tile of workgroup `w`: XCD-major placement of row blocks.
__device__ __forceinline__ void tile_of(int w, int n_qb, int &qb, int &rb)
{
    const int xcd = w & 7, i = w >> 3;
    qb = i % n_qb;
    rb = (i / n_qb) * 8 + xcd;
}

// The tile of workgroup w (qb_size queries, rows of row block rb: the
// caller's tile list, or span rows from rb * stride); false if the
// workgroup has no tile (padding of the XCD placement).
__device__ __forceinline__ bool tile_job(int w, int n_qb, int qb_size, const uint8_t *codes, int64_t N,
                                         const uint8_t *luts, int64_t Q, uint32_t k, bolt::RankOrder order, int n_rb,
                                         uint64_t *cand, uint32_t *ccnt, uint32_t *hist, int shift,
                                         uint32_t *fail, uint32_t *gthr, const int64_t *tiles, int64_t stride,
                                         int64_t span, uint32_t *lcnt, bolt::TileJob &job)
{
    int qb, rb;
    tile_of(w, n_qb, qb, rb);
    if (rb >= n_rb)
        return false;
    job.codes = codes;
    job.luts = luts;
    job.cand = cand;
    job.ccnt = ccnt;
    job.hist = hist;
    job.hist_shift = shift;
    job.fail = fail;
    job.lcnt = lcnt;
    job.gthr = gthr;
    if (tiles) {   // row ranges given by the caller, cut into tiles
        job.r0 = tiles[2 * rb];
        job.r1 = tiles[2 * rb + 1];
    } else {
        job.r0 = (int64_t)rb * stride;
        job.r1 = (job.r0 + span) < N ? (job.r0 + span) : N;
    }
    job.rb = rb;
    job.n_rb = n_rb;
    job.q0 = (int64_t)qb * qb_size;
    job.nq = (int)((Q - job.q0) < qb_size ? (Q - job.q0) : qb_size);
    job.k = k;
    job.order = order;
    return true;
}

template <int MM, int NG>
__global__ __launch_bounds__(256) void scan_topk_grouped_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    uint32_t k, bolt::RankOrder order, int n_rb, int n_qb, uint64_t *__restrict__ cand, uint32_t *__restrict__ ccnt,
    uint32_t *__restrict__ hist, uint32_t *__restrict__ fail, uint32_t *__restrict__ gthr,
    const int64_t *__restrict__ tiles, int64_t stride, int64_t span)
{
    __shared__ bolt::GroupedLds<MM, NG> L;
    bolt::TileJob job;
    if (tile_job(blockIdx.x, n_qb, 8 * NG, codes, N, luts, Q, k, order, n_rb, cand, ccnt, hist,
                 bolt::hist_shift(MM), fail, gthr, tiles, stride, span, nullptr, job))
        bolt::grouped_tile<MM, NG>(job, L);
}

// Matrix-core tiles: 32 NT queries per workgroup (tables in registers);
// FREE: barrier-free passes under speculative bounds (see mfma_tile); SP:
// the sparse matrix instruction.
template <int MM, int NT, bool FREE, bool SP>
__global__ __launch_bounds__(256) void scan_topk_mfma_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    uint32_t k, bolt::RankOrder order, int n_rb, int n_qb, uint64_t *__restrict__ cand, uint32_t *__restrict__ ccnt,
    uint32_t *__restrict__ hist, uint32_t *__restrict__ fail, uint32_t *__restrict__ gthr,
    const int64_t *__restrict__ tiles, int64_t stride, int64_t span, uint32_t *__restrict__ lcnt)
{
    __shared__ bolt::MfmaLds<NT> L;
    bolt::TileJob job;
    if (tile_job(blockIdx.x, n_qb, 32 * NT, codes, N, luts, Q, k, order, n_rb, cand, ccnt, hist,
                 bolt::hist_shift(MM), fail, gthr, tiles, stride, span, lcnt, job))
        bolt::mfma_tile<MM, NT, FREE, SP>(job, L);
}

// ------------------------------------------------------------------ merge

// Lists query q for the exact recomputation (stage 3): q is appended to
// redo[2 ...] (redo[0] counts the list), its bound is opened, its histogram
// and dense list emptied for stage 3a, and fail[q] becomes the count of its
// tiles that stage 3a finished.  Every thread of the one workgroup that
// finishes the query's merge calls it, after the workgroup's last read of
// hist[q], lcnt[q] and fail[q].
__device__ void flag_redo(int64_t q, uint32_t *gthr, uint32_t *hist, uint32_t *lcnt, uint32_t *fail,
                          uint32_t *redo)
{
    __syncthreads();
    for (int i = threadIdx.x; i < bolt::kHistBins; i += blockDim.x)
        hist[q * bolt::kHistBins + i] = 0;
    if (threadIdx.x == 0) {
        fail[q] = 0;
        lcnt[q] = 0;
        gthr[q] = 0xFFFFu;
        const uint32_t pos = atomicAdd(&redo[0], 1u);
        redo[2 + pos] = (uint32_t)q;
    }
}


// Appends to L every key below L.mbound from slots [s_lo, s_hi) (slot s:
// cnt[s] keys at src + s * k), pruning to the k smallest whenever the
// buffer could overflow; returns the number of keys held.  The slots are
// taken 256 at a time: an exclusive prefix sum of their counts (pre, 257
// entries of LDS) numbers their keys 0..total-1, and every thread takes
// four of those numbers per round, finding its slot by binary search.
__device__ uint32_t merge_walk(bolt::MergeLds &L, uint32_t *pre, const uint64_t *__restrict__ src,
                               const uint32_t *__restrict__ cnt, int64_t s_lo, int64_t s_hi, uint32_t k)
{
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t c0 = s_lo; c0 < s_hi; c0 += 256) {
        const int ns = (int)((s_hi - c0) < 256 ? (s_hi - c0) : 256);
        uint32_t c = tid < ns ? cnt[c0 + tid] : 0u;
        c = c < k ? c : k;   // a slot never holds more than k keys
        uint32_t inc = c;    // inclusive scan within the wave, then across waves
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o)
                inc += t;
        }
        if (lane == 63)
            wsum[wave] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w)
            before += wsum[w];
        pre[tid] = before + inc - c;
        if (tid == 255)
            pre[256] = before + inc;
        __syncthreads();
        const uint32_t total = pre[256];
        for (uint32_t b0 = 0; b0 < total; b0 += 256 * 4) {
            const uint64_t bnd = L.mbound;
#pragma unroll 1
            for (int e = 0; e < 4; ++e) {
                const uint32_t i = b0 + tid + 256 * e;
                if (i < total) {
                    int lo = 0, hi = ns - 1;   // last slot with pre[slot] <= i
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (pre[mid] <= i)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    const uint64_t key = src[(c0 + lo) * k + (i - pre[lo])];
                    if (key < bnd) {
                        const uint32_t pos = atomicAdd(&L.mcnt, 1u);
                        L.mb[pos] = key;
                    }
                }
            }
            __syncthreads();
            if (tid < 64 && L.mcnt > bolt::kMergeCap - 256 * 4) {
                const uint64_t kth = bolt::prune_u64<bolt::kMergeCap>(L.mb, L.mcnt, k);
                if (tid == 0) {
                    L.mcnt = k;
                    L.mbound = kth + 1;
                }
            }
            __syncthreads();
        }
    }
    return L.mcnt;
}

// Merge, level 1: one workgroup per (query, chunk of the query's tile
// slots).  Keys with d above the bound from the query's candidate histogram
// cannot be in its top-k and are skipped.  With one chunk the workgroup
// writes the sorted values and rows; with several, the chunk's exact k smallest
// survivors go to its slot dst[q][chunk][k] and their number to
// dst_cnt[q][chunk].  No atomics outside LDS: the slots are fixed.  With
// fail (speculative starting bounds), the workgroup that finds fewer than k
// keys for its query, or its overflow flag set, lists the query for the
// exact recomputation (flag_redo) and writes no result.
__global__ __launch_bounds__(256) void topk_merge_kernel(const uint64_t *__restrict__ cand,
                                                         const uint32_t *__restrict__ ccnt, int64_t n_rb,
                                                         int64_t slots_per_chunk, uint32_t k,
                                                         uint32_t *__restrict__ gthr,
                                                         uint32_t *__restrict__ hist, int shift,
                                                         bolt::RankOrder order, uint32_t smax,
                                                         uint64_t *__restrict__ dst,
                                                         uint32_t *__restrict__ dst_cnt,
                                                         uint16_t *__restrict__ vals,
                                                         int32_t *__restrict__ idx, uint32_t *__restrict__ lcnt,
                                                         uint32_t *__restrict__ fail, uint32_t *__restrict__ redo)
{
    __shared__ bolt::MergeLds L;
    __shared__ uint32_t pre[257];
    const int64_t q = blockIdx.x;
    const int64_t s_lo = (int64_t)blockIdx.y * slots_per_chunk;
    const int64_t s_hi = (s_lo + slots_per_chunk) < n_rb ? (s_lo + slots_per_chunk) : n_rb;
    if (threadIdx.x < 64) {
        const uint32_t b = hist_bound(hist + q * bolt::kHistBins, k, shift, gthr[q]);
        if (threadIdx.x == 0) {
            L.mcnt = 0;
            L.mbound = ((uint64_t)b + 1u) << 32;   // keys with d <= b
            // every workgroup of the query stores the same value (for level 2)
            if (blockIdx.y == 0)
                gthr[q] = b;
        }
    }
    __syncthreads();
    uint32_t n = merge_walk(L, pre, cand + q * n_rb * k, ccnt + q * n_rb, s_lo, s_hi, k);
    if (gridDim.y == 1) {
        if (fail && (n < k || fail[q]))
            flag_redo(q, gthr, hist, lcnt, fail, redo);
        else
            bolt::merge_finish(L, n, k, order.largest(q), smax, vals + q * k, idx + q * k);
        return;
    }
    if (threadIdx.x < 64 && n > k)
        bolt::prune_u64_fit<bolt::kMergeCap>(L.mb, n, k);
    __syncthreads();
    n = n > k ? k : n;
    const int64_t slot = q * gridDim.y + blockIdx.y;
    for (uint32_t r = threadIdx.x; r < n; r += 256)
        dst[slot * k + r] = L.mb[r];
    if (threadIdx.x == 0)
        dst_cnt[slot] = n;
}

// Merge, level 2: one workgroup per query gathers the level-1 survivors
// (only the filled part of each slot) and writes the sorted result.
__global__ __launch_bounds__(256) void topk_merge2_kernel(const uint64_t *__restrict__ src,
                                                          const uint32_t *__restrict__ src_cnt, int n_chunks,
                                                          uint32_t k, uint32_t *__restrict__ gthr,
                                                          bolt::RankOrder order, uint32_t smax,
                                                          uint16_t *__restrict__ vals, int32_t *__restrict__ idx,
                                                          uint32_t *__restrict__ hist, uint32_t *__restrict__ lcnt,
                                                          uint32_t *__restrict__ fail, uint32_t *__restrict__ redo)
{
    __shared__ bolt::MergeLds L;
    __shared__ uint32_t pre[257];
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid == 0) {
        L.mcnt = 0;
        L.mbound = ((uint64_t)gthr[q] + 1u) << 32;
    }
    __syncthreads();
    const uint32_t n = merge_walk(L, pre, src + q * (int64_t)n_chunks * k, src_cnt + q * (int64_t)n_chunks, 0,
                                  n_chunks, k);
    if (fail && (n < k || fail[q])) {
        flag_redo(q, gthr, hist, lcnt, fail, redo);
        return;
    }
    bolt::merge_finish(L, n, k, order.largest(q), smax, vals + q * k, idx + q * k);
}

// Merge of the dense candidate lists (sampled bounds on the pair-table and
// matrix-core tiles; one launch, one workgroup per query): the exact k
// smallest of the lcnt[q] keys of cand[q], sorted.  A query with fewer than
// k keys (its sampled bound failed) or whose barrier-free tile overflowed
// is listed for the recomputation.
__global__ __launch_bounds__(256) void topk_list_merge_kernel(const uint64_t *__restrict__ cand,
                                                              uint32_t *__restrict__ lcnt, int64_t per_query,
                                                              uint32_t k, int shift, uint32_t *__restrict__ gthr,
                                                              bolt::RankOrder order,
                                                              uint32_t smax, uint16_t *__restrict__ vals,
                                                              int32_t *__restrict__ idx, uint32_t *__restrict__ hist,
                                                              uint32_t *__restrict__ fail, uint32_t *__restrict__ redo)
{
    __shared__ bolt::MergeLds L;
    __shared__ __attribute__((aligned(16))) uint32_t h[bolt::kHistBins];
    const int64_t q = blockIdx.x;
    const uint32_t c = lcnt[q];
    const int64_t n_keys = (int64_t)c < per_query ? (int64_t)c : per_query;
    const uint32_t n = bolt::merge_collect_list(L, h, cand + q * per_query, n_keys, k, shift, gthr[q], false);
    if (n < k || fail[q])
        flag_redo(q, gthr, hist, lcnt, fail, redo);
    else
        bolt::merge_finish(L, n, k, order.largest(q), smax, vals + q * k, idx + q * k);
}

// Rows [r0, r1) of tile rb: the caller's list, else rpb rows each.
__device__ __forceinline__ void tile_rows(const int64_t *__restrict__ tiles, int64_t rb, int64_t rpb, int64_t N,
                                          int64_t &r0, int64_t &r1)
{
    if (tiles) {
        r0 = tiles[2 * rb];
        r1 = tiles[2 * rb + 1];
    } else {
        r0 = rb * rpb;
        r1 = (r0 + rpb) < N ? (r0 + rpb) : N;
    }
}

// Stage 3: exact recomputation of the listed queries (redo[0] of them, at
// redo[2 ...]) on the whole GPU, in two launches whose workgroups all exit
// at once when the list is empty.
//
// 3a, the scan: item i of the persistent loop is (listed query i / n_rb,
// tile i % n_rb), a one-query tile from the query's open bound that
// publishes its pruned bounds to the query's other tiles, appends its local
// top-k to the query's dense list (cand[q], free since the merge) and adds
// its d histogram to hist[q] (one_query_tile with HIST).  The workgroup
// that finishes the query's last tile (fail[q] counts them) sets gthr[q] to
// the upper edge of the first bin at which the sum reaches k: the query's
// k-th smallest d lies in that bin, so the merge collects the k smallest
// keys and at most that bin's other keys.
template <int MM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void topk_redo_scan_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, uint32_t k, bolt::RankOrder order,
    int64_t n_rb, int64_t rpb, const int64_t *__restrict__ tiles, uint64_t *cand, uint32_t *hist, uint32_t *gthr,
    uint32_t *done, uint32_t *lcnt, const uint32_t *__restrict__ redo)
{
    constexpr size_t kTile = bolt::one_query_lds_bytes(MM);
    __shared__ __attribute__((aligned(16))) char lds[kTile + bolt::kHistBins * sizeof(uint32_t)];
    __shared__ uint32_t s_last;
    uint32_t *hl = reinterpret_cast<uint32_t *>(lds + kTile);
    const int64_t items = (int64_t)redo[0] * n_rb;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t q = redo[2 + it / n_rb];
        int64_t r0, r1;
        tile_rows(tiles, it % n_rb, rpb, N, r0, r1);
        for (int i = threadIdx.x; i < bolt::kHistBins; i += 256)
            hl[i] = 0;   // the tile's first barrier orders these before the counts
        uint32_t *hq = hist + q * bolt::kHistBins;
        bolt::one_query_tile<MM, true>(codes, r0, r1, luts + q * MM * 16, k, order.largest(q), cand + q * n_rb * k,
                                       nullptr, nullptr, gthr + q, lds, lcnt + q, hl, hq);
        // The tile's bins, bound and list went out as device-scope atomics
        // and stores: each wave waits for its own to complete before the
        // tile is counted (a device-scope fence here would also write back
        // the L2, once per tile: a separate histogram pass ran 3.4 times
        // slower with one), and the last workgroup reads hq with atomics.
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0)
            s_last = atomicAdd(&done[q], 1u) == (uint32_t)(n_rb - 1) ? 1u : 0u;
        __syncthreads();
        if (s_last) {
            uint32_t *h = reinterpret_cast<uint32_t *>(lds);
            for (int i = threadIdx.x; i < bolt::kHistBins; i += 256)
                h[i] = atomicAdd(&hq[i], 0u);
            __syncthreads();
            if (threadIdx.x < 64) {
                const uint32_t b = bolt::hist_bound(h, k, bolt::hist_shift(MM), 0xFFFFu);
                if (threadIdx.x == 0) {
                    atomicExch(&gthr[q], b);
                    atomicExch(&done[q], 0u);
                }
                if (threadIdx.x < 3)   // hq[0 .. 2]: the merge's counters (see 3b)
                    atomicExch(&hq[threadIdx.x], 0u);
            }
        }
        __syncthreads();
    }
}

// 3b, the merge.  The list holds every tile's local top-k (up to k keys per
// tile: hundreds of thousands over 2.5e8 rows) and the exact bound admits
// about k of them, so the list is filtered on the whole GPU first.  Item i
// of the persistent loop is (listed query i / n_chunks, chunk i % n_chunks
// of kRedoChunk list keys): the chunk's keys at or below the bound are
// appended, as device-scope atomic stores, to an area of at most kMergeCap
// keys past the list's end in the query's candidate region (hq[0] counts
// them, hq[2] flags a chunk with more than kMergeCap); the workgroup that
// finishes the query's last chunk (hq[1] counts them) reads the area back
// with atomics and writes the sorted top k.  If the area overflowed (keys
// massively tied at the bound) that workgroup collects from the whole list
// instead.  hq: the query's histogram words, free since 3a.
constexpr int64_t kRedoChunk = 16384;

__global__ __launch_bounds__(256) void topk_redo_merge_kernel(uint64_t *cand, const uint32_t *__restrict__ lcnt,
                                                              int64_t n_rb, uint32_t k,
                                                              const uint32_t *__restrict__ gthr, bolt::RankOrder order,
                                                              uint32_t smax, uint32_t *hist,
                                                              const uint32_t *__restrict__ redo,
                                                              uint16_t *__restrict__ vals, int32_t *__restrict__ idx)
{
    __shared__ bolt::MergeLds L;
    __shared__ uint32_t s_n, s_at, s_last;
    const int tid = threadIdx.x;
    const int64_t per_query = n_rb * k;
    const int64_t n_chunks = (per_query + kRedoChunk - 1) / kRedoChunk;
    const int64_t items = (int64_t)redo[0] * n_chunks;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int64_t q = redo[2 + it / n_chunks];
        uint64_t *list = cand + q * per_query;
        const int64_t c = lcnt[q];
        const int64_t n_keys = c < per_query ? c : per_query;
        const int64_t room = per_query - n_keys;
        const int64_t cap = room < bolt::kMergeCap ? room : bolt::kMergeCap;
        unsigned long long *area = reinterpret_cast<unsigned long long *>(list + per_query - cap);
        uint32_t *hq = hist + q * bolt::kHistBins;
        const uint64_t bnd = ((uint64_t)gthr[q] + 1u) << 32;
        const int64_t lo = (it % n_chunks) * kRedoChunk;
        const int64_t hi = (lo + kRedoChunk) < n_keys ? (lo + kRedoChunk) : n_keys;
        if (tid == 0)
            s_n = 0;
        __syncthreads();
        constexpr int B = 8;   // keys per thread in flight
        for (int64_t i0 = lo; i0 < hi; i0 += 256 * B) {
            uint64_t kk[B];
#pragma unroll
            for (int e = 0; e < B; ++e) {
                const int64_t i = i0 + tid + 256 * e;
                kk[e] = i < hi ? list[i] : ~0ull;
            }
#pragma unroll
            for (int e = 0; e < B; ++e)
                if (kk[e] < bnd) {
                    const uint32_t pos = atomicAdd(&s_n, 1u);
                    if (pos < (uint32_t)bolt::kMergeCap)
                        L.mb[pos] = kk[e];
                }
        }
        __syncthreads();
        const uint32_t n = s_n;
        if (tid == 0 && n > 0) {
            if (n > (uint32_t)bolt::kMergeCap)
                atomicOr(&hq[2], 1u);
            else
                s_at = atomicAdd(&hq[0], n);
        }
        __syncthreads();
        if (n <= (uint32_t)bolt::kMergeCap)
            for (uint32_t r = tid; r < n; r += 256)
                if ((int64_t)s_at + r < cap)
                    atomicExch(&area[s_at + r], (unsigned long long)L.mb[r]);
        // the area's stores complete before the chunk is counted (as in 3a)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0)
            s_last = atomicAdd(&hq[1], 1u) == (uint32_t)(n_chunks - 1) ? 1u : 0u;
        __syncthreads();
        if (s_last) {
            const uint32_t total = atomicAdd(&hq[0], 0u);
            const bool whole = atomicOr(&hq[2], 0u) != 0u || (int64_t)total > cap;
            uint32_t m;
            if (whole) {
                m = bolt::merge_collect_wide(L, list, n_keys, k, gthr[q]);
            } else {
                for (uint32_t r = tid; r < total; r += 256)
                    L.mb[r] = atomicAdd(&area[r], 0ull);
                __syncthreads();
                m = total;
            }
            bolt::merge_finish(L, m, k, order.largest(q), smax, vals + q * k, idx + q * k);
        }
        __syncthreads();
    }
}

// Result padding when no row is scanned (n results, k per query): 65535 / 0
// and index -1.
__global__ void pad_topk_kernel(uint16_t *vals, int32_t *idx, int64_t n, int64_t k, bolt::RankOrder order)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        vals[i] = (uint16_t)(order.largest(i / k) ? 0u : 0xFFFFu);
        idx[i] = -1;
    }
}

// Bounds start open (65535: every d passes) and histograms empty.
__global__ void init_bounds_kernel(uint32_t *gthr, int64_t Q, uint32_t *hist, int64_t n_hist)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < Q)
        gthr[i] = 0xFFFFu;
    if (i < n_hist)
        hist[i] = 0;
}

// Histogram of the d values of the candidate keys: one workgroup per
// (query, 256 tile slots), one slot per thread; counted in LDS, nonzero bins
// added to the query's global histogram.  Used when the tiles do not count
// their keys themselves: without speculative bounds a query may receive up
// to k keys from each of thousands of tiles, all in a few bins, and global
// atomics on one address serialise.
__global__ __launch_bounds__(256) void cand_hist_kernel(const uint64_t *__restrict__ cand,
                                                        const uint32_t *__restrict__ ccnt, int64_t n_rb, uint32_t k,
                                                        int shift, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[bolt::kHistBins];
    for (int i = threadIdx.x; i < bolt::kHistBins; i += 256)
        h[i] = 0;
    __syncthreads();
    const int64_t q = blockIdx.x;
    const int64_t slot = (int64_t)blockIdx.y * 256 + threadIdx.x;
    if (slot < n_rb) {
        uint32_t m = ccnt[q * n_rb + slot];
        m = m < k ? m : k;
        const uint64_t *c = cand + (q * n_rb + slot) * k;
        for (uint32_t j = 0; j < m; ++j)
            atomicAdd(&h[(uint32_t)(c[j] >> 32) >> shift], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bolt::kHistBins; i += 256)
        if (h[i])
            atomicAdd(&hist[q * bolt::kHistBins + i], h[i]);
}

// Sample (speculative bounds): workgroup (query block, chunk c) writes the
// group minima of its queries over rows [c * stride, c * stride + kSpecSpan)
// to out[q][c * kSpecGroups ...] (G entries per query).
template <int MM, int NT, bool SP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void spec_sample_kernel(
    const uint8_t *__restrict__ codes, const uint8_t *__restrict__ luts, int64_t Q, bolt::RankOrder order,
    int64_t stride, int64_t G, uint16_t *__restrict__ out)
{
    __shared__ bolt::OneHot onehot;
    __shared__ __attribute__((aligned(16))) uint16_t gmin[32 * NT * bolt::kSpecGminStride];
    const int64_t q0 = (int64_t)blockIdx.x * 32 * NT;
    const int nq = (int)((Q - q0) < 32 * NT ? (Q - q0) : 32 * NT);
    const int64_t c = blockIdx.y;
    bolt::mfma_sample_tile<MM, NT, SP>(codes, luts, q0, nq, order, c * stride, out, G, c * bolt::kSpecGroups, onehot,
                                   gmin);
}

// Speculative bound of one query (one workgroup): the r-th smallest of its
// G sample group minima (r distinct sample rows lie at or below it), written
// as the query's starting bound (0 when a test forces every query onto the
// recomputation).  Also clears the query's overflow flag and candidate
// histogram (or, for dense candidate lists, the list's count) and the
// recomputation list (this kernel replaces the initialisation when the
// bounds are speculative).
__global__ __launch_bounds__(256) void spec_select_kernel(const uint16_t *__restrict__ gmins, int64_t G,
                                                          uint32_t r, int shift, uint32_t *__restrict__ gthr,
                                                          uint32_t *__restrict__ hist, uint32_t *__restrict__ fail,
                                                          uint32_t *__restrict__ redo, uint32_t *__restrict__ lcnt,
                                                          int force_fail)
{
    __shared__ __attribute__((aligned(16))) uint32_t h[bolt::kHistBins];
    const int64_t q = blockIdx.x;
    if (q == 0 && threadIdx.x == 0)
        redo[0] = 0u;   // the recomputation list starts empty
    if (!lcnt)   // dense candidate lists need no histogram
        for (int i = threadIdx.x; i < bolt::kHistBins; i += 256)
            hist[q * bolt::kHistBins + i] = 0;
    const uint32_t b = bolt::select_rank_u16(gmins + q * G, G, r, shift, h);
    if (threadIdx.x == 0) {
        gthr[q] = force_fail ? 0u : b;
        fail[q] = 0u;
        if (lcnt)
            lcnt[q] = 0u;
    }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Query groups per grouped tile: tables (NG * M * 256 bytes) and candidate
// buffers (NG * 8 * 512 * 4 bytes) within about 48 KB, three workgroups per CU.
template <int MM>
constexpr int ng_for()
{
    return MM <= 32 ? 2 : 1;
}

// Speculative bounds (many queries, one whole database).  The r-th smallest
// d over a sample of S rows (chunks of kSpecSpan rows at a regular stride)
// bounds the k-th smallest d of the database unless r of the database's k
// smallest rows fall in the sample; for a random row order that number is
// binomial(k, S / N), and r is the smallest rank whose tail is below 1e-7
// (r = k: the bound is certain).  The sample's distances come from the
// matrix cores (whatever kernel scans) and are kept as one minimum per group
// of kSpecGroup sample rows: the r-th smallest group minimum still has r
// distinct sample rows at or below it, so the same tail bounds it, and for
// small r it rarely differs from the r-th smallest distance.  It is found
// exactly: a histogram locates its bin, a second count that bin's values.
// The bound only selects candidates: the
// final merge lists any query with fewer than k candidates and
// stage 3 recomputes it exactly, so results never depend on it.
using bolt::kSpecSpan;
using bolt::kSpecMinRows;
using bolt::kSpecMinRowsForced;
using bolt::kSpecMaxDists;

struct FusedPlan {
    bool ok = false;
    int kind = 0;        // 1 few-query, 2 grouped, 3 matrix cores
    int n_rb = 0, n_qb = 0, qb_size = 0, n_chunks = 1;
    int64_t rpb = 0;     // rows per tile
    int64_t chunk = 0;   // tile slots per first-level merge workgroup
    size_t cand_bytes = 0, ccnt_bytes = 0, gthr_bytes = 0, hist_bytes = 0, level2_bytes = 0;
    bool spec = false;   // speculative bound from a sample
    int spec_r = 0, spec_nsc = 0;
    int64_t spec_stride = 0;
    size_t spec_bytes = 0;   // sample group minima [Q][nsc * kSpecGroups] uint16, overflow flags [Q]
    size_t redo_bytes = 0;   // recomputation list: count, spare, queries [Q] (uint32)
};

// The kernel for the shape and its rows per tile (N: rows to scan).
bool plan_kind(int64_t N, int M, int64_t Q, int k, bool vec_ok, FusedPlan &p)
{
    const bool tuned_M = (M == 8 || M == 16 || M == 32 || M == 64);
    if (!tuned_M || !vec_ok || k > 256 || N <= 0 || Q <= 0)
        return false;
    const int force = bolt::g_force_fused_kind;
    const bool mfma_ok = k <= bolt::kMfmaCap - bolt::kMfmaPass;
    if (force != 3 && Q < bolt::kSmallQ && bolt::few_fused_lds_bytes(M, (int)Q) <= 160 * 1024 &&
        (Q < mfma_min_q(M) || !mfma_ok || force == 2)) {
        p.rpb = bolt::few_rows_per_block(N, M, (int)Q);
        p.kind = 1;
        p.n_qb = 1;
        p.qb_size = (int)Q;
    } else {
        p.rpb = kRowsPerBlock;
        if (mfma_ok && (force == 3 || (force != 2 && Q >= mfma_min_q(M)))) {
            p.kind = 3;
            p.qb_size = 32 * kMfmaNT;
        } else {
            p.kind = 2;
            p.qb_size = 8 * (M <= 32 ? 2 : 1);
        }
        p.n_qb = (int)((Q + p.qb_size - 1) / p.qb_size);
    }
    return true;
}

// Speculation for a whole-database plan (any kind: with one or a few
// queries the tiles would otherwise start without a bound and append a
// fraction of every tile's rows): about N / 32 sample rows (16 to 256
// chunks), fewer if Q of them would not fit kSpecMaxDists.
static void plan_spec(FusedPlan &p, int64_t N, int64_t Q, int k)
{
    const int mode = bolt::g_spec_mode;
    if (p.kind < 1 || mode == 0 || N < (mode > 0 ? kSpecMinRowsForced : kSpecMinRows))
        return;
    int64_t nsc = N / 32 / kSpecSpan;
    nsc = nsc < 16 ? 16 : (nsc > 256 ? 256 : nsc);
    while (nsc > 16 && Q * nsc * kSpecSpan > kSpecMaxDists)
        nsc /= 2;
    if (Q * nsc * kSpecSpan > kSpecMaxDists)
        return;
    const int r = bolt::spec_rank(k, (double)(nsc * kSpecSpan) / (double)N);
    p.spec = true;
    p.spec_r = r;
    p.spec_nsc = (int)nsc;
    p.spec_stride = N / nsc;
}

// Workspace layout once the number of tiles p.n_rb is known.
FusedPlan plan_finish(FusedPlan p, int64_t Q, int k)
{
    if (p.kind >= 2 && (int64_t)p.n_qb * ((p.n_rb + 7) / 8) * 8 > INT32_MAX)
        return p;
    p.cand_bytes = align256((size_t)Q * p.n_rb * k * sizeof(uint64_t));
    p.ccnt_bytes = align256((size_t)Q * p.n_rb * sizeof(uint32_t));
    p.gthr_bytes = align256((size_t)Q * sizeof(uint32_t));
    p.hist_bytes = align256((size_t)Q * bolt::kHistBins * sizeof(uint32_t));
    // first-level merge chunks: enough workgroups to fill the GPU, 32..256 slots each
    int64_t chunk = (int64_t)p.n_rb * Q / 512;
    chunk = chunk < 32 ? 32 : (chunk > 256 ? 256 : chunk);
    p.chunk = chunk;
    p.n_chunks = p.n_rb > chunk ? (int)((p.n_rb + chunk - 1) / chunk) : 1;
    p.level2_bytes = p.n_chunks > 1 ? align256((size_t)Q * p.n_chunks * k * sizeof(uint64_t)) +
                                          align256((size_t)Q * p.n_chunks * sizeof(uint32_t))
                                    : 0;
    if (p.n_chunks > 65535)
        return p;
    // sample minima, overflow flags and dense list counts (the pair-table
    // and matrix-core tiles' lists, and the recomputation's)
    p.spec_bytes = p.spec ? align256((size_t)Q * p.spec_nsc * bolt::kSpecGroups * sizeof(uint16_t)) +
                                align256((size_t)Q * sizeof(uint32_t)) * 2
                          : 0;
    p.redo_bytes = p.spec ? align256((size_t)(Q + 2) * sizeof(uint32_t)) : 0;
    p.ok = true;
    return p;
}

FusedPlan plan_fused(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    FusedPlan p;
    if (!plan_kind(N, M, Q, k, vec_ok, p))
        return p;
    p.n_rb = (int)((N + p.rpb - 1) / p.rpb);
    plan_spec(p, N, Q, k);
    return plan_finish(p, Q, k);
}

// One scan + candidate launch of the planned kind: n_rb tiles of the caller's
// list, or of span rows every stride rows; k candidates per tile and query.
template <int MM>
void launch_scan(const FusedPlan &p, const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q, int k,
                 bolt::RankOrder order, int n_rb, uint64_t *cand, uint32_t *ccnt, uint32_t *hist, uint32_t *fail,
                 uint32_t *gthr, const int64_t *tiles, int64_t stride, int64_t span, uint32_t *lcnt,
                 const char *prof_name, hipStream_t s)
{
    if (p.kind == 1) {   // profiled inside under its own name
        bolt::few_scan_topk(codes, N, MM, luts, Q, k, order, n_rb, cand, ccnt, hist, gthr, tiles, lcnt, s);
        return;
    }
    const unsigned grid = (unsigned)(p.n_qb * ((n_rb + 7) / 8 * 8));
    bolt::ProfScope prof_(prof_name, s);
#define BOLT_MFMA_SCAN(FREE, SP)                                                                                  \
    hipLaunchKernelGGL((scan_topk_mfma_kernel<MM, kMfmaNT, FREE, SP>), dim3(grid), dim3(256), 0, s, codes, N,    \
                       luts, Q, (uint32_t)k, order, n_rb, p.n_qb, cand, ccnt, hist, fail, gthr, tiles, stride, \
                       span, FREE ? lcnt : nullptr)
    const bool sp = bolt::g_sparse_mfma != 0;
    if (p.kind == 3 && p.spec && sp)
        BOLT_MFMA_SCAN(true, true);
    else if (p.kind == 3 && p.spec)
        BOLT_MFMA_SCAN(true, false);
    else if (p.kind == 3 && sp)
        BOLT_MFMA_SCAN(false, true);
    else if (p.kind == 3)
        BOLT_MFMA_SCAN(false, false);
#undef BOLT_MFMA_SCAN
    else
        hipLaunchKernelGGL((scan_topk_grouped_kernel<MM, ng_for<MM>()>), dim3(grid), dim3(256), 0, s, codes, N,
                           luts, Q, (uint32_t)k, order, n_rb, p.n_qb, cand, ccnt, hist, fail, gthr, tiles,
                           stride, span);
}

void launch_scan_m(int M, const FusedPlan &p, const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q,
                   int k, bolt::RankOrder order, int n_rb, uint64_t *cand, uint32_t *ccnt, uint32_t *hist,
                   uint32_t *fail, uint32_t *gthr, const int64_t *tiles, int64_t stride, int64_t span,
                   uint32_t *lcnt,
                   const char *prof_name, hipStream_t s)
{
#define BOLT_SCAN_M(MMV)                                                                                         \
    launch_scan<MMV>(p, codes, N, luts, Q, k, order, n_rb, cand, ccnt, hist, fail, gthr, tiles, stride, span,  \
                     lcnt, prof_name, s)
    switch (M) {
    case 8: BOLT_SCAN_M(8); break;
    case 16: BOLT_SCAN_M(16); break;
    case 32: BOLT_SCAN_M(32); break;
    case 64: BOLT_SCAN_M(64); break;
    }
#undef BOLT_SCAN_M
}

void launch_spec_sample(int M, const uint8_t *codes, const uint8_t *luts, int64_t Q, bolt::RankOrder order,
                        int64_t stride, int64_t G, int nsc, uint16_t *out, hipStream_t s)
{
    const int nt = kMfmaNT;
    const dim3 grid((unsigned)((Q + 32 * nt - 1) / (32 * nt)), (unsigned)nsc);
#define BOLT_SAMPLE_M(MM)                                                                                           \
    if (bolt::g_sparse_mfma)                                                                                        \
        hipLaunchKernelGGL((spec_sample_kernel<MM, kMfmaNT, true>), grid, dim3(256), 0, s, codes, luts, Q, order, \
                           stride, G, out);                                                                         \
    else                                                                                                            \
        hipLaunchKernelGGL((spec_sample_kernel<MM, kMfmaNT, false>), grid, dim3(256), 0, s, codes, luts, Q, order,\
                           stride, G, out)
    switch (M) {
    case 8: BOLT_SAMPLE_M(8); break;
    case 16: BOLT_SAMPLE_M(16); break;
    case 32: BOLT_SAMPLE_M(32); break;
    case 64: BOLT_SAMPLE_M(64); break;
    }
#undef BOLT_SAMPLE_M
}

// Stage 3 launches: persistent grids of at most kRedoGrid scan and
// kRedoMergeGrid merge workgroups (the list's length is known only on the
// device).
constexpr int64_t kRedoGrid = 1024;
constexpr int64_t kRedoMergeGrid = 256;

void launch_redo(int M, const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q, int k, bolt::RankOrder order,
                 const FusedPlan &p, const int64_t *tiles, uint64_t *cand, uint32_t *gthr, uint32_t *hist,
                 uint32_t *fail, uint32_t *lcnt, const uint32_t *redo, uint16_t *vals, int32_t *idx, hipStream_t s)
{
    const int64_t items = (int64_t)p.n_rb * Q;
    const dim3 grid((unsigned)(items < kRedoGrid ? items : kRedoGrid));
#define BOLT_REDO_M(MM)                                                                                          \
    hipLaunchKernelGGL(topk_redo_scan_kernel<MM>, grid, dim3(256), 0, s, codes, N, luts, (uint32_t)k, order,   \
                       (int64_t)p.n_rb, p.rpb, tiles, cand, hist, gthr, fail, lcnt, redo)
    switch (M) {
    case 8: BOLT_REDO_M(8); break;
    case 16: BOLT_REDO_M(16); break;
    case 32: BOLT_REDO_M(32); break;
    case 64: BOLT_REDO_M(64); break;
    }
#undef BOLT_REDO_M
    const int64_t merge_items = Q * (((int64_t)p.n_rb * k + kRedoChunk - 1) / kRedoChunk);
    hipLaunchKernelGGL(topk_redo_merge_kernel,
                       dim3((unsigned)(merge_items < kRedoMergeGrid ? merge_items : kRedoMergeGrid)), dim3(256), 0, s,
                       cand, lcnt, (int64_t)p.n_rb, (uint32_t)k, gthr, order, 255u * (uint32_t)M, hist, redo, vals,
                       idx);
}

const char *scan_prof_name(int kind)
{
    return kind == 1 ? "scan_topk_few" : (kind == 3 ? "scan_topk_mfma" : "scan_topk_grouped");
}

}  // namespace

namespace bolt {

// Smallest r with P(binomial(k, p) >= r) <= 1e-7, at most k.
int spec_rank(int k, double pr)
{
    std::vector<double> pmf(k + 1);
    double tail = 0.0;
    // pmf by the recurrence from j = 0 (pr < 1/16 here, so (1 - pr)^k > 0)
    pmf[0] = std::pow(1.0 - pr, k);
    for (int j = 1; j <= k; ++j)
        pmf[j] = pmf[j - 1] * (double)(k - j + 1) / (double)j * pr / (1.0 - pr);
    int r = k;
    for (int j = k; j >= 1; --j) {
        tail += pmf[j];
        if (tail > 1e-7)
            break;
        r = j;
    }
    return r;
}

bool fused_supported(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    return plan_fused(N, M, Q, k, vec_ok).ok;
}

static size_t plan_bytes(const FusedPlan &p)
{
    return p.cand_bytes + p.ccnt_bytes + p.gthr_bytes + p.hist_bytes + p.level2_bytes + p.spec_bytes +
           p.redo_bytes;
}

bool fused_on_matrix_cores(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    const FusedPlan p = plan_fused(N, M, Q, k, vec_ok);
    return p.ok && p.kind == 3;
}

size_t fused_ws_bytes(int64_t N, int M, int64_t Q, int k)
{
    FusedPlan p = plan_fused(N, M, Q, k, true);
    if (!p.ok)
        return 0;
    return plan_bytes(p);
}

// Launches of a planned fused scan + top-k (tiles: null, or the caller's
// row ranges cut into p.n_rb tiles, already in device memory).
static int run_fused(const FusedPlan &p, const uint8_t *codes, int64_t N, int M, const uint8_t *luts,
                     int64_t Q, int k, bolt::RankOrder order, uint16_t *vals, int32_t *idx, char *w,
                     const int64_t *tiles, hipStream_t s)
{
    uint64_t *cand = reinterpret_cast<uint64_t *>(w);
    w += p.cand_bytes;
    uint32_t *ccnt = reinterpret_cast<uint32_t *>(w);
    w += p.ccnt_bytes;
    uint32_t *gthr = reinterpret_cast<uint32_t *>(w);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + p.gthr_bytes);
    uint64_t *level2 = reinterpret_cast<uint64_t *>(w + p.gthr_bytes + p.hist_bytes);
    uint32_t *level2_cnt = reinterpret_cast<uint32_t *>(w + p.gthr_bytes + p.hist_bytes +
                                                        align256((size_t)Q * p.n_chunks * k * sizeof(uint64_t)));
    char *ws_spec = w + p.gthr_bytes + p.hist_bytes + p.level2_bytes;
    const int64_t G = (int64_t)p.spec_nsc * bolt::kSpecGroups;
    uint16_t *gmins = p.spec ? reinterpret_cast<uint16_t *>(ws_spec) : nullptr;
    uint32_t *fail = p.spec ? reinterpret_cast<uint32_t *>(ws_spec + align256((size_t)Q * G * sizeof(uint16_t)))
                            : nullptr;
    uint32_t *redo = p.spec ? reinterpret_cast<uint32_t *>(ws_spec + p.spec_bytes) : nullptr;
    // sampled bounds on the pair-table and matrix-core tiles: dense
    // per-query candidate lists
    const bool lists = p.spec && p.kind != 2;
    uint32_t *lcnt_all = p.spec ? fail + align256((size_t)Q * sizeof(uint32_t)) / sizeof(uint32_t) : nullptr;
    uint32_t *lcnt = lists ? lcnt_all : nullptr;
    if (p.spec) {
        // sample group minima, then each query's starting bound (and cleared histogram)
        {
            bolt::ProfScope prof_("spec_sample", s);
            launch_spec_sample(M, codes, luts, Q, order, p.spec_stride, G, p.spec_nsc, gmins, s);
        }
        bolt::ProfScope prof_("spec_select", s);
        hipLaunchKernelGGL(spec_select_kernel, dim3((unsigned)Q), dim3(256), 0, s, gmins, G, (uint32_t)p.spec_r,
                           bolt::hist_shift(M), gthr, hist, fail, redo, lcnt, bolt::g_spec_mode == 2 ? 1 : 0);
    } else {
        const int64_t n_hist = Q * bolt::kHistBins;
        hipLaunchKernelGGL(init_bounds_kernel, dim3((unsigned)((n_hist + 255) / 256)), dim3(256), 0, s, gthr, Q,
                           hist, n_hist);
    }
    // with speculative bounds (a few keys per tile and query) the tiles count
    // their kept keys into hist as they write them; otherwise a separate
    // kernel aggregates the counts per workgroup first
    launch_scan_m(M, p, codes, N, luts, Q, k, order, p.n_rb, cand, ccnt, p.spec && !lists ? hist : nullptr,
                  fail, gthr, tiles, kRowsPerBlock, kRowsPerBlock, lcnt, scan_prof_name(p.kind), s);
    if (!p.spec) {
        bolt::ProfScope prof_("cand_hist", s);
        hipLaunchKernelGGL(cand_hist_kernel, dim3((unsigned)Q, (unsigned)((p.n_rb + 255) / 256)), dim3(256), 0, s,
                           cand, ccnt, (int64_t)p.n_rb, (uint32_t)k, bolt::hist_shift(M), hist);
    }
    const uint32_t smax = 255u * (uint32_t)M;
    if (lists) {
        bolt::ProfScope prof_("topk_merge", s);
        hipLaunchKernelGGL(topk_list_merge_kernel, dim3((unsigned)Q), dim3(256), 0, s, cand, lcnt,
                           (int64_t)p.n_rb * k, (uint32_t)k, bolt::hist_shift(M), gthr, order, smax, vals, idx,
                           hist, fail, redo);
    } else {
        bolt::ProfScope prof_("topk_merge", s);
        hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)Q, (unsigned)p.n_chunks), dim3(256), 0, s, cand, ccnt,
                           (int64_t)p.n_rb, p.n_chunks > 1 ? p.chunk : (int64_t)p.n_rb, (uint32_t)k, gthr, hist,
                           bolt::hist_shift(M), order, smax, level2, level2_cnt, vals, idx, lcnt_all, fail,
                           redo);
        if (p.n_chunks > 1)
            hipLaunchKernelGGL(topk_merge2_kernel, dim3((unsigned)Q), dim3(256), 0, s, level2, level2_cnt,
                               p.n_chunks, (uint32_t)k, gthr, order, smax, vals, idx, hist, lcnt_all, fail,
                               redo);
    }
    if (p.spec) {
        bolt::ProfScope prof_("topk_redo", s);
        launch_redo(M, codes, N, luts, Q, k, order, p, tiles, cand, gthr, hist, fail, lcnt_all, redo, vals,
                    idx, s);
    }
    return check_launch("bolt_scan_topk (fused)");
}


// Fused scan + top-k; returns BOLT_ERR_UNSUPPORTED when the shape has no fused kernel.
int scan_topk_fused(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                    bolt::RankOrder order, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes, hipStream_t s)
{
    const bool vec_ok = aligned(codes, 16) && aligned(luts, 16);
    FusedPlan p = plan_fused(N, M, Q, k, vec_ok);
    if (!p.ok)
        return BOLT_ERR_UNSUPPORTED;
    const size_t need = plan_bytes(p);
    if (ws_bytes < need || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "fused scan+top-k needs %zu workspace bytes", need);
    return run_fused(p, codes, N, M, luts, Q, k, order, vals, idx, reinterpret_cast<char *>(ws), nullptr, s);
}

// Row ranges: the tiles of [start, end) ranges of at most p.rpb rows each.
static void range_tiles(const int64_t *ranges, int n_ranges, int64_t rpb, std::vector<int64_t> &tiles)
{
    tiles.clear();
    for (int r = 0; r < n_ranges; ++r)
        for (int64_t a = ranges[2 * r]; a < ranges[2 * r + 1]; a += rpb) {
            tiles.push_back(a);
            tiles.push_back(a + rpb < ranges[2 * r + 1] ? a + rpb : ranges[2 * r + 1]);
        }
}

// Plan of a ranges call (p.ok false: no fused kernel for the shape).
static FusedPlan plan_ranges(const int64_t *ranges, int n_ranges, int M, int64_t Q, int k, bool vec_ok,
                             std::vector<int64_t> &tiles, size_t *tiles_bytes)
{
    FusedPlan p;
    int64_t rows = 0;
    for (int r = 0; r < n_ranges; ++r)
        rows += ranges[2 * r + 1] - ranges[2 * r];
    if (!plan_kind(rows > 0 ? rows : 1, M, Q, k, vec_ok, p))
        return p;
    range_tiles(ranges, n_ranges, p.rpb, tiles);
    p.n_rb = (int)(tiles.size() / 2);
    if (p.n_rb == 0)
        return p;
    *tiles_bytes = align256(tiles.size() * sizeof(int64_t));
    return plan_finish(p, Q, k);
}

size_t ranges_ws_bytes(const int64_t *ranges, int n_ranges, int M, int64_t Q, int k)
{
    std::vector<int64_t> tiles;
    size_t tb = 0;
    FusedPlan p = plan_ranges(ranges, n_ranges, M, Q, k, true, tiles, &tb);
    return p.ok ? plan_bytes(p) + tb : 0;
}

int scan_topk_ranges(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                     bool largest, const int64_t *ranges, int n_ranges, uint16_t *vals, int32_t *idx, void *ws,
                     size_t ws_bytes, hipStream_t s)
{
    const bool vec_ok = aligned(codes, 16) && aligned(luts, 16);
    std::vector<int64_t> tiles;
    size_t tb = 0;
    FusedPlan p = plan_ranges(ranges, n_ranges, M, Q, k, vec_ok, tiles, &tb);
    if (p.n_rb == 0 && p.kind != 0) {
        // no rows at all: the padding of an empty database
        hipLaunchKernelGGL(pad_topk_kernel, dim3((unsigned)((Q * k + 255) / 256)), dim3(256), 0, s, vals, idx,
                           Q * k, (int64_t)k, bolt::one_order(largest));
        return check_launch("bolt_scan_topk_ranges");
    }
    if (!p.ok)
        return fail(BOLT_ERR_UNSUPPORTED, "row-range scans need M in {8, 16, 32, 64}, k <= 256 and 16-byte "
                                          "aligned codes and tables");
    const size_t need = plan_bytes(p) + tb;
    if (ws_bytes < need || !ws || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "row-range scan needs %zu workspace bytes", need);
    char *w = reinterpret_cast<char *>(ws);
    int64_t *dtiles = reinterpret_cast<int64_t *>(w + plan_bytes(p));
    if (hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(int64_t), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return check_launch("bolt_scan_topk_ranges (tile list)");
    return run_fused(p, codes, N, M, luts, Q, k, bolt::one_order(largest), vals, idx, w, dtiles, s);
}

}  // namespace bolt
