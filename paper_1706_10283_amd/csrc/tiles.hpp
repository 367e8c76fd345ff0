// Tile processors of the fused scan + top-k (Sec. 3.1 scan; Sec. 1.2 the k
// closest vectors), shared by the one-database kernels and the persistent
// many-database kernel.
//
// A tile is (query range of one database, row range of at most 65536 rows).
// Its workgroup computes the sums of every (query, row) pair, keeps the rows
// whose d passes the query's bound in an LDS candidate buffer (see
// topk_device.hpp), and finally writes the tile's exact local top-k of every
// query as 48-bit keys (d << 32 | row) to cand[q][rb][k].  d is the sum (k
// smallest) or 255*M - sum (k largest), so that d <= 65280 and every bound
// fits in 16 bits.  Bounds are published to, and refreshed from, the
// database's per-query global bounds gthr with atomicMin: a tile that holds k
// or more rows with d <= T proves that no row with d > T is in the top-k.
// The bounds only decide which rows become candidates, so results are exact
// and independent of timing.
#pragma once

#include "common.hpp"
#include "scan_common.hpp"
#include "topk_device.hpp"

namespace bolt {

constexpr int kTileRowsMax = 65536;   // 16-bit local rows

// Grouped tiles (8 queries per group as uint16 lanes; see scan.hip).
constexpr int kGroupedCap = 512;      // candidate slots per query
constexpr int kRefresh = 8;           // passes between reads of the published bounds

// Per-query histogram of the d values of all tiles' final local top-k keys
// (distinct rows), kHistBins bins of 2^hist_shift(M) values each, built after
// the scan.  The first bin at which the running count reaches k bounds the
// k-th smallest d of the whole database from above, far more tightly than
// the best single tile's bound, and lets the merge skip nearly every
// candidate.
constexpr int kHistBins = 1024;

__host__ __device__ constexpr int hist_shift(int M)
{
    int s = 0;
    while (((255 * M) >> s) >= kHistBins)
        ++s;
    return s;
}

struct TileJob {
    const uint8_t *codes;   // the database's codes [N][M/2]
    const uint8_t *luts;    // the database's tables [Q][M][16]
    uint64_t *cand;         // the database's candidates [Q][n_rb][k]
    uint32_t *ccnt = nullptr;   // their counts [Q][n_rb] (packed slots), or null: padded slots
    uint32_t *hist = nullptr;   // with ccnt: per-query histograms [Q][kHistBins] of the kept keys
    int hist_shift = 0;
    uint32_t *fail = nullptr;   // per-query flags [Q]: set when a barrier-free tile overflows
    uint32_t *lcnt = nullptr;   // with sampled bounds: per-query dense candidate lists, cand[q] holding
                                // lcnt[q] keys back to back (instead of slots per row block)
    uint32_t *gthr;         // the database's bounds [Q]
    int64_t r0, r1;         // rows of the tile
    int64_t rb;             // row-block index of the tile
    int64_t n_rb;           // row blocks of the database
    int64_t q0;             // first query of the tile
    int nq;                 // queries of the tile
    uint32_t k;
    RankOrder order;
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per 16-bit lane max(a - b, 0): nonzero lanes are those with b < a.
__device__ __forceinline__ uint32_t sub_sat_u16x2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}

__device__ __forceinline__ uint32_t read_bound(const uint32_t *g) { return __atomic_load_n(g, __ATOMIC_RELAXED); }

// Lowers the published bound to T, unless T does not beat the exclusive
// bound the caller already holds (which includes the published one as last
// read): same-address atomics from thousands of tiles would serialise.
__device__ __forceinline__ void publish(uint32_t *g, uint32_t T, uint32_t known)
{
    if (T <= 0xFFFFu && T + 1u < known)
        atomicMin(g, T);
}

// Final exact local top-k of one query (one wave), written as 48-bit keys.
// known: the exclusive bound the tile holds (see publish).  Keys above the
// published bound as read now cannot be in the top-k; the tile that
// published the final bound still writes its k keys at or below it, so the
// histogram built from the written keys always reaches k.  With cnt_dst the
// kept keys are packed at the front of dst and their number goes to
// *cnt_dst (readers walk only that part), and with hist_q each kept key is
// also counted in the query's histogram (bin d >> shift); without cnt_dst
// all k slots are written, the dropped keys as padding (~0) that the
// readers skip.  With list_cnt the kept keys are appended to the query's
// dense list dst instead, at a position reserved with one atomic add on
// *list_cnt (the list holds every tile's keys back to back).
template <int CAP, bool LDS_PRUNE>
__device__ void write_local_topk(uint32_t *buf, uint32_t n, uint32_t k, int64_t r0,
                                 uint64_t *__restrict__ dst, uint32_t *gthr_q, uint32_t known,
                                 uint32_t *cnt_dst = nullptr, uint32_t *hist_q = nullptr, int shift = 0,
                                 uint32_t *list_cnt = nullptr)
{
    const int lane = threadIdx.x & 63;
    if (n > k) {
        const PruneResult pr = LDS_PRUNE ? prune_local_lds<CAP>(buf, n, k, true)
                                         : prune_local<CAP>(buf, n, k, true);
        n = pr.count;
        if (lane == 0)
            publish(gthr_q, pr.T, known);
    }
    const uint32_t g = __builtin_amdgcn_readfirstlane(read_bound(gthr_q));
    if (list_cnt) {
        uint32_t m = 0;
        for (uint32_t j0 = 0; j0 < n; j0 += 64) {
            const uint32_t j = j0 + lane;
            m += ballot_count(j < n && (buf[j < n ? j : 0] >> 16) <= g);
        }
        if (m == 0)
            return;
        uint32_t at = 0;
        if (lane == 0)
            at = atomicAdd(list_cnt, m);
        at = __builtin_amdgcn_readfirstlane(at);
        for (uint32_t j0 = 0; j0 < n; j0 += 64) {
            const uint32_t j = j0 + lane;
            const uint32_t lk = j < n ? buf[j] : 0xFFFFFFFFu;
            const bool keep = j < n && (lk >> 16) <= g;
            const uint32_t r = ballot_rank(keep);
            if (keep)
                dst[at + r] = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
            at += ballot_count(keep);
        }
        return;
    }
    if (cnt_dst) {
        uint32_t m = 0;
        for (uint32_t j0 = 0; j0 < n; j0 += 64) {
            const uint32_t j = j0 + lane;
            const uint32_t lk = j < n ? buf[j] : 0xFFFFFFFFu;
            const bool keep = j < n && (lk >> 16) <= g;
            const uint32_t r = ballot_rank(keep);
            if (keep) {
                dst[m + r] = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
                if (hist_q)
                    atomicAdd(&hist_q[(lk >> 16) >> shift], 1u);
            }
            m += ballot_count(keep);
        }
        if (lane == 0)
            *cnt_dst = m;
        return;
    }
    for (uint32_t j = lane; j < k; j += 64) {
        uint64_t key = ~0ull;
        if (j < n) {
            const uint32_t lk = buf[j];
            if ((lk >> 16) <= g)
                key = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
        }
        dst[j] = key;
    }
}

// ------------------------------------------------------------------ grouped

template <int MM, int NG>
struct GroupedLds {
    uint4 tab[NG * MM * 256 / 16];                  // [g][m][c][8 queries] uint16
    uint32_t buf[NG * 8 * kGroupedCap];
    uint32_t cnt[NG * 8];
    uint32_t bnd[NG * 8];
    __attribute__((aligned(16))) uint16_t bnd16[NG * 8];
};

template <int MM, int NG>
__device__ void grouped_tile(const TileJob &job, GroupedLds<MM, NG> &L)
{
    constexpr int QG = 8;
    constexpr int QB = QG * NG;
    constexpr int CAP = kGroupedCap;
    constexpr int GROUP_BYTES = MM * 256;
    constexpr int NW = MM / 8;
    constexpr int GU = NG >= 2 ? 2 : 1;
    constexpr uint32_t SMAX = 255u * MM;
    constexpr uint32_t SMAX2 = SMAX | (SMAX << 16);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nq = job.nq;
    const uint32_t k = job.k;
    // one order per grouped tile: calls that mix orders never plan grouped tiles
    const int largest = job.order.largest(job.q0);
    const int64_t q0 = job.q0;

    uint16_t *tab16 = reinterpret_cast<uint16_t *>(L.tab);
    for (int e = tid; e < NG * MM * 16 * QG; e += 256) {
        const int qq = e & 7, c = (e >> 3) & 15;
        const int m = (e >> 7) % MM, g = (e >> 7) / MM;
        const int q = g * QG + qq;
        tab16[e] = q < nq ? job.luts[(q0 + q) * MM * 16 + m * 16 + c] : (uint16_t)0;
    }
    for (int q = tid; q < QB; q += 256) {
        const uint32_t b = q < nq ? read_bound(&job.gthr[q0 + q]) + 1u : 0u;
        L.cnt[q] = 0;
        L.bnd[q] = b;
        L.bnd16[q] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
    }
    __syncthreads();

    const int64_t r0 = job.r0, r1 = job.r1;
    const char *tabb = reinterpret_cast<const char *>(L.tab);
    const uint32_t *bnd2 = reinterpret_cast<const uint32_t *>(L.bnd16);
    int pass = 0;
    // codes are loaded one pass ahead, clamped to the last row so that the
    // load is unconditional and in flight during the whole pass
    uint32_t nxt[NW];
    if (r0 < r1) {
        const int64_t n = r0 + tid;
        load_row<MM>(job.codes, n < r1 ? n : r1 - 1, nxt);
    }
    for (int64_t base = r0; base < r1; base += 256, ++pass) {
        const int64_t n = base + tid;
        const bool valid = n < r1;
        uint32_t cw[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v)
            cw[v] = nxt[v];
        {
            const int64_t nn = n + 256;
            load_row<MM>(job.codes, nn < r1 ? nn : r1 - 1, nxt);
        }
        // the published bounds are read at the start of every pass (an
        // unconditional load, so nothing waits for it early) and folded in at
        // the end of every kRefresh-th pass: the read's latency overlaps the pass
        const bool refresh = (pass % kRefresh) == kRefresh - 1;
        const uint32_t gpre = read_bound(&job.gthr[q0 + (tid < nq ? tid : nq - 1)]);
        const uint32_t local = (uint32_t)(n - r0);
#pragma unroll 1
        for (int g = 0; g < NG; g += GU) {
            const char *tg = tabb + g * GROUP_BYTES;
            uint32_t acc[GU][4];
#pragma unroll
            for (int u = 0; u < GU; ++u)
                acc[u][0] = acc[u][1] = acc[u][2] = acc[u][3] = 0;
#pragma unroll 1
            for (int t = 0; t < NW; ++t) {
                uint32_t w = cw[0];
#pragma unroll
                for (int v = 1; v < NW; ++v)
                    w = (t == v) ? cw[v] : w;
                const char *tt = tg + t * 8 * 256;
#pragma unroll
                for (int kk = 0; kk < 8; kk += 2) {
                    const uint32_t am = (uint32_t)(kk * 256) + (((w >> (4 * kk)) & 15u) << 4);
                    const uint32_t am1 = (uint32_t)((kk + 1) * 256) + (((w >> (4 * kk + 4)) & 15u) << 4);
#pragma unroll
                    for (int u = 0; u < GU; ++u) {
                        const uint4 a = *reinterpret_cast<const uint4 *>(tt + am + u * GROUP_BYTES);
                        const uint4 b = *reinterpret_cast<const uint4 *>(tt + am1 + u * GROUP_BYTES);
                        acc[u][0] += a.x + b.x;
                        acc[u][1] += a.y + b.y;
                        acc[u][2] += a.z + b.z;
                        acc[u][3] += a.w + b.w;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int gg = g + u;
                uint32_t dd[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    dd[v] = largest ? sub_sat_u16x2(SMAX2, acc[u][v]) : acc[u][v];
                const uint4 bp = *reinterpret_cast<const uint4 *>(&bnd2[gg * 4]);
                const uint32_t h0 = sub_sat_u16x2(bp.x, dd[0]), h1 = sub_sat_u16x2(bp.y, dd[1]);
                const uint32_t h2 = sub_sat_u16x2(bp.z, dd[2]), h3 = sub_sat_u16x2(bp.w, dd[3]);
                if (valid && (h0 | h1 | h2 | h3)) {
                    // one bit per query of the group whose d passes its bound
                    uint32_t hm = (h0 & 0xFFFFu ? 1u : 0u) | (h0 >> 16 ? 2u : 0u) | (h1 & 0xFFFFu ? 4u : 0u) |
                                  (h1 >> 16 ? 8u : 0u) | (h2 & 0xFFFFu ? 16u : 0u) | (h2 >> 16 ? 32u : 0u) |
                                  (h3 & 0xFFFFu ? 64u : 0u) | (h3 >> 16 ? 128u : 0u);
                    const uint64_t dlo = (uint64_t)dd[0] | ((uint64_t)dd[1] << 32);
                    const uint64_t dhi = (uint64_t)dd[2] | ((uint64_t)dd[3] << 32);
                    while (hm) {
                        const uint32_t qq = (uint32_t)__builtin_ctz(hm);
                        hm &= hm - 1u;
                        const uint32_t d = (uint32_t)(((qq < 4 ? dlo : dhi) >> (16 * (qq & 3))) & 0xFFFFu);
                        const int q = gg * QG + (int)qq;
                        const uint32_t pos = atomicAdd(&L.cnt[q], 1u);
                        L.buf[q * CAP + pos] = local_key(d, local);
                    }
                }
            }
        }
        __syncthreads();
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = L.cnt[q];
            if (c > CAP - 256) {
                PruneResult pr = prune_local<CAP>(L.buf + q * CAP, c, k, false);
                if (pr.count > CAP - 256)
                    pr = prune_local<CAP>(L.buf + q * CAP, pr.count, k, true);
                if (lane == 0) {
                    L.cnt[q] = pr.count;
                    publish(&job.gthr[q0 + q], pr.T, L.bnd[q]);
                    uint32_t b = L.bnd[q];
                    b = pr.T < b ? pr.T : b;
                    L.bnd[q] = b;
                    L.bnd16[q] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
                }
            }
        }
        if (refresh) {
            __syncthreads();
            if (tid < nq) {
                uint32_t b = L.bnd[tid];
                const uint32_t gb = gpre + 1u;
                b = gb < b ? gb : b;
                L.bnd[tid] = b;
                L.bnd16[tid] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4)
        write_local_topk<CAP, false>(L.buf + q * CAP, L.cnt[q], k, r0,
                                     job.cand + ((q0 + q) * job.n_rb + job.rb) * (int64_t)k,
                                     &job.gthr[q0 + q], L.bnd[q],
                                     job.ccnt ? job.ccnt + (q0 + q) * job.n_rb + job.rb : nullptr,
                                     job.hist ? job.hist + (q0 + q) * kHistBins : nullptr, job.hist_shift);
}

// ------------------------------------------------------------------ matrix cores
//
// With many queries the scan is a matrix product (Sec. 3.1 written as a
// contraction): write row n's codes one-hot, 16 entries per subspace of
// which the code's entry is 1; the sum of query q over row n is the dot
// product of that 16M-entry row with column q of the tables.  The int8
// matrix cores evaluate it exactly in int32.  A table entry T enters as the
// int8 value T - 128, or (255 - T) - 128 when the largest sums are wanted,
// so that acc + 128 M is d itself: the sum, or 255 M - sum (M entries of
// each one-hot row are 1).
//
// v_mfma_i32_32x32x32_i8: lane l supplies row l % 32 of the one-hot codes
// and column l % 32 of the tables, both over the same 16 K entries of its
// half l / 32 (here the 16 centroids of subspace 2 s + l / 32 at step s),
// and receives rows 8 (v / 4) + 4 (l / 32) + v % 4 of column l % 32 in
// accumulator v.  A wave holds the tables of its NT query tiles (32 queries
// each) in registers for the whole tile and takes 32 rows per pass; the
// one-hot operand comes from a 16-entry LDS table, conflict free.
//
// Sparse form (SP): a one-hot row has one nonzero in every group of four
// entries at most, which is the 4:2 structure of the sparse matrix
// instruction v_smfmac_i32_32x32x64_i8: it contracts 64 entries (four
// subspaces) in the time the dense one takes for 32, from a compressed
// operand of two (value, 2-bit position) slots per group.  Its lanes pair
// up as follows: compressed element j (0..15) of lane l (row l % 32, half
// h = l / 32) multiplies byte 16 h + 4 ((j / 2) % 4) + pos_j of the table
// operand of lane 32 (j / 8) + l % 32, whose 32 bytes are two 16-byte
// blocks.  So with the table operand of step i (lane half g) made of the
// tables of subspaces 4 i + g and 4 i + 2 + g -- the dense form's steps
// 2 i and 2 i + 1, unchanged in registers -- lane half h covers subspaces
// 4 i + 2 h (elements 0..7) and 4 i + 2 h + 1 (elements 8..15), the two
// nibbles of code byte 2 i + h.  Code c of the low nibble is element
// 2 (c / 4) with value 1 and position c % 4, that of the high nibble
// element 8 + 2 (c / 4); every other element is 0.  The values depend only
// on the two group numbers (a 16-entry table, conflict free) and the
// positions on the byte (a 256-entry table of index words).  The result
// lanes are those of the dense form.
//
// FREE (with speculative starting bounds only): the bounds are taken as
// they are and never tightened, so the waves need no barriers between
// passes, and no atomics either: the query's buffer is cut into kMfmaSegs
// segments, one per (wave, lane half), each lane appending to its own with
// a private count; the tile's end packs the segments.  A query whose
// segment would overflow (never in practice: the bound admits a few rows
// per tile) is flagged in job.fail, writes no keys, and is recomputed
// exactly by the final merge.

constexpr int kMfmaCap = 256;    // candidate slots per query: k <= kMfmaCap - kMfmaPass
constexpr int kMfmaPass = 128;   // rows per pass: 4 waves x 32
constexpr int kMfmaSegs = 8;     // FREE: one buffer segment per (wave, lane half)
constexpr int kMfmaSeg = kMfmaCap / kMfmaSegs;

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// Operand tables of the one-hot codes in LDS.
struct OneHot {
    uint4 dense[16];     // entry c: byte c is 1
    uint4 sval[16];      // sparse values, entry g0 + 4 g1: bytes 2 g0 and 8 + 2 g1 are 1
    uint32_t sidx[256];  // sparse positions of code byte b: (b & 3) << 4 (b >> 2 & 3), (b >> 4 & 3) << 16 + 4 (b >> 6)
};

template <int NT>
struct MfmaLds {
    uint32_t buf[NT * 32 * kMfmaCap];
    uint32_t cnt[NT * 32];
    uint32_t bnd[NT * 32];
    uint32_t seg[NT * 32 * kMfmaSegs];   // FREE: keys appended to each segment
    OneHot oh;
};

// Fills the one-hot tables (every thread of a 256-thread workgroup takes part).
__device__ __forceinline__ void onehot_init(OneHot &T)
{
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int c = tid >> 2, j = tid & 3;
        reinterpret_cast<uint32_t *>(T.dense)[tid] = (c >> 2) == j ? (1u << (8 * (c & 3))) : 0u;
        const int g = j < 2 ? (c & 3) : (c >> 2);   // entry c = g0 + 4 g1; words 0, 1 hold g0, words 2, 3 g1
        reinterpret_cast<uint32_t *>(T.sval)[tid] = (g >> 1) == (j & 1) ? (1u << (16 * (g & 1))) : 0u;
    }
    for (int b = tid; b < 256; b += blockDim.x) {
        const uint32_t c0 = b & 15u, c1 = (uint32_t)b >> 4;
        T.sidx[b] = ((c0 & 3u) << (4u * (c0 >> 2))) | ((c1 & 3u) << (16u + 4u * (c1 >> 2)));
    }
}

// Whether the matrix-core tiles use the sparse instruction (test hook).
extern int g_sparse_mfma;

// This lane's table columns (queries q0 + 32 t + l % 32, subspace 2 s + l / 32)
// as int8 T - 128 (or (255 - T) - 128 for the largest sums); queries at or
// beyond nq get zeros.  The loads are unconditional (clamped query) so that
// all of them are in flight together.
template <int MM, int NT>
__device__ __forceinline__ void mfma_load_tables(const uint8_t *__restrict__ luts, int64_t q0, int nq,
                                                 RankOrder order, i32x4 (&tb)[NT][MM / 2])
{
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int q = 32 * t + col;
        const uint32_t flip = order.largest(q0 + q) ? 0x7F7F7F7Fu : 0x80808080u;
        const uint32_t keep = q < nq ? 0xFFFFFFFFu : 0u;
        const uint8_t *src = luts + ((q0 + (q < nq ? q : nq - 1)) * MM + half) * 16;
#pragma unroll
        for (int s = 0; s < MM / 2; ++s) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src + 2 * s * 16);
            tb[t][s] = i32x4{(int)((v.x ^ flip) & keep), (int)((v.y ^ flip) & keep), (int)((v.z ^ flip) & keep),
                             (int)((v.w ^ flip) & keep)};
        }
    }
}

// acc[t] = d - 128 M of this lane's 16 rows (its code row cw is row l % 32 of
// the wave's 32) against the queries of table tile t.
template <int MM, int NT, bool SP>
__device__ __forceinline__ void mfma_pass(const uint32_t (&cw)[MM / 8], const OneHot &T,
                                          const i32x4 (&tb)[NT][MM / 2], i32x16 (&acc)[NT])
{
    constexpr int NW = MM / 8;
    const int half = (threadIdx.x & 63) >> 5;
    if constexpr (SP) {
        const char *sv = reinterpret_cast<const char *>(T.sval);
        const char *oh = reinterpret_cast<const char *>(T.dense);
        // Subspaces 0-3 take two dense steps: the first one starts the
        // accumulators from zero, which the sparse instruction (it
        // accumulates in place) could only do after 16 register moves.
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const i32x4 av = *reinterpret_cast<const i32x4 *>(oh + ((cw[0] >> (8 * s + 4 * half)) & 15u) * 16u);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, tb[t][s], s == 0 ? i32x16{} : acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            // bytes 0 and 2 of w: the code bytes of steps 2 v and 2 v + 1
            const uint32_t w = cw[v] >> (8 * half);
            // per 16-bit half: 16 (g0 + 4 g1), the offset of the values entry
            const uint32_t off = ((w & 0x000C000Cu) << 2) | (w & 0x00C000C0u);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (v == 0 && e == 0)
                    continue;   // subspaces 0-3: the dense steps above
                const uint32_t pos = T.sidx[(w >> (16 * e)) & 0xFFu];
                const i32x4 av = *reinterpret_cast<const i32x4 *>(sv + ((off >> (16 * e)) & 0xFFFFu));
                const int s = 4 * v + 2 * e;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const i32x8 bv = __builtin_shufflevector(tb[t][s], tb[t][s + 1], 0, 1, 2, 3, 4, 5, 6, 7);
                    acc[t] = __builtin_amdgcn_smfmac_i32_32x32x64_i8(av, bv, acc[t], (int)pos, 0, 0);
                }
            }
        }
        return;
    }
    const char *oh = reinterpret_cast<const char *>(T.dense);
    // byte s of wa: the LDS offset (16 x code) of subspace 2 s + half
    uint32_t wa[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v)
        wa[v] = (cw[v] << (4 - 4 * half)) & 0xF0F0F0F0u;
#pragma unroll
    for (int t = 0; t < NT; ++t)
        acc[t] = i32x16{};
    if constexpr (MM >= 64) {
        // two waves per SIMD at this width: keep four one-hot reads in flight,
        // in the order written (the scheduler would otherwise sink them)
        constexpr int D = 4;
        i32x4 av[D];
#pragma unroll
        for (int s = 0; s < D - 1; ++s)
            av[s] = *reinterpret_cast<const i32x4 *>(oh + ((wa[s >> 2] >> (8 * (s & 3))) & 0xFFu));
#pragma unroll
        for (int s = 0; s < MM / 2; ++s) {
            if (s + D - 1 < MM / 2) {
                const int u = s + D - 1;
                av[u % D] = *reinterpret_cast<const i32x4 *>(oh + ((wa[u >> 2] >> (8 * (u & 3))) & 0xFFu));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[s % D], tb[t][s], acc[t], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < MM / 2; ++s) {
            const uint32_t a = (wa[s >> 2] >> (8 * (s & 3))) & 0xFFu;
            const i32x4 av = *reinterpret_cast<const i32x4 *>(oh + a);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, tb[t][s], acc[t], 0, 0, 0);
        }
    }
}

template <int MM, int NT, bool FREE, bool SP>
__device__ void mfma_tile(const TileJob &job, MfmaLds<NT> &L)
{
    constexpr int KS = MM / 2;       // matrix-core steps per row, two subspaces each
    constexpr int NW = MM / 8;       // code dwords per row
    constexpr int QB = 32 * NT;
    constexpr int CAP = kMfmaCap;
    constexpr int OFF = 128 * MM;
    constexpr int PER_WAVE = QB / 4;  // queries each wave checks for pruning
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, col = lane & 31;
    const int nq = job.nq;
    const uint32_t k = job.k;
    const int64_t q0 = job.q0;

    onehot_init(L.oh);
    for (int q = tid; q < QB; q += 256) {
        L.cnt[q] = 0;
        L.bnd[q] = q < nq ? read_bound(&job.gthr[q0 + q]) + 1u : 0u;
    }
    // absent queries: zero tables and bound 0
    i32x4 tb[NT][KS];
    mfma_load_tables<MM, NT>(job.luts, q0, nq, job.order, tb);
    __syncthreads();

    const int64_t r0 = job.r0, r1 = job.r1;
    // codes one pass ahead, clamped to the last row (unconditional loads)
    uint32_t nxt[NW];
    if (r0 < r1) {
        const int64_t n = r0 + 32 * wave + col;
        load_row<MM>(job.codes, n < r1 ? n : r1 - 1, nxt);
    }
    // hit iff d = acc + OFF < bound (FREE: the bounds never change)
    int thr[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        thr[t] = (int)L.bnd[32 * t + col] - OFF;
    // FREE: this lane's segment of each query's buffer and its append count
    const int sg = 2 * wave + half;
    uint32_t pc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        pc[t] = 0;
    int pass = 0;
    for (int64_t base = r0; base < r1; base += kMfmaPass, ++pass) {
        // published bounds: read at the start of every pass (unconditional,
        // before the code prefetch), folded in at the end of every
        // kRefresh-th pass
        const bool refresh = !FREE && (pass % kRefresh) == kRefresh - 1;
        const uint32_t gpre = FREE ? 0u : read_bound(&job.gthr[q0 + (tid < nq ? tid : nq - 1)]);
        uint32_t cw[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v)
            cw[v] = nxt[v];
        {
            const int64_t nn = base + kMfmaPass + 32 * wave + col;
            load_row<MM>(job.codes, nn < r1 ? nn : r1 - 1, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of the pass
        if (!FREE) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                thr[t] = (int)L.bnd[32 * t + col] - OFF;
        }

        i32x16 acc[NT];
        mfma_pass<MM, NT, SP>(cw, L.oh, tb, acc);

        // rows of accumulator v: rb + 8 (v / 4) + v % 4
        const int64_t rb = base + 32 * wave + 4 * half;
        if (base + kMfmaPass > r1) {   // ragged last pass: rows past the tile never pass
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (rb + 8 * (v >> 2) + (v & 3) >= r1)
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[t][v] = 1 << 30;
        }
        bool any = false;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int mn = acc[t][0];
#pragma unroll
            for (int v = 1; v < 16; ++v)
                mn = acc[t][v] < mn ? acc[t][v] : mn;
            any = any || mn < thr[t];
        }
        if (__ballot(any)) {
            const uint32_t lbase = (uint32_t)(rb - r0);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int q = 32 * t + col;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    if (acc[t][v] < thr[t]) {
                        const uint32_t d = (uint32_t)(acc[t][v] + OFF);
                        const uint32_t key = local_key(d, lbase + 8 * (v >> 2) + (v & 3));
                        if (FREE) {
                            if (pc[t] < (uint32_t)kMfmaSeg)
                                L.buf[q * CAP + sg * kMfmaSeg + pc[t]] = key;
                            ++pc[t];
                        } else {
                            L.buf[q * CAP + atomicAdd(&L.cnt[q], 1u)] = key;
                        }
                    }
                }
            }
        }
        if (FREE)
            continue;
        __syncthreads();
        {
            const int qw = wave * PER_WAVE;
            const uint32_t c = lane < PER_WAVE ? L.cnt[qw + lane] : 0u;
            uint64_t full = __ballot(c > CAP - kMfmaPass);
            while (full) {
                const int q = qw + (int)__builtin_ctzll(full);
                full &= full - 1;
                PruneResult pr = prune_local<CAP>(L.buf + q * CAP, L.cnt[q], k, false);
                if (pr.count > CAP - kMfmaPass)
                    pr = prune_local<CAP>(L.buf + q * CAP, pr.count, k, true);
                if (lane == 0) {
                    L.cnt[q] = pr.count;
                    publish(&job.gthr[q0 + q], pr.T, L.bnd[q]);
                    const uint32_t b = L.bnd[q];
                    L.bnd[q] = pr.T < b ? pr.T : b;
                }
            }
        }
        if (refresh) {
            __syncthreads();
            if (tid < nq && tid < QB) {
                const uint32_t b = L.bnd[tid], gb = gpre + 1u;
                L.bnd[tid] = gb < b ? gb : b;
            }
        }
        __syncthreads();
    }
    if (FREE) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
            L.seg[(32 * t + col) * kMfmaSegs + sg] = pc[t];
        __syncthreads();   // every append is done
    }
    // dense lists: reserve each query's place now (its count is known from
    // the segment counts: min(n, k), 0 on overflow), so that the atomic's
    // round trip overlaps the packing below; the offset is used after it
    uint32_t list_at = 0;
    if (FREE && job.lcnt && tid < nq && tid < QB) {
        uint32_t n = 0;
        bool over = false;
#pragma unroll
        for (int g = 0; g < kMfmaSegs; ++g) {
            const uint32_t c = L.seg[tid * kMfmaSegs + g];
            over = over || c > (uint32_t)kMfmaSeg;
            n += c;
        }
        const uint32_t m = over ? 0u : (n < k ? n : k);
        if (m)
            list_at = atomicAdd(job.lcnt + q0 + tid, m);
    }
    for (int q = wave; q < nq && q < QB; q += 4) {
        if (FREE) {
            // pack the segments in place: a wave reads all of the query's
            // keys into registers before it writes any
            const uint32_t c = lane < kMfmaSegs ? L.seg[q * kMfmaSegs + lane] : 0u;
            if (__ballot(c > (uint32_t)kMfmaSeg)) {   // overflowed: no keys, the merge recomputes the query
                if (lane == 0) {
                    job.fail[q0 + q] = 1u;
                    if (job.ccnt && !job.lcnt)
                        job.ccnt[(q0 + q) * job.n_rb + job.rb] = 0u;
                    L.cnt[q] = 0u;
                }
                continue;
            }
            // key i of the packed list sits at slot i + (g kMfmaSeg - pre_g) of
            // its segment g: the gaps of the segments before it
            uint32_t pre[kMfmaSegs], gap[kMfmaSegs];
            uint32_t n = 0;
#pragma unroll
            for (int g = 0; g < kMfmaSegs; ++g) {
                const uint32_t cg = __shfl(c, g);
                pre[g] = n;
                gap[g] = (uint32_t)kMfmaSeg - cg;
                n += cg;
            }
            constexpr int PER = CAP / 64;
            uint32_t key[PER];
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const uint32_t i = (uint32_t)(lane + 64 * e);
                uint32_t src = i;
#pragma unroll
                for (int g = 1; g < kMfmaSegs; ++g)
                    src += i >= pre[g] ? gap[g - 1] : 0u;
                key[e] = i < n ? L.buf[q * CAP + src] : 0u;
            }
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const uint32_t i = (uint32_t)(lane + 64 * e);
                if (i < n)
                    L.buf[q * CAP + i] = key[e];
            }
            if (lane == 0)
                L.cnt[q] = n;
        }
        if (FREE && job.lcnt) {
            // dense lists: keep at most k keys (all of them are below the
            // query's fixed bound); their place in the list is reserved below
            if (L.cnt[q] > k) {
                const PruneResult pr = prune_local<CAP>(L.buf + q * CAP, L.cnt[q], k, true);
                if (lane == 0)
                    L.cnt[q] = pr.count;
            }
            continue;
        }
        write_local_topk<CAP, false>(L.buf + q * CAP, L.cnt[q], k, r0,
                                     job.cand + ((q0 + q) * job.n_rb + job.rb) * (int64_t)k,
                                     &job.gthr[q0 + q], L.bnd[q],
                                     job.ccnt ? job.ccnt + (q0 + q) * job.n_rb + job.rb : nullptr,
                                     job.hist ? job.hist + (q0 + q) * kHistBins : nullptr, job.hist_shift);
    }
    if (FREE && job.lcnt) {
        // the keys of each query in one contiguous run at its reserved place
        __syncthreads();
        if (tid < nq && tid < QB)
            L.bnd[tid] = list_at;
        __syncthreads();
        for (int q = wave; q < nq && q < QB; q += 4) {
            const uint32_t n = L.cnt[q], at = L.bnd[q];
            uint64_t *dst = job.cand + (q0 + q) * job.n_rb * (int64_t)k + at;
            for (uint32_t j = lane; j < n; j += 64) {
                const uint32_t lk = L.buf[q * CAP + j];
                dst[j] = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
            }
        }
    }
}

// Sample for the speculative bounds: the d of every (query, row) of the
// kSpecSpan consecutive rows from r0, reduced to one minimum per group of
// kSpecGroup rows (the 16 rows one lane's accumulators hold in a pass, from
// four runs of four), written as uint16 to out[q][g0 .. g0 + kSpecGroups)
// (out has G entries per query).  The minima are staged in LDS (gmin, at
// least 32 * NT * kSpecGminStride entries) and stored as 16-byte rows.
constexpr int kSpecGminStride = kSpecGroups + 8;   // uint16 per query row in LDS (2-way banks)

template <int MM, int NT, bool SP>
__device__ void mfma_sample_tile(const uint8_t *__restrict__ codes, const uint8_t *__restrict__ luts, int64_t q0,
                                 int nq, RankOrder order, int64_t r0, uint16_t *__restrict__ out, int64_t G,
                                 int64_t g0, OneHot &oh, uint16_t *gmin)
{
    constexpr int NW = MM / 8;
    constexpr int OFF = 128 * MM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, col = lane & 31;
    onehot_init(oh);
    i32x4 tb[NT][MM / 2];
    mfma_load_tables<MM, NT>(luts, q0, nq, order, tb);
    __syncthreads();
    // codes one pass ahead (the last pass re-reads its own rows)
    uint32_t nxt[NW];
    load_row<MM>(codes, r0 + 32 * wave + col, nxt);
    for (int base = 0; base < (int)kSpecSpan; base += kMfmaPass) {
        uint32_t cw[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v)
            cw[v] = nxt[v];
        const int ahead = base + kMfmaPass < (int)kSpecSpan ? base + kMfmaPass : base;
        load_row<MM>(codes, r0 + ahead + 32 * wave + col, nxt);
        __builtin_amdgcn_sched_barrier(0);
        i32x16 acc[NT];
        mfma_pass<MM, NT, SP>(cw, oh, tb, acc);
        const int g = base / kSpecGroup + 2 * wave + half;   // this lane's group in the chunk
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int m = acc[t][0];
#pragma unroll
            for (int v = 1; v < 16; ++v)
                m = acc[t][v] < m ? acc[t][v] : m;
            gmin[(32 * t + col) * kSpecGminStride + g] = (uint16_t)(m + OFF);
        }
    }
    __syncthreads();
    constexpr int V = kSpecGroups / 8;   // 16-byte words per query
    for (int e = tid; e < nq * V; e += 256) {
        const int q = e / V, v = e - q * V;
        reinterpret_cast<uint4 *>(out + (q0 + q) * G + g0)[v] =
            reinterpret_cast<const uint4 *>(gmin + q * kSpecGminStride)[v];
    }
}

// ------------------------------------------------------------------ few queries

// Rows per lane per pass: enough code bytes in flight per lane (32 to 128)
// to keep HBM busy, at most 32 registers of codes per buffer.
__host__ __device__ constexpr int few_r(int M) { return M >= 32 ? 4 : 8; }
__host__ __device__ constexpr int few_pass(int M) { return 256 * few_r(M); }
// Candidate slots per query: a full pass plus room for k <= 256 and slack.
__host__ __device__ constexpr int few_cap(int M) { return few_pass(M) + 1024; }

// Pair tables of nq queries: entry b of pair p is lut[2p][b & 15] +
// lut[2p+1][b >> 4].  stage (LDS, nq * MM * 16 bytes, 16-byte aligned, free
// until the next barrier) takes the raw tables first with one 16-byte load
// per table, so each entry is then built from LDS; without it (or with
// unaligned tables) the entries read the tables from global memory byte by
// byte.  Every thread of the workgroup must call it.
template <int MM>
__device__ __forceinline__ void build_pair_tables(const uint8_t *__restrict__ luts, int nq, uint16_t *pt,
                                                  uint8_t *stage = nullptr)
{
    constexpr int NP = MM / 2;
    const uint8_t *src = luts;
    if (stage && (reinterpret_cast<uintptr_t>(luts) & 15) == 0) {
        for (int t = threadIdx.x; t < nq * MM; t += 256)
            reinterpret_cast<uint4 *>(stage)[t] = reinterpret_cast<const uint4 *>(luts)[t];
        __syncthreads();
        src = stage;
    }
    for (int e = threadIdx.x; e < nq * NP * 256; e += 256) {
        const int b = e & 255, p = (e >> 8) % NP, q = (e >> 8) / NP;
        const uint8_t *l = src + ((int64_t)q * MM + 2 * p) * 16;
        pt[e] = (uint16_t)(l[b & 15] + l[16 + (b >> 4)]);
    }
}

// Byte J of w times 2 (the byte offset of a uint16 table entry) in one
// VALU instruction: the SDWA source select extracts the byte.  Written as
// volatile asm (an ALU instruction, not a load) so that it keeps its place
// in the pipelined order below instead of being hoisted with all the others.
template <int J>
__device__ __forceinline__ uint32_t byte_x2(uint32_t w)
{
    uint32_t r;
    asm volatile("v_lshlrev_b32_sdwa %0, 1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_%2"
                 : "=v"(r)
                 : "v"(w), "i"(J));
    return r;
}

// a + b + c, kept in program order for the same reason.
__device__ __forceinline__ uint32_t add3_ordered(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm volatile("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Table reads of code dword t of the R rows (4 bytes each, one pair table per byte).
template <int MM, int R>
__device__ __forceinline__ void pair_reads(const char *tq, const uint32_t (&cw)[R][MM / 8], int t,
                                           uint32_t (&v)[R][4])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t w = cw[r][t];
        v[r][0] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 0) * 512 + byte_x2<0>(w));
        v[r][1] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 1) * 512 + byte_x2<1>(w));
        v[r][2] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 2) * 512 + byte_x2<2>(w));
        v[r][3] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 3) * 512 + byte_x2<3>(w));
    }
}

// Table reads of code dword t of rows g G .. g G + G - 1 of cw.
template <int MM, int R, int G>
__device__ __forceinline__ void pair_reads_group(const char *tq, const uint32_t (&cw)[R][MM / 8], int g, int t,
                                                 uint32_t (&v)[G][4])
{
#pragma unroll
    for (int r = 0; r < G; ++r) {
        const uint32_t w = cw[g * G + r][t];
        v[r][0] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 0) * 512 + byte_x2<0>(w));
        v[r][1] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 1) * 512 + byte_x2<1>(w));
        v[r][2] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 2) * 512 + byte_x2<2>(w));
        v[r][3] = *reinterpret_cast<const uint16_t *>(tq + (4 * t + 3) * 512 + byte_x2<3>(w));
    }
}

// Sums of one query for the R rows held in cw; tq is the query's pair
// tables (MM/2 tables of 256 uint16, 512 bytes each).  Every code byte is one
// 16-bit LDS read at byte offset 512 * pair + 2 * byte.
//
// UNROLL (one query per tile, tables at a fixed LDS address): fully
// unrolled, so each pair offset is an immediate of its read and a code byte
// costs one VALU instruction plus half an add; the reads of dword t + 1 are
// issued before the adds of dword t (two dwords of reads in flight).
// Otherwise (several queries): the dword loop stays rolled and selects the
// dword with a short chain, which keeps the registers low when the offsets
// would otherwise be hoisted out of the loop over queries.
template <int MM, int R, bool UNROLL>
__device__ __forceinline__ void pair_sums(const char *tq, const uint32_t (&cw)[R][MM / 8], uint32_t (&s)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r)
        s[r] = 0;
    if constexpr (UNROLL) {
        // steps of (group of G rows, code dword t): the reads of step i + 1
        // are issued before the adds of step i, with 8 G registers of reads
        // in flight whatever R is
        constexpr int T = MM / 8;
        constexpr int G = R < 4 ? R : 4;
        constexpr int NS = (R / G) * T;
        static_assert(R % G == 0, "whole row groups");
        uint32_t v[2][G][4];
        pair_reads_group<MM, R, G>(tq, cw, 0, 0, v[0]);
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            if (st + 1 < NS)
                pair_reads_group<MM, R, G>(tq, cw, (st + 1) / T, (st + 1) % T, v[(st + 1) & 1]);
            const int g = st / T;
#pragma unroll
            for (int r = 0; r < G; ++r) {
                s[g * G + r] = add3_ordered(s[g * G + r], v[st & 1][r][0], v[st & 1][r][1]);
                s[g * G + r] = add3_ordered(s[g * G + r], v[st & 1][r][2], v[st & 1][r][3]);
            }
        }
    } else {
#pragma unroll 1
        for (int t = 0; t < MM / 8; ++t) {
            uint32_t w[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                w[r] = cw[r][0];
#pragma unroll
                for (int v = 1; v < MM / 8; ++v)
                    w[r] = (t == v) ? cw[r][v] : w[r];
            }
            const char *tt = tq + t * 4 * 512;
            uint32_t v[R][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t byte = (w[r] >> (8 * j)) & 0xFFu;
                    v[r][j] = *reinterpret_cast<const uint16_t *>(tt + j * 512 + 2 * byte);
                }
#pragma unroll
            for (int r = 0; r < R; ++r)
                s[r] += v[r][0] + v[r][1] + v[r][2] + v[r][3];
        }
    }
}

// Rows [base, min(r1, base + 256 R)) into cw (lane row tid + 256 r; zeros
// past the end): a uniform base pointer and 32-bit lane offsets.  These
// rows are streamed once per call (one or a few queries): non-temporal
// loads unless NT is false.
template <int MM, int R, bool NT = true>
__device__ __forceinline__ void load_rows(const uint8_t *__restrict__ codes, int64_t base, int64_t r1,
                                          uint32_t (&cw)[R][MM / 8])
{
    const uint8_t *p = codes + base * (MM / 2);
    const int64_t avail = r1 - base;
    const uint32_t lim = avail >= 256 * R ? 256u * R : (avail > 0 ? (uint32_t)avail : 0u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + 256u * r;
        if (i < lim)
            load_row<MM, NT>(p, (int64_t)i, cw[r]);
        else
#pragma unroll
            for (int v = 0; v < MM / 8; ++v)
                cw[r][v] = 0;
    }
}

// As load_rows, but every lane loads: a lane past the end re-reads the last
// row of the range (row 0 of codes if the range is empty) and the caller
// ignores it.  Unconditional loads keep the number of loads in flight known
// to the compiler, so it waits only for the older batch, not for all.
template <int MM, int R, bool NT = true>
__device__ __forceinline__ void load_rows_clamped(const uint8_t *__restrict__ codes, int64_t base, int64_t r1,
                                                  uint32_t (&cw)[R][MM / 8])
{
    const int64_t avail = r1 - base;
    const uint8_t *p = avail > 0 ? codes + base * (MM / 2) : codes;
    const uint32_t last = avail >= 256 * R ? 256u * R - 1 : (avail > 0 ? (uint32_t)avail - 1 : 0u);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + 256u * r;
        load_row<MM, NT>(p, (int64_t)(i < last ? i : last), cw[r]);
    }
}

template <int MM, int R>
__device__ __forceinline__ void copy_rows(const uint32_t (&a)[R][MM / 8], uint32_t (&b)[R][MM / 8])
{
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < MM / 8; ++v)
            b[r][v] = a[r][v];
}

// Exact local top-k of one query over rows [r0, r1) of codes (at most 65536
// rows), one 256-thread workgroup: the pair tables of the query's tables
// luts ([M][16]) are static LDS at a fixed address, so their offsets fold
// into the reads; rows are loaded with a uniform base and 32-bit lane
// offsets, unconditionally, so the next pass stays in flight while this one
// is computed.  Keys below the bound (from *gthr, refreshed every 8 passes
// and lowered by pruning, published to *gthr) go to an LDS buffer; the
// kept keys (d << 32 | row) are written packed to dst with their count in
// *cnt_dst and counted in hist (when cnt_dst is given), else as k padded
// slots, or appended to the dense list dst with its count in *list_cnt
// when list_cnt is given.
// lds: one_query_lds_bytes(MM) bytes, 16-byte aligned (a static
// array, so that the table offsets stay compile-time constants).  Wave 0
// still writes the result when the other waves return: a caller that
// reuses lds must synchronise first.
// The pair tables' random 16-bit reads conflict on LDS banks (about 60% of
// the LDS cycles at M = 16 and 32, and the LDS is then the busiest unit):
// one 16-byte table per subspace, which lies in one bank row, removes the
// conflicts but doubles the reads and the address arithmetic, and measured
// equal at M = 16 and 11% slower at M = 32.
// Rows per lane per pass of the one-query tile (its codes in flight per lane:
// R M / 2 bytes; 128 at M = 32, measured 4% faster than 64 over 2.5e8 rows,
// 64 at M = 16 where 96 was slower), a pass and the candidate buffer (a
// pass plus room for k <= 256 and slack).
__host__ __device__ constexpr int one_r(int M) { return M == 32 ? 8 : (M > 32 ? 4 : 8); }
__host__ __device__ constexpr int one_pass(int M) { return 256 * one_r(M); }
__host__ __device__ constexpr int one_cap(int M) { return one_pass(M) + 1024; }

__host__ __device__ constexpr size_t one_query_lds_bytes(int M)
{
    return (size_t)(M / 2) * 256 * sizeof(uint16_t) + (size_t)one_cap(M) * sizeof(uint32_t);
}

//
// HIST (the exact recomputation): the tile also counts, in the LDS
// histogram hl (kHistBins words, zeroed by the caller), the d of every row
// at or below the query's published bound (s_hlim: inclusive, lowered with
// the tile's own pruned bound), and adds the bins up to that bound to the
// query's histogram hq.  The published bound never drops below the query's
// k-th smallest d, so every tile counts every row at or below it, and the
// sum over the tiles is exact on every bin up to the one holding it.
template <int MM, bool HIST = false>
__device__ __forceinline__ void one_query_tile(const uint8_t *__restrict__ codes, int64_t r0, int64_t r1,
                                               const uint8_t *__restrict__ luts, uint32_t k, int largest,
                                               uint64_t *__restrict__ dst, uint32_t *cnt_dst, uint32_t *hist,
                                               uint32_t *gthr, char *lds, uint32_t *list_cnt = nullptr,
                                               uint32_t *hl = nullptr, uint32_t *hq = nullptr)
{
    constexpr int R = one_r(MM);
    constexpr int PASS = one_pass(MM);
    constexpr int CAP = one_cap(MM);
    constexpr uint32_t SMAX = 255u * MM;
    constexpr int SHIFT = hist_shift(MM);
    uint16_t *pt = reinterpret_cast<uint16_t *>(lds);
    uint32_t *buf = reinterpret_cast<uint32_t *>(lds + (MM / 2) * 256 * sizeof(uint16_t));
    __shared__ uint32_t s_cnt, s_bnd, s_hlim;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t cw[R][MM / 8], nx[R][MM / 8];
    load_rows_clamped<MM, R>(codes, r0, r1, nx);
    build_pair_tables<MM>(luts, 1, pt, reinterpret_cast<uint8_t *>(buf));
    if (tid == 0) {
        s_cnt = 0;
        s_bnd = read_bound(gthr) + 1u;
        s_hlim = s_bnd - 1u;
    }
    __syncthreads();
    int pass = 0;
    for (int64_t base = r0; base < r1; base += PASS, ++pass) {
        copy_rows<MM, R>(nx, cw);
        if (base + PASS < r1)
            load_rows_clamped<MM, R>(codes, base + PASS, r1, nx);
        uint32_t s[R];
        pair_sums<MM, R, true>(reinterpret_cast<const char *>(pt), cw, s);
        const uint32_t bq = s_bnd;
        const uint32_t hlim = HIST ? s_hlim : 0u;
        const uint32_t loc = (uint32_t)(base - r0) + (uint32_t)tid;
        const uint32_t lim = (uint32_t)((r1 - base) < PASS ? (r1 - base) : PASS);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = largest ? SMAX - s[r] : s[r];
            if (d < bq && (uint32_t)tid + 256u * r < lim) {
                const uint32_t pos = atomicAdd(&s_cnt, 1u);
                buf[pos] = local_key(d, loc + 256u * r);
            }
            if constexpr (HIST)
                if (d <= hlim && (uint32_t)tid + 256u * r < lim)
                    atomicAdd(&hl[d >> SHIFT], 1u);
        }
        __syncthreads();
        if (wave == 0) {
            const uint32_t c = s_cnt;
            uint32_t nb = 0xFFFFFFFFu;
            if (c > CAP - PASS) {
                PruneResult pr = prune_local_lds<CAP>(buf, c, k, false);
                if (pr.count > CAP - PASS)
                    pr = prune_local_lds<CAP>(buf, pr.count, k, true);
                if (lane == 0) {
                    s_cnt = pr.count;
                    publish(gthr, pr.T, s_bnd);
                }
                nb = pr.T;
            }
            if (lane == 0 && (nb != 0xFFFFFFFFu || (pass & 7) == 7)) {
                uint32_t b = s_bnd;
                b = nb < b ? nb : b;
                const uint32_t gb = read_bound(gthr) + 1u;
                s_bnd = gb < b ? gb : b;
                if constexpr (HIST) {   // inclusive: the pruned k-th d and the published bound
                    uint32_t h = s_hlim;
                    h = nb < h ? nb : h;
                    s_hlim = gb - 1u < h ? gb - 1u : h;
                }
            }
        }
        __syncthreads();
    }
    if (wave == 0)
        write_local_topk<CAP, true>(buf, s_cnt, k, r0, dst, gthr, s_bnd, cnt_dst, hist, hist_shift(MM), list_cnt);
    if constexpr (HIST) {
        const uint32_t top = s_hlim >> SHIFT;   // no row above this bin was counted in every pass
        for (uint32_t i = tid; i <= top && i < (uint32_t)kHistBins; i += 256)
            if (hl[i])
                atomicAdd(&hq[i], hl[i]);
    }
}

// LDS of a few-query tile: pair tables, then candidate buffers and counters.
__host__ __device__ constexpr size_t few_tile_lds_bytes(int M, int nq)
{
    return (size_t)nq * (M / 2) * 256 * sizeof(uint16_t) + (size_t)nq * (few_cap(M) + 2) * sizeof(uint32_t);
}

// ONE: the tile has exactly one query (compile-time), so the table base is
// the start of LDS and every table offset folds into the reads.
template <int MM, bool ONE>
__device__ void few_tile_impl(const TileJob &job, char *lds)
{
    constexpr uint32_t SMAX = 255u * MM;
    constexpr int R = few_r(MM);
    constexpr int PASS = few_pass(MM);
    constexpr int CAP = few_cap(MM);
    const int nq = ONE ? 1 : job.nq;
    const uint32_t k = job.k;
    uint16_t *pt = reinterpret_cast<uint16_t *>(lds);                         // [nq][MM/2][256]
    uint32_t *buf = reinterpret_cast<uint32_t *>(pt + nq * (MM / 2) * 256);  // [nq][CAP]
    uint32_t *cnt = buf + nq * CAP;
    uint32_t *bnd = cnt + nq;
    uint32_t *gthr = job.gthr + job.q0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    build_pair_tables<MM>(job.luts + job.q0 * MM * 16, nq, pt, reinterpret_cast<uint8_t *>(buf));
    if (tid < nq) {
        cnt[tid] = 0;
        bnd[tid] = read_bound(&gthr[tid]) + 1u;
    }
    __syncthreads();
    const int64_t r0 = job.r0, r1 = job.r1;
    int pass = 0;
    uint32_t cw[R][MM / 8], nx[R][MM / 8];
    load_rows<MM, R>(job.codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += PASS, ++pass) {
        copy_rows<MM, R>(nx, cw);
        if (base + PASS < r1)   // next pass in flight while this one is computed
            load_rows<MM, R>(job.codes, base + PASS, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[R];
            pair_sums<MM, R, ONE>(reinterpret_cast<const char *>(pt + q * (MM / 2) * 256), cw, s);
            const uint32_t bq = bnd[q];
            const bool largest = job.order.largest(job.q0 + q);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = base + tid + 256 * r;
                const uint32_t d = largest ? SMAX - s[r] : s[r];
                if (n < r1 && d < bq) {
                    const uint32_t pos = atomicAdd(&cnt[q], 1u);
                    buf[q * CAP + pos] = local_key(d, (uint32_t)(n - r0));
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass & 7) == 7;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = cnt[q];
            uint32_t nb = 0xFFFFFFFFu;
            if (c > CAP - PASS) {
                PruneResult pr = prune_local_lds<CAP>(buf + q * CAP, c, k, false);
                if (pr.count > CAP - PASS)
                    pr = prune_local_lds<CAP>(buf + q * CAP, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    publish(&gthr[q], pr.T, bnd[q]);
                }
                nb = pr.T;
            }
            if (lane == 0 && (nb != 0xFFFFFFFFu || refresh)) {
                uint32_t b = bnd[q];
                b = nb < b ? nb : b;
                const uint32_t gb = read_bound(&gthr[q]) + 1u;
                bnd[q] = gb < b ? gb : b;
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4) {
        if (job.lcnt)
            write_local_topk<CAP, true>(buf + q * CAP, cnt[q], k, r0, job.cand + (job.q0 + q) * job.n_rb * (int64_t)k,
                                        &gthr[q], bnd[q], nullptr, nullptr, 0, job.lcnt + job.q0 + q);
        else
            write_local_topk<CAP, true>(buf + q * CAP, cnt[q], k, r0,
                                        job.cand + ((job.q0 + q) * job.n_rb + job.rb) * (int64_t)k,
                                        &gthr[q], bnd[q],
                                        job.ccnt ? job.ccnt + (job.q0 + q) * job.n_rb + job.rb : nullptr,
                                        job.hist ? job.hist + (job.q0 + q) * kHistBins : nullptr, job.hist_shift);
    }
}

// A few-query tile; ONE requires job.nq == 1.
template <int MM, bool ONE>
__device__ void few_tile(const TileJob &job, char *lds)
{
    few_tile_impl<MM, ONE>(job, lds);
}

// ------------------------------------------------------------------ merge

constexpr int kMergeCap = 2048;   // merge buffer (keys)
constexpr int kMergeE = 4;        // keys per thread per merge pass

struct MergeLds {
    uint64_t mb[kMergeCap];
    uint64_t mbound;
    uint32_t mcnt;
    uint32_t misc;
};

// Exact k smallest of the 48-bit keys src[lo, hi) with d <= bound (one
// workgroup): left unsorted in L.mb[0, n), n <= k returned.  With fit
// false the final selection is left to merge_finish: every collected key
// stays (n may exceed k; the k smallest are among them).
__device__ uint32_t merge_collect(MergeLds &L, const uint64_t *__restrict__ src, int64_t lo, int64_t hi,
                                 uint32_t k, uint32_t bound, bool fit = true)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        L.mcnt = 0;
        L.mbound = ((uint64_t)bound + 1u) << 32;   // keys with d <= bound
    }
    __syncthreads();
    for (int64_t c0 = lo; c0 < hi; c0 += 256 * kMergeE) {
        const uint64_t bnd = L.mbound;
#pragma unroll
        for (int e = 0; e < kMergeE; ++e) {
            const int64_t i = c0 + tid + 256 * e;
            if (i < hi) {
                const uint64_t key = src[i];
                if (key < bnd) {
                    const uint32_t pos = atomicAdd(&L.mcnt, 1u);
                    L.mb[pos] = key;
                }
            }
        }
        __syncthreads();
        if (tid < 64 && L.mcnt > kMergeCap - 256 * kMergeE) {
            const uint64_t kth = prune_u64<kMergeCap>(L.mb, L.mcnt, k);
            if (tid == 0) {
                L.mcnt = k;
                L.mbound = kth + 1;
            }
        }
        __syncthreads();
    }
    uint32_t n = L.mcnt;
    if (!fit)
        return n;
    if (tid < 64 && n > k)
        prune_u64_fit<kMergeCap>(L.mb, n, k);
    __syncthreads();
    return n > k ? k : n;
}

// merge_collect (fit false) for a long list whose bound is known to admit
// few keys (at most kMergeCap): one pass with 16 keys per thread in flight
// and no barrier inside, where merge_collect keeps 4 keys per thread in
// flight and meets two barriers per 1024 keys.  If more than kMergeCap keys
// pass the bound after all, it falls back to merge_collect.
__device__ uint32_t merge_collect_wide(MergeLds &L, const uint64_t *__restrict__ src, int64_t n, uint32_t k,
                                       uint32_t bound)
{
    constexpr int W = 8;   // 16-byte loads (two keys) per thread per round
    const int tid = threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(src) & 15) != 0)
        return merge_collect(L, src, 0, n, k, bound, false);
    if (tid == 0)
        L.mcnt = 0;
    __syncthreads();
    const uint64_t bnd = ((uint64_t)bound + 1u) << 32;
    const uint4 *s2 = reinterpret_cast<const uint4 *>(src);
    const int64_t n2 = n / 2;
    for (int64_t p0 = 0; p0 < n2; p0 += 256 * W) {
        uint4 v[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int64_t p = p0 + tid + 256 * w;
            v[w] = p < n2 ? s2[p] : make_uint4(~0u, ~0u, ~0u, ~0u);
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t a = ((uint64_t)v[w].y << 32) | v[w].x, b = ((uint64_t)v[w].w << 32) | v[w].z;
            if (a < bnd) {
                const uint32_t pos = atomicAdd(&L.mcnt, 1u);
                if (pos < kMergeCap)
                    L.mb[pos] = a;
            }
            if (b < bnd) {
                const uint32_t pos = atomicAdd(&L.mcnt, 1u);
                if (pos < kMergeCap)
                    L.mb[pos] = b;
            }
        }
    }
    if (tid == 0 && (n & 1) && src[n - 1] < bnd) {
        const uint32_t pos = atomicAdd(&L.mcnt, 1u);
        if (pos < kMergeCap)
            L.mb[pos] = src[n - 1];
    }
    __syncthreads();
    const uint32_t c = L.mcnt;
    __syncthreads();   // every thread has read the count before a fallback resets it
    if (c > (uint32_t)kMergeCap)
        return merge_collect(L, src, 0, n, k, bound, false);
    return c;
}

// Sorts L.mb[0, n) and writes values (sums, converted back from d) and rows,
// padded to k with 65535 / 0 and -1.
__device__ void merge_emit(MergeLds &L, uint32_t n, uint32_t k, int largest, uint32_t smax,
                           uint16_t *__restrict__ vals, int32_t *__restrict__ idx)
{
    const int tid = threadIdx.x;
    uint32_t P = 1;
    while (P < n)
        P <<= 1;
    for (uint32_t i = n + tid; i < P; i += 256)
        L.mb[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = tid; t < P / 2; t += 256) {
                const uint32_t i = 2 * t - (t & (stride - 1));
                const uint32_t j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = L.mb[i], b = L.mb[j];
                if ((a > b) == asc) {
                    L.mb[i] = b;
                    L.mb[j] = a;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t r = tid; r < k; r += 256) {
        if (r < n) {
            const uint32_t d = (uint32_t)(L.mb[r] >> 32);
            vals[r] = (uint16_t)(largest ? smax - d : d);
            idx[r] = (int32_t)(L.mb[r] & 0xFFFFFFFFu);
        } else {
            vals[r] = (uint16_t)(largest ? 0u : 0xFFFFu);
            idx[r] = -1;
        }
    }
}

// The sorted k smallest of the n distinct keys in L.mb (any n up to
// kMergeCap; the workgroup is synchronised on entry), written as merge_emit
// writes them.  Up to 256 keys: every thread places one key at its rank
// (the number of smaller keys), one pass with no barriers; more: the exact
// k smallest are selected first, then sorted.
__device__ void merge_finish(MergeLds &L, uint32_t n, uint32_t k, int largest, uint32_t smax,
                             uint16_t *__restrict__ vals, int32_t *__restrict__ idx)
{
    const int tid = threadIdx.x;
    if (n > 256) {
        if (tid < 64)
            prune_u64_fit<kMergeCap>(L.mb, n, k);
        __syncthreads();
        merge_emit(L, n > k ? k : n, k, largest, smax, vals, idx);
        return;
    }
    if ((uint32_t)tid < n) {
        const uint64_t key = L.mb[tid];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < n; ++j)
            rank += L.mb[j] < key ? 1u : 0u;
        if (rank < k) {
            const uint32_t d = (uint32_t)(key >> 32);
            vals[rank] = (uint16_t)(largest ? smax - d : d);
            idx[rank] = (int32_t)(key & 0xFFFFFFFFu);
        }
    }
    for (uint32_t r = n + tid; r < k; r += 256) {
        vals[r] = (uint16_t)(largest ? 0u : 0xFFFFu);
        idx[r] = -1;
    }
}

// The first histogram bin at which the running count of candidate keys
// reaches k; its upper edge bounds the query's k-th smallest d (that many
// distinct rows have d at or below it).  One wave; returns `bound` lowered to
// that edge (unchanged if fewer than k keys were counted).
__device__ uint32_t hist_bound(const uint32_t *__restrict__ hq, uint32_t k, int shift, uint32_t bound)
{
    constexpr int PER = kHistBins / 64;
    const int lane = threadIdx.x & 63;
    const uint4 *h = reinterpret_cast<const uint4 *>(hq + lane * PER);
    uint32_t b[PER];
#pragma unroll
    for (int v = 0; v < PER / 4; ++v) {
        const uint4 t = h[v];
        b[4 * v + 0] = t.x;
        b[4 * v + 1] = t.y;
        b[4 * v + 2] = t.z;
        b[4 * v + 3] = t.w;
    }
    uint32_t own = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i)
        own += b[i];
    uint32_t inc = own;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o)
            inc += t;
    }
    const uint64_t hit = __ballot(inc >= k);
    if (hit == 0)
        return bound;
    const int first = (int)__builtin_ctzll(hit);
    int bin = lane * PER + PER - 1;
    uint32_t run = inc - own;
    for (int i = 0; i < PER; ++i) {
        run += b[i];
        if (run >= k) {
            bin = lane * PER + i;
            break;
        }
    }
    const uint32_t edge = (((uint32_t)__shfl(bin, first) + 1u) << shift) - 1u;
    return edge < bound ? edge : bound;
}

// merge_collect over a query's dense candidate list src[0, n_keys).  A
// long list is first bounded by its own histogram of d (h: kHistBins words
// of LDS): the first bin at which the count reaches k bounds the k-th
// smallest d, so that only about k keys are collected and selected; a
// short one (at most 256 keys) is collected whole.
constexpr int64_t kWideListKeys = 4096;

__device__ uint32_t merge_collect_list(MergeLds &L, uint32_t *h, const uint64_t *__restrict__ src, int64_t n_keys,
                                      uint32_t k, int shift, uint32_t bound, bool fit = true)
{
    __shared__ uint32_t s_bound;
    const int tid = threadIdx.x;
    if (n_keys <= 256)   // a short list: collected whole, placed by rank
        return merge_collect(L, src, 0, n_keys, k, bound, fit);
    for (int i = tid; i < kHistBins; i += 256)
        h[i] = 0;
    __syncthreads();
    // Long lists (one query over a large database: thousands of keys) keep
    // 8 keys per thread in flight here and take the wide collect below;
    // short ones (hundreds of keys per query of a large batch) measured
    // faster with the plain loops.
    const bool wide = n_keys > kWideListKeys;
    if (!wide)
        for (int64_t i = tid; i < n_keys; i += 256)
            atomicAdd(&h[(uint32_t)(src[i] >> 32) >> shift], 1u);
    constexpr int B = 8;   // keys per thread in flight
    for (int64_t i0 = 0; wide && i0 < n_keys; i0 += 256 * B) {
        uint64_t kk[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t i = i0 + tid + 256 * b;
            kk[b] = i < n_keys ? src[i] : ~0ull;
        }
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (i0 + tid + 256 * b < n_keys)
                atomicAdd(&h[(uint32_t)(kk[b] >> 32) >> shift], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        const uint32_t b = hist_bound(h, k, shift, bound);
        if (tid == 0)
            s_bound = b;
    }
    __syncthreads();
    if (!fit && wide)   // the histogram's bound admits about k keys
        return merge_collect_wide(L, src, n_keys, k, s_bound);
    return merge_collect(L, src, 0, n_keys, k, s_bound, fit);
}


// Exact r-th smallest of the G uint16 values v[0, G) (G a multiple of 8, v
// 16-byte aligned), by one workgroup of 256 threads: a histogram (h, LDS,
// kHistBins bins of 2^shift values) finds the value's bin and the count
// below it, a second pass counts that bin's values one by one.  Returns
// 0xFFFF when G < r.
__device__ uint32_t select_rank_u16(const uint16_t *__restrict__ v, int64_t G, uint32_t r, int shift, uint32_t *h)
{
    __shared__ uint32_t sub[64];   // one counter per value of the bin (2^shift <= 64)
    __shared__ uint32_t loc[2];    // the bin, the count below it
    const int tid = threadIdx.x;
    for (int i = tid; i < kHistBins; i += 256)
        h[i] = 0;
    if (tid < 64)
        sub[tid] = 0;
    __syncthreads();
    const uint4 *d = reinterpret_cast<const uint4 *>(v);   // 8 values per load
    for (int64_t i = tid; i < G / 8; i += 256) {
        const uint4 t = d[i];
        const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            atomicAdd(&h[(w[j] & 0xFFFFu) >> shift], 1u);
            atomicAdd(&h[(w[j] >> 16) >> shift], 1u);
        }
    }
    __syncthreads();
    if (tid < 64) {
        constexpr int PER = kHistBins / 64;
        uint32_t own = 0;
        for (int i = 0; i < PER; ++i)
            own += h[tid * PER + i];
        uint32_t inc = own;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (tid >= o)
                inc += t;
        }
        const uint64_t hit = __ballot(inc >= r);
        if (tid == (hit ? (int)__builtin_ctzll(hit) : 0)) {
            uint32_t run = inc - own, bin = 0xFFFFFFFFu;
            for (int i = 0; hit && i < PER; ++i) {
                const uint32_t c = h[tid * PER + i];
                if (run + c >= r) {
                    bin = (uint32_t)(tid * PER + i);
                    break;
                }
                run += c;
            }
            loc[0] = bin;
            loc[1] = run;
        }
    }
    __syncthreads();
    const uint32_t bin = loc[0];
    if (bin == 0xFFFFFFFFu)
        return 0xFFFFu;
    for (int64_t i = tid; i < G / 8; i += 256) {
        const uint4 t = d[i];
        const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t a = w[j] & 0xFFFFu, b = w[j] >> 16;
            if ((a >> shift) == bin)
                atomicAdd(&sub[a & ((1u << shift) - 1u)], 1u);
            if ((b >> shift) == bin)
                atomicAdd(&sub[b & ((1u << shift) - 1u)], 1u);
        }
    }
    __syncthreads();
    uint32_t run = loc[1], j = 0;
    while (run + sub[j] < r)   // the bin holds the r-th value: ends at j < 2^shift
        run += sub[j++];
    return (bin << shift) + j;
}

}  // namespace bolt
