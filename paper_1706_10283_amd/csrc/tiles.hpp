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

// Few-query tiles (pair tables; see few.hip).
constexpr int kFewR = 4;              // rows per lane per pass
constexpr int kFewPass = 256 * kFewR;
constexpr int kFewCap = 2 * kFewPass; // candidate slots per query

struct TileJob {
    const uint8_t *codes;   // the database's codes [N][M/2]
    const uint8_t *luts;    // the database's tables [Q][M][16]
    uint64_t *cand;         // the database's candidates [Q][n_rb][k]
    uint32_t *gthr;         // the database's bounds [Q]
    int64_t r0, r1;         // rows of the tile
    int64_t rb;             // row-block index of the tile
    int64_t n_rb;           // row blocks of the database
    int64_t q0;             // first query of the tile
    int nq;                 // queries of the tile
    uint32_t k;
    int largest;
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per 16-bit lane max(a - b, 0): nonzero lanes are those with b < a.
__device__ __forceinline__ uint32_t sub_sat_u16x2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}

__device__ __forceinline__ uint32_t read_bound(const uint32_t *g) { return __atomic_load_n(g, __ATOMIC_RELAXED); }

__device__ __forceinline__ void publish(uint32_t *g, uint32_t T)
{
    if (T <= 0xFFFFu)
        atomicMin(g, T);
}

// Final exact local top-k of one query (one wave), written as 48-bit keys.
template <int CAP, bool LDS_PRUNE>
__device__ void write_local_topk(uint32_t *buf, uint32_t n, uint32_t k, int64_t r0,
                                 uint64_t *__restrict__ dst, uint32_t *gthr_q)
{
    const int lane = threadIdx.x & 63;
    if (n > k) {
        const PruneResult pr = LDS_PRUNE ? prune_local_lds<CAP>(buf, n, k, true)
                                         : prune_local<CAP>(buf, n, k, true);
        n = pr.count;
        if (lane == 0)
            publish(gthr_q, pr.T);
    }
    for (uint32_t j = lane; j < k; j += 64) {
        uint64_t key = ~0ull;
        if (j < n) {
            const uint32_t lk = buf[j];
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
    const int largest = job.largest;
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
    for (int64_t base = r0; base < r1; base += 256, ++pass) {
        const int64_t n = base + tid;
        const bool valid = n < r1;
        uint32_t cw[NW];
        if (valid)
            load_row<MM>(job.codes, n, cw);
        else
#pragma unroll
            for (int v = 0; v < NW; ++v)
                cw[v] = 0;
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
                const uint32_t hit = sub_sat_u16x2(bp.x, dd[0]) | sub_sat_u16x2(bp.y, dd[1]) |
                                     sub_sat_u16x2(bp.z, dd[2]) | sub_sat_u16x2(bp.w, dd[3]);
                if (valid && hit) {
#pragma unroll
                    for (int qq = 0; qq < 8; ++qq) {
                        const int q = gg * QG + qq;
                        const uint32_t d = (dd[qq >> 1] >> (16 * (qq & 1))) & 0xFFFFu;
                        if (d < (uint32_t)L.bnd16[q]) {
                            const uint32_t pos = atomicAdd(&L.cnt[q], 1u);
                            L.buf[q * CAP + pos] = local_key(d, local);
                        }
                    }
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass % kRefresh) == kRefresh - 1;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = L.cnt[q];
            uint32_t nb = 0xFFFFFFFFu;
            if (c > CAP - 256) {
                PruneResult pr = prune_local<CAP>(L.buf + q * CAP, c, k, false);
                if (pr.count > CAP - 256)
                    pr = prune_local<CAP>(L.buf + q * CAP, pr.count, k, true);
                if (lane == 0) {
                    L.cnt[q] = pr.count;
                    publish(&job.gthr[q0 + q], pr.T);
                }
                nb = pr.T;
            }
            if (lane == 0 && (nb != 0xFFFFFFFFu || refresh)) {
                uint32_t b = L.bnd[q];
                b = nb < b ? nb : b;
                const uint32_t gb = read_bound(&job.gthr[q0 + q]) + 1u;
                b = gb < b ? gb : b;
                L.bnd[q] = b;
                L.bnd16[q] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4)
        write_local_topk<CAP, false>(L.buf + q * CAP, L.cnt[q], k, r0,
                                     job.cand + ((q0 + q) * job.n_rb + job.rb) * (int64_t)k,
                                     &job.gthr[q0 + q]);
}

// ------------------------------------------------------------------ few queries

template <int MM>
__device__ __forceinline__ void build_pair_tables(const uint8_t *__restrict__ luts, int nq, uint16_t *pt)
{
    constexpr int NP = MM / 2;
    for (int e = threadIdx.x; e < nq * NP * 256; e += 256) {
        const int b = e & 255, p = (e >> 8) % NP, q = (e >> 8) / NP;
        const uint8_t *l = luts + ((int64_t)q * MM + 2 * p) * 16;
        pt[e] = (uint16_t)(l[b & 15] + l[16 + (b >> 4)]);
    }
}

// Sums of one query for the kFewR rows held in cw (pair tables of the query at tq).
template <int MM>
__device__ __forceinline__ void pair_sums(const uint16_t *tq, const uint32_t (&cw)[kFewR][MM / 8],
                                          uint32_t (&s)[kFewR])
{
    const char *tb = reinterpret_cast<const char *>(tq);
    uint32_t part[kFewR];
#pragma unroll
    for (int r = 0; r < kFewR; ++r)
        part[r] = 0;
    // one code dword (four pairs) per step keeps 4*kFewR reads in flight and
    // the register count low
#pragma unroll 1
    for (int t = 0; t < MM / 8; ++t) {
        uint32_t w[kFewR];
#pragma unroll
        for (int r = 0; r < kFewR; ++r) {
            w[r] = cw[r][0];
#pragma unroll
            for (int v = 1; v < MM / 8; ++v)
                w[r] = (t == v) ? cw[r][v] : w[r];
        }
        const char *tt = tb + t * 4 * 512;
        uint32_t v[kFewR][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < kFewR; ++r) {
                const uint32_t byte = (w[r] >> (8 * j)) & 0xFFu;
                v[r][j] = *reinterpret_cast<const uint16_t *>(tt + j * 512 + 2 * byte);
            }
#pragma unroll
        for (int r = 0; r < kFewR; ++r)
            part[r] += v[r][0] + v[r][1] + v[r][2] + v[r][3];
    }
#pragma unroll
    for (int r = 0; r < kFewR; ++r)
        s[r] = part[r];
}

template <int MM>
__device__ __forceinline__ void load_rows4(const uint8_t *__restrict__ codes, int64_t base, int64_t r1,
                                           uint32_t (&cw)[kFewR][MM / 8])
{
#pragma unroll
    for (int r = 0; r < kFewR; ++r) {
        const int64_t n = base + threadIdx.x + 256 * r;
        if (n < r1)
            load_row<MM>(codes, n, cw[r]);
        else
#pragma unroll
            for (int v = 0; v < MM / 8; ++v)
                cw[r][v] = 0;
    }
}

template <int MM>
__device__ __forceinline__ void copy_rows4(const uint32_t (&a)[kFewR][MM / 8], uint32_t (&b)[kFewR][MM / 8])
{
#pragma unroll
    for (int r = 0; r < kFewR; ++r)
#pragma unroll
        for (int v = 0; v < MM / 8; ++v)
            b[r][v] = a[r][v];
}

// LDS of a few-query tile: pair tables, then candidate buffers and counters.
__host__ __device__ constexpr size_t few_tile_lds_bytes(int M, int nq)
{
    return (size_t)nq * (M / 2) * 256 * sizeof(uint16_t) + (size_t)nq * (kFewCap + 2) * sizeof(uint32_t);
}

template <int MM>
__device__ void few_tile(const TileJob &job, char *lds)
{
    constexpr uint32_t SMAX = 255u * MM;
    const int nq = job.nq;
    const uint32_t k = job.k;
    const int largest = job.largest;
    uint16_t *pt = reinterpret_cast<uint16_t *>(lds);                         // [nq][MM/2][256]
    uint32_t *buf = reinterpret_cast<uint32_t *>(pt + nq * (MM / 2) * 256);  // [nq][kFewCap]
    uint32_t *cnt = buf + nq * kFewCap;
    uint32_t *bnd = cnt + nq;
    uint32_t *gthr = job.gthr + job.q0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    build_pair_tables<MM>(job.luts + job.q0 * MM * 16, nq, pt);
    if (tid < nq) {
        cnt[tid] = 0;
        bnd[tid] = read_bound(&gthr[tid]) + 1u;
    }
    __syncthreads();
    const int64_t r0 = job.r0, r1 = job.r1;
    int pass = 0;
    uint32_t cw[kFewR][MM / 8], nx[kFewR][MM / 8];
    load_rows4<MM>(job.codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += kFewPass, ++pass) {
        copy_rows4<MM>(nx, cw);
        if (base + kFewPass < r1)   // next pass in flight while this one is computed
            load_rows4<MM>(job.codes, base + kFewPass, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[kFewR];
            pair_sums<MM>(pt + q * (MM / 2) * 256, cw, s);
            const uint32_t bq = bnd[q];
#pragma unroll
            for (int r = 0; r < kFewR; ++r) {
                const int64_t n = base + tid + 256 * r;
                const uint32_t d = largest ? SMAX - s[r] : s[r];
                if (n < r1 && d < bq) {
                    const uint32_t pos = atomicAdd(&cnt[q], 1u);
                    buf[q * kFewCap + pos] = local_key(d, (uint32_t)(n - r0));
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass & 7) == 7;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = cnt[q];
            uint32_t nb = 0xFFFFFFFFu;
            if (c > kFewCap - kFewPass) {
                PruneResult pr = prune_local_lds<kFewCap>(buf + q * kFewCap, c, k, false);
                if (pr.count > kFewCap - kFewPass)
                    pr = prune_local_lds<kFewCap>(buf + q * kFewCap, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    publish(&gthr[q], pr.T);
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
    for (int q = wave; q < nq; q += 4)
        write_local_topk<kFewCap, true>(buf + q * kFewCap, cnt[q], k, r0,
                                        job.cand + ((job.q0 + q) * job.n_rb + job.rb) * (int64_t)k,
                                        &gthr[q]);
}

// ------------------------------------------------------------------ merge

constexpr int kMergeCap = 2048;   // merge buffer (keys)
constexpr int kMergeE = 4;        // keys per thread per merge pass

// Exact k smallest of the 48-bit keys src[lo, hi) with d <= bound (one
// workgroup).  out != NULL: the k keys (unsorted, ~0 padded) are written to
// out; otherwise they are sorted and written as values (sum, converted back
// from d) and rows, padded with 65535 / 0 and -1.
__device__ void merge_keys(const uint64_t *__restrict__ src, int64_t lo, int64_t hi, uint32_t k,
                           uint32_t bound, uint64_t *__restrict__ out, int largest, uint32_t smax,
                           uint16_t *__restrict__ vals, int32_t *__restrict__ idx)
{
    __shared__ uint64_t mb[kMergeCap];
    __shared__ uint32_t mcnt;
    __shared__ uint64_t mbound;
    const int tid = threadIdx.x;
    if (tid == 0) {
        mcnt = 0;
        mbound = ((uint64_t)bound + 1u) << 32;   // keys with d <= bound
    }
    __syncthreads();
    for (int64_t c0 = lo; c0 < hi; c0 += 256 * kMergeE) {
        const uint64_t bnd = mbound;
#pragma unroll
        for (int e = 0; e < kMergeE; ++e) {
            const int64_t i = c0 + tid + 256 * e;
            if (i < hi) {
                const uint64_t key = src[i];
                if (key < bnd) {
                    const uint32_t pos = atomicAdd(&mcnt, 1u);
                    mb[pos] = key;
                }
            }
        }
        __syncthreads();
        if (tid < 64 && mcnt > kMergeCap - 256 * kMergeE) {
            const uint64_t kth = prune_u64<kMergeCap>(mb, mcnt, k);
            if (tid == 0) {
                mcnt = k;
                mbound = kth + 1;
            }
        }
        __syncthreads();
    }
    uint32_t n = mcnt;
    if (tid < 64 && n > k)
        prune_u64<kMergeCap>(mb, n, k);
    __syncthreads();
    if (n > k)
        n = k;
    if (out) {
        for (uint32_t r = tid; r < k; r += 256)
            out[r] = r < n ? mb[r] : ~0ull;
        return;
    }
    uint32_t P = 1;
    while (P < n)
        P <<= 1;
    for (uint32_t i = n + tid; i < P; i += 256)
        mb[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = tid; t < P / 2; t += 256) {
                const uint32_t i = 2 * t - (t & (stride - 1));
                const uint32_t j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = mb[i], b = mb[j];
                if ((a > b) == asc) {
                    mb[i] = b;
                    mb[j] = a;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t r = tid; r < k; r += 256) {
        if (r < n) {
            const uint32_t d = (uint32_t)(mb[r] >> 32);
            vals[r] = (uint16_t)(largest ? smax - d : d);
            idx[r] = (int32_t)(mb[r] & 0xFFFFFFFFu);
        } else {
            vals[r] = (uint16_t)(largest ? 0u : 0xFFFFu);
            idx[r] = -1;
        }
    }
}

}  // namespace bolt
