// Scan fused with top-k selection (Sec. 3.1 scan; Sec. 1.2 the k closest
// vectors) for gfx950: the [Q][N] sums are never written to memory.
//
// Stage 1, one workgroup per (row block of <= 65536 rows, query block): the
// scan of the grouped (many queries) or few-query kernel computes the sums;
// each sum is compared with its query's bound and the rare survivors are
// appended to that query's LDS buffer (see topk_device.hpp).  Between passes
// of 256 rows the buffers that could overflow are pruned, one wave per query.
// A pruned bound is also published to the other workgroups with a global
// atomicMin (any row whose d exceeds a workgroup's k-th smallest d cannot be
// in the global top-k), and every workgroup folds the published bounds into
// its own every few passes.  The bounds only decide which rows are kept as
// candidates, never the result, so the answer is exact and independent of
// timing.  Each workgroup finally writes its exact local top-k per query.
//
// Stage 2, one workgroup per query: the row blocks' candidates are merged by
// the same append-and-prune scheme on 48-bit keys (d << 32 | row) and the k
// survivors are sorted.
//
// Workgroups of one row block are placed on one XCD (consecutive workgroup
// ids are dispatched round-robin to the 8 XCDs), so each XCD's L2 holds only
// its share of the codes while all query blocks reuse them.
#include "common.hpp"
#include "scan_common.hpp"
#include "topk_device.hpp"

namespace {

using bolt::code_at;
using bolt::load_row;
using bolt::PruneResult;

constexpr int kCap = 512;                 // candidate slots per query (grouped kernel)
constexpr int kCapSmall = 2048;           // candidate slots per query (few-query kernel)
constexpr int kRowsPerBlock = 16384;      // rows per workgroup (<= 65536: 16-bit local rows)
constexpr int kMergeCap = 2048;           // merge buffer (keys)
constexpr int kMergeE = 4;                // keys per thread per merge pass
constexpr int kRefresh = 8;               // passes between reads of the published bounds

__device__ __forceinline__ uint32_t read_bound(const uint32_t *g)
{
    return __atomic_load_n(g, __ATOMIC_RELAXED);
}

// Publish and fold: after a prune with result T (k or more keys with d <= T in
// this workgroup), rows with d > T are useless everywhere.
__device__ __forceinline__ void publish(uint32_t *gthr, uint32_t T)
{
    if (T <= 0xFFFFu)
        atomicMin(gthr, T);
}

// Final local selection of one query and write-out of its k candidates as
// 48-bit keys; missing entries are ~0.
template <int CAP>
__device__ void write_local_topk(uint32_t *buf, uint32_t n, uint32_t k, int64_t r0,
                                 uint64_t *__restrict__ dst)
{
    const int lane = threadIdx.x & 63;
    if (n > k)
        n = bolt::prune_local<CAP>(buf, n, k, true).count;
    for (uint32_t j = lane; j < k; j += 64) {
        uint64_t key = ~0ull;
        if (j < n) {
            const uint32_t lk = buf[j];
            key = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
        }
        dst[j] = key;
    }
}

// Decode the tile of workgroup `w`: XCD-major placement of row blocks.
__device__ __forceinline__ void tile_of(int w, int n_qb, int &qb, int &rb)
{
    const int xcd = w & 7, i = w >> 3;
    qb = i % n_qb;
    rb = (i / n_qb) * 8 + xcd;
}

// ------------------------------------------------------------------ many queries

template <int MM, int NG>
__global__ __launch_bounds__(256) void scan_topk_grouped_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    uint32_t k, uint32_t flip, int n_rb, int n_qb, uint64_t *__restrict__ cand,
    uint32_t *__restrict__ gthr)
{
    constexpr int QG = 8;
    constexpr int QB = QG * NG;
    constexpr int GROUP_BYTES = MM * 256;
    constexpr int NW = MM / 8;
    __shared__ uint4 tab[NG * GROUP_BYTES / 16];
    __shared__ uint32_t buf[QB * kCap];
    __shared__ uint32_t cnt[QB];
    __shared__ __attribute__((aligned(16))) uint32_t bnd[QB];

    int qb, rb;
    tile_of(blockIdx.x, n_qb, qb, rb);
    if (rb >= n_rb)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q0 = (int64_t)qb * QB;
    const int nq = (int)((Q - q0) < QB ? (Q - q0) : QB);

    uint16_t *tab16 = reinterpret_cast<uint16_t *>(tab);
    for (int e = tid; e < NG * MM * 16 * QG; e += 256) {
        const int qq = e & 7, c = (e >> 3) & 15;
        const int m = (e >> 7) % MM, g = (e >> 7) / MM;
        const int q = g * QG + qq;
        tab16[e] = q < nq ? luts[(q0 + q) * MM * 16 + m * 16 + c] : (uint16_t)0;
    }
    for (int q = tid; q < QB; q += 256) {
        cnt[q] = 0;
        bnd[q] = q < nq ? read_bound(&gthr[q0 + q]) + 1u : 0u;
    }
    __syncthreads();

    const int64_t r0 = (int64_t)rb * kRowsPerBlock;
    const int64_t r1 = (r0 + kRowsPerBlock) < N ? (r0 + kRowsPerBlock) : N;
    const char *tabb = reinterpret_cast<const char *>(tab);
    int pass = 0;
    for (int64_t base = r0; base < r1; base += 256, ++pass) {
        const int64_t n = base + tid;
        const bool valid = n < r1;
        uint32_t cw[NW];
        if (valid)
            load_row<MM>(codes, n, cw);
        else
#pragma unroll
            for (int v = 0; v < NW; ++v)
                cw[v] = 0;
        const uint32_t local = (uint32_t)(n - r0);
#pragma unroll 1
        for (int g = 0; g < NG; ++g) {
            const char *tg = tabb + g * GROUP_BYTES;
            uint32_t acc[4] = {0, 0, 0, 0};
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
                    const uint4 a = *reinterpret_cast<const uint4 *>(tt + am);
                    const uint4 b = *reinterpret_cast<const uint4 *>(tt + am1);
                    acc[0] += a.x + b.x;
                    acc[1] += a.y + b.y;
                    acc[2] += a.z + b.z;
                    acc[3] += a.w + b.w;
                }
            }
            const uint4 bl = *reinterpret_cast<const uint4 *>(&bnd[g * QG]);
            const uint4 bh = *reinterpret_cast<const uint4 *>(&bnd[g * QG + 4]);
            const uint32_t bq[8] = {bl.x, bl.y, bl.z, bl.w, bh.x, bh.y, bh.z, bh.w};
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
                const uint32_t d = ((acc[qq >> 1] >> (16 * (qq & 1))) & 0xFFFFu) ^ flip;
                if (valid && d < bq[qq]) {
                    const int q = g * QG + qq;
                    const uint32_t pos = atomicAdd(&cnt[q], 1u);
                    buf[q * kCap + pos] = bolt::local_key(d, local);
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass % kRefresh) == kRefresh - 1;
        for (int q = wave; q < nq; q += 4) {
            uint32_t c = cnt[q];
            if (c > kCap - 256) {
                PruneResult pr = bolt::prune_local<kCap>(buf + q * kCap, c, k, false);
                if (pr.count > kCap - 256)
                    pr = bolt::prune_local<kCap>(buf + q * kCap, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    publish(&gthr[q0 + q], pr.T);
                    uint32_t b = bnd[q];
                    b = pr.T < b ? pr.T : b;
                    const uint32_t gb = read_bound(&gthr[q0 + q]) + 1u;
                    bnd[q] = gb < b ? gb : b;
                }
            } else if (refresh && lane == 0) {
                const uint32_t gb = read_bound(&gthr[q0 + q]) + 1u;
                if (gb < bnd[q])
                    bnd[q] = gb;
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4)
        write_local_topk<kCap>(buf + q * kCap, cnt[q], k, r0,
                               cand + ((q0 + q) * n_rb + rb) * (int64_t)k);
}

// ------------------------------------------------------------------ few queries

template <int MM>
__global__ __launch_bounds__(256) void scan_topk_small_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int nq,
    uint32_t k, uint32_t flip, int n_rb, uint64_t *__restrict__ cand, uint32_t *__restrict__ gthr)
{
    constexpr int R = (128 / MM) < 1 ? 1 : ((128 / MM) > 4 ? 4 : (128 / MM));
    constexpr int NW = MM / 8;
    constexpr int kQ = bolt::kSmallQ - 1;
    __shared__ uint4 tab[kQ * MM];
    __shared__ uint32_t buf[kQ * kCapSmall];
    __shared__ uint32_t cnt[kQ];
    __shared__ uint32_t bnd[kQ];

    const int rb = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint4 *src = reinterpret_cast<const uint4 *>(luts);
    for (int e = tid; e < nq * MM; e += 256)
        tab[e] = src[e];
    if (tid < kQ) {
        cnt[tid] = 0;
        bnd[tid] = tid < nq ? read_bound(&gthr[tid]) + 1u : 0u;
    }
    __syncthreads();
    const uint8_t *tb = reinterpret_cast<const uint8_t *>(tab);
    const int64_t r0 = (int64_t)rb * kRowsPerBlock;
    const int64_t r1 = (r0 + kRowsPerBlock) < N ? (r0 + kRowsPerBlock) : N;
    int pass = 0;
    for (int64_t base = r0; base < r1; base += 256 * R, ++pass) {
        uint32_t cw[R][NW];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t n = base + tid + 256 * r;
            if (n < r1)
                load_row<MM>(codes, n, cw[r]);
            else
#pragma unroll
                for (int v = 0; v < NW; ++v)
                    cw[r][v] = 0;
        }
        for (int q = 0; q < nq; ++q) {
            const uint8_t *tq = tb + q * MM * 16;
            const uint32_t bq = bnd[q];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = base + tid + 256 * r;
                uint32_t s = 0;
#pragma unroll
                for (int m = 0; m < MM; m += 2)
                    s += (uint32_t)tq[m * 16 + code_at<MM>(cw[r], m)] +
                         (uint32_t)tq[(m + 1) * 16 + code_at<MM>(cw[r], m + 1)];
                const uint32_t d = s ^ flip;
                if (n < r1 && d < bq) {
                    const uint32_t pos = atomicAdd(&cnt[q], 1u);
                    buf[q * kCapSmall + pos] = bolt::local_key(d, (uint32_t)(n - r0));
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass % kRefresh) == kRefresh - 1;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = cnt[q];
            if (c > kCapSmall - 256 * R) {
                PruneResult pr = bolt::prune_local<kCapSmall>(buf + q * kCapSmall, c, k, false);
                if (pr.count > kCapSmall - 256 * R)
                    pr = bolt::prune_local<kCapSmall>(buf + q * kCapSmall, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    publish(&gthr[q], pr.T);
                    uint32_t b = bnd[q];
                    b = pr.T < b ? pr.T : b;
                    const uint32_t gb = read_bound(&gthr[q]) + 1u;
                    bnd[q] = gb < b ? gb : b;
                }
            } else if (refresh && lane == 0) {
                const uint32_t gb = read_bound(&gthr[q]) + 1u;
                if (gb < bnd[q])
                    bnd[q] = gb;
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4)
        write_local_topk<kCapSmall>(buf + q * kCapSmall, cnt[q], k, r0,
                                    cand + ((int64_t)q * n_rb + rb) * (int64_t)k);
}

// ------------------------------------------------------------------ merge

__global__ __launch_bounds__(256) void topk_merge_kernel(const uint64_t *__restrict__ cand,
                                                         int64_t per_query, uint32_t k,
                                                         uint32_t flip, uint16_t *__restrict__ vals,
                                                         int32_t *__restrict__ idx)
{
    __shared__ uint64_t mb[kMergeCap];
    __shared__ uint32_t mcnt;
    __shared__ uint64_t mbound;
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x;
    const uint64_t *src = cand + q * per_query;
    if (tid == 0) {
        mcnt = 0;
        mbound = 1ull << 48;   // keys are < 2^48; missing entries (~0) never enter
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < per_query; c0 += 256 * kMergeE) {
        const uint64_t bound = mbound;
#pragma unroll
        for (int e = 0; e < kMergeE; ++e) {
            const int64_t i = c0 + tid + 256 * e;
            if (i < per_query) {
                const uint64_t key = src[i];
                if (key < bound) {
                    const uint32_t pos = atomicAdd(&mcnt, 1u);
                    mb[pos] = key;
                }
            }
        }
        __syncthreads();
        if (tid < 64 && mcnt > kMergeCap - 256 * kMergeE) {
            const uint64_t kth = bolt::prune_u64<kMergeCap>(mb, mcnt, k);
            if (tid == 0) {
                mcnt = k;
                mbound = kth + 1;
            }
        }
        __syncthreads();
    }
    uint32_t n = mcnt;
    if (tid < 64 && n > k)
        bolt::prune_u64<kMergeCap>(mb, n, k);
    __syncthreads();
    if (n > k)
        n = k;
    // sort the survivors (bitonic over the next power of two)
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
            vals[q * k + r] = (uint16_t)((uint32_t)(mb[r] >> 32) ^ flip);
            idx[q * k + r] = (int32_t)(mb[r] & 0xFFFFFFFFu);
        } else {
            vals[q * k + r] = (uint16_t)(flip ? 0u : 0xFFFFu);
            idx[q * k + r] = -1;
        }
    }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        p[i] = v;
}

template <int MM>
constexpr int groups_for()
{
    // LDS: NG * (MM*256 table bytes + 8*kCap*4 buffer bytes) <= ~64 KB
    return MM <= 32 ? 2 : 1;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct FusedPlan {
    bool ok = false;
    int kind = 0;        // 1 few-query, 2 grouped
    int n_rb = 0, n_qb = 0, qb_size = 0;
    size_t cand_bytes = 0, gthr_bytes = 0;
};

FusedPlan plan_fused(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    FusedPlan p;
    const bool tuned_M = (M == 8 || M == 16 || M == 32 || M == 64);
    if (!tuned_M || !vec_ok || k > kCap - 256 || N <= 0 || Q <= 0)
        return p;
    p.n_rb = (int)((N + kRowsPerBlock - 1) / kRowsPerBlock);
    if (Q < bolt::kSmallQ) {
        p.kind = 1;
        p.n_qb = 1;
        p.qb_size = (int)Q;
    } else {
        p.kind = 2;
        int ng = 1;
        switch (M) {
        case 8: ng = groups_for<8>(); break;
        case 16: ng = groups_for<16>(); break;
        case 32: ng = groups_for<32>(); break;
        case 64: ng = groups_for<64>(); break;
        }
        p.qb_size = 8 * ng;
        p.n_qb = (int)((Q + p.qb_size - 1) / p.qb_size);
        if ((int64_t)p.n_qb * ((p.n_rb + 7) / 8) * 8 > INT32_MAX)
            return p;
    }
    p.cand_bytes = align256((size_t)Q * p.n_rb * k * sizeof(uint64_t));
    p.gthr_bytes = align256((size_t)Q * sizeof(uint32_t));
    p.ok = true;
    return p;
}

template <int MM>
void launch_fused(const FusedPlan &p, const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q,
                  int k, uint32_t flip, uint64_t *cand, uint32_t *gthr, hipStream_t s)
{
    if (p.kind == 1) {
        hipLaunchKernelGGL(scan_topk_small_kernel<MM>, dim3(p.n_rb), dim3(256), 0, s, codes, N, luts,
                           (int)Q, (uint32_t)k, flip, p.n_rb, cand, gthr);
    } else {
        constexpr int NG = groups_for<MM>();
        const int rb_pad = (p.n_rb + 7) / 8 * 8;
        hipLaunchKernelGGL((scan_topk_grouped_kernel<MM, NG>), dim3(p.n_qb * rb_pad), dim3(256), 0, s,
                           codes, N, luts, Q, (uint32_t)k, flip, p.n_rb, p.n_qb, cand, gthr);
    }
}

}  // namespace

namespace bolt {

size_t fused_ws_bytes(int64_t N, int M, int64_t Q, int k)
{
    FusedPlan p = plan_fused(N, M, Q, k, true);
    if (!p.ok)
        return 0;
    return p.cand_bytes + p.gthr_bytes;
}

// Fused scan + top-k; returns BOLT_ERR_UNSUPPORTED when the shape has no fused kernel.
int scan_topk_fused(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                    bool largest, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
                    hipStream_t s)
{
    const bool vec_ok = aligned(codes, 16) && aligned(luts, 16);
    FusedPlan p = plan_fused(N, M, Q, k, vec_ok);
    if (!p.ok)
        return BOLT_ERR_UNSUPPORTED;
    if (ws_bytes < p.cand_bytes + p.gthr_bytes || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "fused scan+top-k needs %zu workspace bytes",
                    p.cand_bytes + p.gthr_bytes);
    uint64_t *cand = reinterpret_cast<uint64_t *>(ws);
    uint32_t *gthr = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + p.cand_bytes);
    const uint32_t flip = largest ? 0xFFFFu : 0u;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, gthr, Q,
                       0xFFFFu);
    switch (M) {
    case 8: launch_fused<8>(p, codes, N, luts, Q, k, flip, cand, gthr, s); break;
    case 16: launch_fused<16>(p, codes, N, luts, Q, k, flip, cand, gthr, s); break;
    case 32: launch_fused<32>(p, codes, N, luts, Q, k, flip, cand, gthr, s); break;
    case 64: launch_fused<64>(p, codes, N, luts, Q, k, flip, cand, gthr, s); break;
    }
    hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)Q), dim3(256), 0, s, cand,
                       (int64_t)p.n_rb * k, (uint32_t)k, flip, vals, idx);
    return check_launch("bolt_scan_topk (fused)");
}

}  // namespace bolt
