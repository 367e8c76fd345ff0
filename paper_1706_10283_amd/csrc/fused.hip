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

constexpr int kRowsPerBlock = 16384;      // rows per workgroup (<= 65536: 16-bit local rows)
constexpr int kMergeCap = 2048;           // merge buffer (keys)
constexpr int kMergeE = 4;                // keys per thread per merge pass
constexpr int64_t kMergeChunk = 16384;    // keys per first-level merge workgroup
constexpr int kRefresh = 8;               // passes between reads of the published bounds

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per 16-bit lane max(a - b, 0): nonzero lanes are those with b < a.
__device__ __forceinline__ uint32_t sub_sat_u16x2(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}

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
                                 uint64_t *__restrict__ dst, uint32_t *gthr)
{
    const int lane = threadIdx.x & 63;
    if (n > k) {
        const PruneResult pr = bolt::prune_local<CAP>(buf, n, k, true);
        n = pr.count;
        if (lane == 0)
            publish(gthr, pr.T);
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

// Decode the tile of workgroup `w`: XCD-major placement of row blocks.
__device__ __forceinline__ void tile_of(int w, int n_qb, int &qb, int &rb)
{
    const int xcd = w & 7, i = w >> 3;
    qb = i % n_qb;
    rb = (i / n_qb) * 8 + xcd;
}

// ------------------------------------------------------------------ many queries

// d of a sum s: s itself (k smallest), or smax - s (k largest), smax = 255 * M,
// so that d <= 65280 < 0xFFFF and every bound fits in 16 bits.
template <int MM, int NG, int CAP>
__global__ __launch_bounds__(256) void scan_topk_grouped_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    uint32_t k, int largest, int n_rb, int n_qb, uint64_t *__restrict__ cand,
    uint32_t *__restrict__ gthr)
{
    constexpr int QG = 8;
    constexpr int QB = QG * NG;
    constexpr int GROUP_BYTES = MM * 256;
    constexpr int NW = MM / 8;
    constexpr int GU = NG >= 2 ? 2 : 1;
    constexpr uint32_t SMAX = 255u * MM;
    constexpr uint32_t SMAX2 = SMAX | (SMAX << 16);
    __shared__ uint4 tab[NG * GROUP_BYTES / 16];
    __shared__ uint32_t buf[QB * CAP];
    __shared__ uint32_t cnt[QB];
    __shared__ uint32_t bnd[QB];                                   // exclusive bound on d
    __shared__ __attribute__((aligned(16))) uint16_t bnd16[QB];    // the same, as packed lanes

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
        const uint32_t b = q < nq ? read_bound(&gthr[q0 + q]) + 1u : 0u;
        cnt[q] = 0;
        bnd[q] = b;
        bnd16[q] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
    }
    __syncthreads();

    const int64_t r0 = (int64_t)rb * kRowsPerBlock;
    const int64_t r1 = (r0 + kRowsPerBlock) < N ? (r0 + kRowsPerBlock) : N;
    const char *tabb = reinterpret_cast<const char *>(tab);
    const uint32_t *bnd2 = reinterpret_cast<const uint32_t *>(bnd16);
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
                        if (d < (uint32_t)bnd16[q]) {
                            const uint32_t pos = atomicAdd(&cnt[q], 1u);
                            buf[q * CAP + pos] = bolt::local_key(d, local);
                        }
                    }
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass % kRefresh) == kRefresh - 1;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = cnt[q];
            uint32_t nb = 0xFFFFFFFFu;
            if (c > CAP - 256) {
                PruneResult pr = bolt::prune_local<CAP>(buf + q * CAP, c, k, false);
                if (pr.count > CAP - 256)
                    pr = bolt::prune_local<CAP>(buf + q * CAP, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    publish(&gthr[q0 + q], pr.T);
                }
                nb = pr.T;
            }
            if (lane == 0 && (nb != 0xFFFFFFFFu || refresh)) {
                uint32_t b = bnd[q];
                b = nb < b ? nb : b;
                const uint32_t gb = read_bound(&gthr[q0 + q]) + 1u;
                b = gb < b ? gb : b;
                bnd[q] = b;
                bnd16[q] = (uint16_t)(b < 0xFFFFu ? b : 0xFFFFu);
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4)
        write_local_topk<CAP>(buf + q * CAP, cnt[q], k, r0,
                              cand + ((q0 + q) * n_rb + rb) * (int64_t)k, &gthr[q0 + q]);
}

// ------------------------------------------------------------------ merge

// One workgroup per (query, chunk of a query's candidate keys).  Keys with
// d above the query's final published bound cannot be in its top-k and are
// skipped.  final_out = 0: the chunk's exact k smallest keys go to dst[q][chunk][k]
// (unsorted, ~0 padded); final_out = 1 (one chunk): sorted values and rows.
__global__ __launch_bounds__(256) void topk_merge_kernel(const uint64_t *__restrict__ cand,
                                                         int64_t per_query, int64_t chunk,
                                                         uint32_t k, const uint32_t *__restrict__ gthr,
                                                         int final_out, int largest, uint32_t smax,
                                                         uint64_t *__restrict__ dst,
                                                         uint16_t *__restrict__ vals,
                                                         int32_t *__restrict__ idx)
{
    __shared__ uint64_t mb[kMergeCap];
    __shared__ uint32_t mcnt;
    __shared__ uint64_t mbound;
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x;
    const int64_t c_lo = (int64_t)blockIdx.y * chunk;
    const int64_t c_hi = (c_lo + chunk) < per_query ? (c_lo + chunk) : per_query;
    const uint64_t *src = cand + q * per_query;
    if (tid == 0) {
        mcnt = 0;
        // keys are (d << 32 | row) < 2^48; keep d <= final bound
        mbound = ((uint64_t)gthr[q] + 1u) << 32;
    }
    __syncthreads();
    for (int64_t c0 = c_lo; c0 < c_hi; c0 += 256 * kMergeE) {
        const uint64_t bound = mbound;
#pragma unroll
        for (int e = 0; e < kMergeE; ++e) {
            const int64_t i = c0 + tid + 256 * e;
            if (i < c_hi) {
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
    if (!final_out) {
        uint64_t *out = dst + (q * gridDim.y + blockIdx.y) * (int64_t)k;
        for (uint32_t r = tid; r < k; r += 256)
            out[r] = r < n ? mb[r] : ~0ull;
        return;
    }
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
            const uint32_t d = (uint32_t)(mb[r] >> 32);
            vals[q * k + r] = (uint16_t)(largest ? smax - d : d);
            idx[q * k + r] = (int32_t)(mb[r] & 0xFFFFFFFFu);
        } else {
            vals[q * k + r] = (uint16_t)(largest ? 0u : 0xFFFFu);
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

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Grouped-kernel shapes: (candidate slots, query groups of 8) such that the
// tables (NG * M * 256 bytes) and buffers (NG * 8 * CAP * 4 bytes) fit two
// workgroups per CU.  CAP - 256 bounds k (one pass appends at most 256).
// 376 candidate slots keeps 32 queries at M = 32 within 80 KB (k <= 120).
constexpr int kGCapA = 376;
constexpr int kGCapB = 512;

template <int MM>
constexpr int ng_for(int cap)
{
    return cap == kGCapA ? (MM <= 32 ? 4 : 2) : (MM <= 32 ? 2 : 1);
}

struct FusedPlan {
    bool ok = false;
    int kind = 0;        // 1 few-query, 2 grouped
    int cap = 0;
    int n_rb = 0, n_qb = 0, qb_size = 0, n_chunks = 1;
    int64_t chunk = 0;
    size_t cand_bytes = 0, gthr_bytes = 0, level2_bytes = 0;
};

FusedPlan plan_fused(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    FusedPlan p;
    const bool tuned_M = (M == 8 || M == 16 || M == 32 || M == 64);
    if (!tuned_M || !vec_ok || k > 256 || N <= 0 || Q <= 0)
        return p;
    if (Q < bolt::kSmallQ && bolt::few_fused_lds_bytes(M, (int)Q) <= 160 * 1024) {
        const int64_t rpb = bolt::few_rows_per_block(N);
        p.n_rb = (int)((N + rpb - 1) / rpb);
        p.kind = 1;
        p.n_qb = 1;
        p.qb_size = (int)Q;
    } else {
        p.n_rb = (int)((N + kRowsPerBlock - 1) / kRowsPerBlock);
        p.kind = 2;
        p.cap = kGCapB;   // the 376-slot variant prunes too often to pay for its extra queries
        const int ng = (M <= 32) ? (p.cap == kGCapA ? 4 : 2) : (p.cap == kGCapA ? 2 : 1);
        p.qb_size = 8 * ng;
        p.n_qb = (int)((Q + p.qb_size - 1) / p.qb_size);
        if ((int64_t)p.n_qb * ((p.n_rb + 7) / 8) * 8 > INT32_MAX)
            return p;
    }
    p.cand_bytes = align256((size_t)Q * p.n_rb * k * sizeof(uint64_t));
    p.gthr_bytes = align256((size_t)Q * sizeof(uint32_t));
    const int64_t per_query = (int64_t)p.n_rb * k;
    // first-level chunks: enough workgroups to fill the GPU, 2048..16384 keys each
    int64_t chunk = per_query * Q / 512;
    chunk = chunk < 2048 ? 2048 : (chunk > kMergeChunk ? kMergeChunk : chunk);
    chunk = (chunk + 1023) / 1024 * 1024;
    p.chunk = chunk;
    p.n_chunks = per_query > 2 * chunk ? (int)((per_query + chunk - 1) / chunk) : 1;
    p.level2_bytes = p.n_chunks > 1 ? align256((size_t)Q * p.n_chunks * k * sizeof(uint64_t)) : 0;
    if (p.n_chunks > 65535)
        return p;
    p.ok = true;
    return p;
}

template <int MM>
void launch_fused(const FusedPlan &p, const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q,
                  int k, int largest, uint64_t *cand, uint32_t *gthr, hipStream_t s)
{
    if (p.kind == 1) {
        bolt::few_scan_topk(codes, N, MM, luts, Q, k, largest != 0, p.n_rb, cand, gthr, s);
        return;
    }
    const unsigned grid = (unsigned)(p.n_qb * ((p.n_rb + 7) / 8 * 8));
    if (p.cap == kGCapA)
        hipLaunchKernelGGL((scan_topk_grouped_kernel<MM, ng_for<MM>(kGCapA), kGCapA>), dim3(grid),
                           dim3(256), 0, s, codes, N, luts, Q, (uint32_t)k, largest, p.n_rb, p.n_qb,
                           cand, gthr);
    else
        hipLaunchKernelGGL((scan_topk_grouped_kernel<MM, ng_for<MM>(kGCapB), kGCapB>), dim3(grid),
                           dim3(256), 0, s, codes, N, luts, Q, (uint32_t)k, largest, p.n_rb, p.n_qb,
                           cand, gthr);
}

}  // namespace

namespace bolt {

size_t fused_ws_bytes(int64_t N, int M, int64_t Q, int k)
{
    FusedPlan p = plan_fused(N, M, Q, k, true);
    if (!p.ok)
        return 0;
    return p.cand_bytes + p.gthr_bytes + p.level2_bytes;
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
    const size_t need = p.cand_bytes + p.gthr_bytes + p.level2_bytes;
    if (ws_bytes < need || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "fused scan+top-k needs %zu workspace bytes", need);
    uint64_t *level2 = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(ws) + p.cand_bytes +
                                                    p.gthr_bytes);
    uint64_t *cand = reinterpret_cast<uint64_t *>(ws);
    uint32_t *gthr = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ws) + p.cand_bytes);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, gthr, Q,
                       0xFFFFu);
    switch (M) {
    case 8: launch_fused<8>(p, codes, N, luts, Q, k, largest, cand, gthr, s); break;
    case 16: launch_fused<16>(p, codes, N, luts, Q, k, largest, cand, gthr, s); break;
    case 32: launch_fused<32>(p, codes, N, luts, Q, k, largest, cand, gthr, s); break;
    case 64: launch_fused<64>(p, codes, N, luts, Q, k, largest, cand, gthr, s); break;
    }
    const int64_t per_query = (int64_t)p.n_rb * k;
    const uint32_t smax = 255u * (uint32_t)M;
    if (p.n_chunks > 1) {
        hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)Q, (unsigned)p.n_chunks), dim3(256), 0, s,
                           cand, per_query, p.chunk, (uint32_t)k, gthr, 0, (int)largest, smax,
                           level2, vals, idx);
        const int64_t per2 = (int64_t)p.n_chunks * k;
        hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)Q, 1), dim3(256), 0, s, level2, per2, per2,
                           (uint32_t)k, gthr, 1, (int)largest, smax, nullptr, vals, idx);
    } else {
        hipLaunchKernelGGL(topk_merge_kernel, dim3((unsigned)Q, 1), dim3(256), 0, s, cand, per_query,
                           per_query, (uint32_t)k, gthr, 1, (int)largest, smax, nullptr, vals, idx);
    }
    return check_launch("bolt_scan_topk (fused)");
}

}  // namespace bolt
