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
#include "tiles.hpp"

namespace {

using bolt::code_at;
using bolt::load_row;
using bolt::PruneResult;

constexpr int kRowsPerBlock = 16384;      // rows per workgroup (<= 65536: 16-bit local rows)
constexpr int64_t kMergeChunk = 16384;    // keys per first-level merge workgroup

// Decode the tile of workgroup `w`: XCD-major placement of row blocks.
__device__ __forceinline__ void tile_of(int w, int n_qb, int &qb, int &rb)
{
    const int xcd = w & 7, i = w >> 3;
    qb = i % n_qb;
    rb = (i / n_qb) * 8 + xcd;
}

template <int MM, int NG>
__global__ __launch_bounds__(256) void scan_topk_grouped_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    uint32_t k, int largest, int n_rb, int n_qb, uint64_t *__restrict__ cand,
    uint32_t *__restrict__ gthr)
{
    __shared__ bolt::GroupedLds<MM, NG> L;
    int qb, rb;
    tile_of(blockIdx.x, n_qb, qb, rb);
    if (rb >= n_rb)
        return;
    constexpr int QB = 8 * NG;
    bolt::TileJob job;
    job.codes = codes;
    job.luts = luts;
    job.cand = cand;
    job.gthr = gthr;
    job.r0 = (int64_t)rb * kRowsPerBlock;
    job.r1 = (job.r0 + kRowsPerBlock) < N ? (job.r0 + kRowsPerBlock) : N;
    job.rb = rb;
    job.n_rb = n_rb;
    job.q0 = (int64_t)qb * QB;
    job.nq = (int)((Q - job.q0) < QB ? (Q - job.q0) : QB);
    job.k = k;
    job.largest = largest;
    bolt::grouped_tile<MM, NG>(job, L);
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
    const int64_t q = blockIdx.x;
    const int64_t c_lo = (int64_t)blockIdx.y * chunk;
    const int64_t c_hi = (c_lo + chunk) < per_query ? (c_lo + chunk) : per_query;
    uint64_t *out = final_out ? nullptr : dst + (q * gridDim.y + blockIdx.y) * (int64_t)k;
    bolt::merge_keys(cand + q * per_query, c_lo, c_hi, k, gthr[q], out, largest, smax,
                     vals + q * k, idx + q * k);
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
// Query groups per grouped tile: tables (NG * M * 256 bytes) and candidate
// buffers (NG * 8 * 512 * 4 bytes) within about 48 KB, three workgroups per CU.
template <int MM>
constexpr int ng_for()
{
    return MM <= 32 ? 2 : 1;
}

struct FusedPlan {
    bool ok = false;
    int kind = 0;        // 1 few-query, 2 grouped
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
        const int ng = M <= 32 ? 2 : 1;
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
    {
        bolt::ProfScope prof_("scan_topk_grouped", s);
        hipLaunchKernelGGL((scan_topk_grouped_kernel<MM, ng_for<MM>()>), dim3(grid), dim3(256), 0, s, codes,
                           N, luts, Q, (uint32_t)k, largest, p.n_rb, p.n_qb, cand, gthr);
    }
}

}  // namespace

namespace bolt {

bool fused_supported(int64_t N, int M, int64_t Q, int k, bool vec_ok)
{
    return plan_fused(N, M, Q, k, vec_ok).ok;
}

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
    bolt::ProfScope prof_("topk_merge", s);
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
