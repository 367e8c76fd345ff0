// Top-k retrieval over uint16 sums for gfx950 (Sec. 1.2: the k closest
// vectors; Sec. 4.5: ranking by the smallest approximate distance; the dot
// product ranks by the largest, i.e. maximum inner product search).
//
// The answer is made unique by ordering on the key (value, index): among
// equal values the lower index comes first.  Because the values are 16-bit
// integers the k-th smallest value T is found exactly by a two-level radix
// select (a 256-bin histogram of the high byte, then of the low byte inside
// the selected bucket).  Every value below T is taken; of the values equal
// to T, the ones with the lowest indices are taken, in index order, by a
// block-wide prefix sum over contiguous per-thread runs.  The k survivors are
// sorted by key with a bitonic network in LDS.  One workgroup per row.
// For the largest-k direction every value v is replaced by 65535 - v.
#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "scan_common.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int kE = 8;   // contiguous values per thread per chunk (one 16-byte load)

__device__ __forceinline__ void load8(const uint16_t *__restrict__ row, int64_t i0, int64_t N,
                                      int vec, uint32_t *v)
{
    if (vec && i0 + kE <= N) {
        uint4 t = *reinterpret_cast<const uint4 *>(row + i0);
        v[0] = t.x & 0xFFFFu; v[1] = t.x >> 16;
        v[2] = t.y & 0xFFFFu; v[3] = t.y >> 16;
        v[4] = t.z & 0xFFFFu; v[5] = t.z >> 16;
        v[6] = t.w & 0xFFFFu; v[7] = t.w >> 16;
    } else {
#pragma unroll
        for (int e = 0; e < kE; ++e)
            v[e] = (i0 + e < N) ? (uint32_t)row[i0 + e] : 0xFFFFFFFFu;   // 0xFFFFFFFF = absent
    }
}

// Exclusive prefix sum over the 256 threads; returns the total in *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *wave_sums,
                                                         uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += y;
    }
    if (lane == 63)
        wave_sums[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        uint32_t s = wave_sums[w];
        before += (w < wave) ? s : 0;
        all += s;
    }
    *total = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kThreads) void topk_rows_kernel(
    const uint16_t *__restrict__ d, int64_t N, int64_t ldd, int k, uint32_t flip,
    uint16_t *__restrict__ vals, int32_t *__restrict__ idx, int vec)
{
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sel[BOLT_TOPK_MAX_K];
    __shared__ uint32_t wave_sums[kThreads / 64];
    __shared__ uint32_t sh_T, sh_lt, sh_nlt;
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x;
    const uint16_t *row = d + q * ldd;
    const int kk = ((int64_t)k < N) ? k : (int)N;

    uint32_t T, count_lt, need_eq;
    if ((int64_t)kk == N) {
        T = 0x10000u;          // every value is below: take all N
        count_lt = (uint32_t)N;
        need_eq = 0;
    } else {
        // level 1: high byte
        hist[tid] = 0;
        __syncthreads();
        for (int64_t i0 = (int64_t)tid * kE; i0 < N; i0 += (int64_t)kThreads * kE) {
            uint32_t v[kE];
            load8(row, i0, N, vec, v);
#pragma unroll
            for (int e = 0; e < kE; ++e)
                if (v[e] != 0xFFFFFFFFu)
                    atomicAdd(&hist[(v[e] ^ flip) >> 8], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t cum = 0;
            int B = 0;
            for (; B < 255; ++B) {
                if (cum + hist[B] >= (uint32_t)k)
                    break;
                cum += hist[B];
            }
            sh_T = (uint32_t)B;
            sh_lt = cum;
        }
        __syncthreads();
        const uint32_t B = sh_T, lt_B = sh_lt;
        hist[tid] = 0;
        __syncthreads();
        // level 2: low byte inside bucket B
        for (int64_t i0 = (int64_t)tid * kE; i0 < N; i0 += (int64_t)kThreads * kE) {
            uint32_t v[kE];
            load8(row, i0, N, vec, v);
#pragma unroll
            for (int e = 0; e < kE; ++e)
                if (v[e] != 0xFFFFFFFFu && ((v[e] ^ flip) >> 8) == B)
                    atomicAdd(&hist[(v[e] ^ flip) & 255u], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t cum = lt_B;
            int L = 0;
            for (; L < 255; ++L) {
                if (cum + hist[L] >= (uint32_t)k)
                    break;
                cum += hist[L];
            }
            sh_T = (B << 8) | (uint32_t)L;
            sh_lt = cum;
        }
        __syncthreads();
        T = sh_T;
        count_lt = sh_lt;
        need_eq = (uint32_t)k - count_lt;
    }

    // collect: all values < T, and the first need_eq values == T in index order
    if (tid == 0)
        sh_nlt = 0;
    __syncthreads();
    uint32_t eq_base = 0;
    for (int64_t c0 = 0; c0 < N; c0 += (int64_t)kThreads * kE) {
        const int64_t i0 = c0 + (int64_t)tid * kE;
        uint32_t v[kE];
        load8(row, i0, N, vec, v);
        uint32_t my_eq = 0;
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            if (v[e] == 0xFFFFFFFFu)
                continue;
            const uint32_t w = v[e] ^ flip;
            if (w < T) {
                uint32_t pos = atomicAdd(&sh_nlt, 1u);
                sel[pos] = ((uint64_t)w << 32) | (uint64_t)(i0 + e);
            } else if (w == T) {
                ++my_eq;
            }
        }
        uint32_t total;
        uint32_t r = eq_base + block_exclusive_scan(my_eq, wave_sums, &total);
        if (my_eq) {
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                if (v[e] != 0xFFFFFFFFu && (v[e] ^ flip) == T) {
                    if (r < need_eq)
                        sel[count_lt + r] = ((uint64_t)T << 32) | (uint64_t)(i0 + e);
                    ++r;
                }
            }
        }
        eq_base += total;
        __syncthreads();
        if (eq_base >= need_eq && sh_nlt == count_lt)
            break;
    }
    __syncthreads();

    // bitonic sort of sel[0 .. P), P = next power of two >= kk
    int P = 1;
    while (P < kk)
        P <<= 1;
    for (int i = kk + tid; i < P; i += kThreads)
        sel[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += kThreads) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool asc = (i & size) == 0;
                const uint64_t a = sel[i], b = sel[j];
                if ((a > b) == asc) {
                    sel[i] = b;
                    sel[j] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int r = tid; r < k; r += kThreads) {
        if (r < kk) {
            vals[q * k + r] = (uint16_t)((uint32_t)(sel[r] >> 32) ^ flip);
            idx[q * k + r] = (int32_t)(sel[r] & 0xFFFFFFFFu);
        } else {
            vals[q * k + r] = (uint16_t)(flip ? 0u : 0xFFFFu);
            idx[q * k + r] = -1;
        }
    }
}

int validate_topk(int64_t Q, int64_t N, int32_t k)
{
    using namespace bolt;
    BOLT_TRY(check_N(Q, "Q"));
    BOLT_TRY(check_N(N, "N"));
    if (k < 1)
        return fail(BOLT_ERR_INVALID, "k must be >= 1 (got %d)", k);
    if (k > BOLT_TOPK_MAX_K)
        return fail(BOLT_ERR_UNSUPPORTED, "k must be <= %d (got %d)", BOLT_TOPK_MAX_K, k);
    return BOLT_OK;
}

}  // namespace

namespace bolt {
int topk_u16(const uint16_t *d, int64_t Q, int64_t N, int64_t ldd, int k, int largest,
             uint16_t *vals, int32_t *idx, hipStream_t s)
{
    const int vec = aligned(d, 16) && (ldd % 8 == 0);
    {
        bolt::ProfScope prof_("topk_rows", s);
        hipLaunchKernelGGL(topk_rows_kernel, dim3((unsigned)Q), dim3(kThreads), 0, s, d, N, ldd, k,
                           largest ? 0xFFFFu : 0u, vals, idx, vec);
    }
    return check_launch("bolt_topk");
}
}  // namespace bolt

extern "C" size_t bolt_topk_ws_bytes(int64_t Q, int64_t N, int32_t k)
{
    (void)Q;
    (void)N;
    (void)k;
    return 0;
}

extern "C" int bolt_topk(const uint16_t *dists, int64_t Q, int64_t N, int64_t ldd, int32_t k,
                         int32_t largest, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
                         void *stream)
{
    using namespace bolt;
    (void)ws;
    (void)ws_bytes;
    BOLT_TRY(validate_topk(Q, N, k));
    if (ldd < N)
        return fail(BOLT_ERR_INVALID, "ldd (%lld) < N (%lld)", (long long)ldd, (long long)N);
    if (Q == 0)
        return BOLT_OK;
    if (!vals || !idx || (N > 0 && !dists))
        return fail(BOLT_ERR_INVALID, "bolt_topk: null pointer");
    return topk_u16(dists, Q, N, ldd, k, largest != 0, vals, idx, as_stream(stream));
}

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

namespace bolt {
int g_force_unfused_topk = 0;
int g_force_fused_kind = -1;
int g_spec_mode = -1;
int g_sparse_mfma = 1;
}

static size_t unfused_ws_bytes(int64_t N, int64_t Q)
{
    if (N <= 0 || Q <= 0)
        return 0;
    return round_up((size_t)Q * (size_t)N * sizeof(uint16_t), 256);
}

// The fused path needs only its candidate buffers; the scan-then-select path
// (shapes without a fused kernel, unaligned operands, or the test hook) needs
// the whole [Q][N] sum matrix.
static size_t scan_topk_need(int64_t N, int32_t M, int64_t Q, int32_t k, bool vec_ok)
{
    if (N > 0 && !bolt::g_force_unfused_topk && bolt::fused_supported(N, M, Q, k, vec_ok))
        return bolt::fused_ws_bytes(N, M, Q, k);
    return unfused_ws_bytes(N, Q);
}

extern "C" size_t bolt_scan_topk_ws_bytes(int64_t N, int32_t M, int64_t Q, int32_t k)
{
    return scan_topk_need(N, M, Q, k, true);
}

static int scan_topk_impl(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8, int64_t Q,
                          int32_t metric, int32_t k, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
                          void *stream);

extern "C" int bolt_scan_topk(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                              int64_t Q, int32_t metric, int32_t k, uint16_t *vals, int32_t *idx,
                              void *ws, size_t ws_bytes, void *stream)
{
    return scan_topk_impl(codes, N, M, luts_u8, Q, metric, k, vals, idx, ws, ws_bytes, stream);
}

// The workspace of bolt_scan_topk_noalloc: a file-scope device array, one
// copy per GPU the library runs on, held until the process ends.  Host code
// never uses the array's name as an address: the device address of each
// GPU's copy comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[BOLT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch (set up on its first use).
int scratch_address(void **out)
{
    using namespace bolt;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return fail(BOLT_ERR_DEVICE, "bolt_scan_topk_noalloc: no current device");
    if (dev >= kMaxDevices)
        return fail(BOLT_ERR_UNSUPPORTED, "bolt_scan_topk_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BOLT_ERR_DEVICE, "bolt_scan_topk_noalloc: hipGetSymbolAddress of the scratch failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BOLT_OK;
}
}  // namespace

extern "C" int bolt_scan_topk_noalloc(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                                      int64_t Q, int32_t metric, int32_t k, uint16_t *vals, int32_t *idx,
                                      void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(validate_topk(Q, N, k));
    const size_t need = scan_topk_need(N, M, Q, k, true);
    if (need > (size_t)BOLT_NOALLOC_SCRATCH_BYTES)
        return fail(BOLT_ERR_UNSUPPORTED,
                    "bolt_scan_topk_noalloc: this call needs %zu workspace bytes, above the %llu bytes of its "
                    "static scratch (use bolt_scan_topk with a workspace)",
                    need, (unsigned long long)BOLT_NOALLOC_SCRATCH_BYTES);
    if (Q == 0)
        return scan_topk_impl(codes, N, M, luts_u8, Q, metric, k, vals, idx, nullptr, 0, stream);
    void *ws = nullptr;
    BOLT_TRY(scratch_address(&ws));
    return scan_topk_impl(codes, N, M, luts_u8, Q, metric, k, vals, idx, ws, (size_t)BOLT_NOALLOC_SCRATCH_BYTES,
                          stream);
}

static int scan_topk_impl(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8, int64_t Q,
                          int32_t metric, int32_t k, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes,
                          void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(validate_topk(Q, N, k));
    Metric mt;
    BOLT_TRY(decode_metric(metric, &mt));
    if (Q == 0)
        return BOLT_OK;
    if (!vals || !idx || (N > 0 && (!codes || !luts_u8)))
        return fail(BOLT_ERR_INVALID, "bolt_scan_topk: null pointer");
    if (N > 0 && !(aligned(codes, 16) && aligned(luts_u8, 16)))
        return fail(BOLT_ERR_INVALID, "bolt_scan_topk: codes and luts_u8 must be 16-byte aligned");
    const size_t need = scan_topk_need(N, M, Q, k, true);
    if (ws_bytes < need || (need && !ws))
        return fail(BOLT_ERR_NOMEM, "workspace of %zu bytes needed (got %zu)", need, ws_bytes);
    if (need && !aligned(ws, 256))
        return fail(BOLT_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = as_stream(stream);
    const bool largest = mt.largest;
    if (N > 0 && !g_force_unfused_topk) {
        const int st = scan_topk_fused(codes, N, M, luts_u8, Q, k, one_order(largest), vals, idx, ws, ws_bytes, s);
        if (st != BOLT_ERR_UNSUPPORTED)
            return st;
    }
    uint16_t *d = reinterpret_cast<uint16_t *>(ws);
    if (N > 0)
        BOLT_TRY(scan_u16(codes, N, M, luts_u8, Q, d, N, s));
    return topk_u16(d, Q, N, N, k, largest, vals, idx, s);
}

extern "C" size_t bolt_scan_topk_split_ws_bytes(int64_t N, int32_t M, int64_t Q, int64_t q_split, int32_t k)
{
    if (Q <= 0 || q_split < 0 || q_split > Q)
        return 0;
    // enough for one set of launches over all Q queries and for either side alone
    size_t need = scan_topk_need(N, M, Q, k, true);
    if (q_split > 0)
        need = std::max(need, scan_topk_need(N, M, q_split, k, true));
    if (q_split < Q)
        need = std::max(need, scan_topk_need(N, M, Q - q_split, k, true));
    return need;
}

extern "C" int bolt_scan_topk_split(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                                    int64_t Q, int64_t q_split, int32_t metric_lo, int32_t metric_hi, int32_t k,
                                    uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(validate_topk(Q, N, k));
    Metric lo, hi;
    BOLT_TRY(decode_metric(metric_lo, &lo));
    BOLT_TRY(decode_metric(metric_hi, &hi));
    if (q_split < 0 || q_split > Q)
        return fail(BOLT_ERR_INVALID, "q_split must be in [0, Q] (got %lld, Q = %lld)", (long long)q_split,
                    (long long)Q);
    if (Q == 0)
        return BOLT_OK;
    if (!vals || !idx || (N > 0 && (!codes || !luts_u8)))
        return fail(BOLT_ERR_INVALID, "bolt_scan_topk_split: null pointer");
    if (N > 0 && !(aligned(codes, 16) && aligned(luts_u8, 16)))
        return fail(BOLT_ERR_INVALID, "bolt_scan_topk_split: codes and luts_u8 must be 16-byte aligned");
    const size_t need = bolt_scan_topk_split_ws_bytes(N, M, Q, q_split, k);
    if (ws_bytes < need || (need && !ws))
        return fail(BOLT_ERR_NOMEM, "workspace of %zu bytes needed (got %zu)", need, ws_bytes);
    if (need && !aligned(ws, 256))
        return fail(BOLT_ERR_INVALID, "workspace must be 256-byte aligned");
    // the result depends on the metric only through the direction
    if (lo.largest == hi.largest || q_split == Q)
        return scan_topk_impl(codes, N, M, luts_u8, Q, metric_lo, k, vals, idx, ws, ws_bytes, stream);
    if (q_split == 0)
        return scan_topk_impl(codes, N, M, luts_u8, Q, metric_hi, k, vals, idx, ws, ws_bytes, stream);
    if (N > 0 && !g_force_unfused_topk && fused_on_matrix_cores(N, M, Q, k, true))
        return scan_topk_fused(codes, N, M, luts_u8, Q, k, RankOrder{q_split, lo.largest ? 1 : 0}, vals, idx, ws,
                               ws_bytes, as_stream(stream));
    BOLT_TRY(scan_topk_impl(codes, N, M, luts_u8, q_split, metric_lo, k, vals, idx, ws, ws_bytes, stream));
    return scan_topk_impl(codes, N, M, luts_u8 + q_split * M * 16, Q - q_split, metric_hi, k, vals + q_split * k,
                          idx + q_split * k, ws, ws_bytes, stream);
}

static int validate_ranges(const int64_t *ranges, int32_t n_ranges, int64_t N)
{
    using namespace bolt;
    if (n_ranges < 0)
        return fail(BOLT_ERR_INVALID, "n_ranges must be >= 0 (got %d)", n_ranges);
    if (n_ranges > 0 && !ranges)
        return fail(BOLT_ERR_INVALID, "ranges is null");
    int64_t prev_end = 0;
    for (int32_t r = 0; r < n_ranges; ++r) {
        const int64_t a = ranges[2 * r], b = ranges[2 * r + 1];
        if (a < prev_end || b < a || b > N)
            return fail(BOLT_ERR_INVALID,
                        "range %d = [%lld, %lld): ranges must be ascending, disjoint and inside [0, %lld]", r,
                        (long long)a, (long long)b, (long long)N);
        prev_end = b;
    }
    return BOLT_OK;
}

extern "C" size_t bolt_scan_topk_ranges_ws_bytes(const int64_t *ranges, int32_t n_ranges, int32_t M, int64_t Q,
                                                 int32_t k)
{
    if (n_ranges <= 0 || !ranges || Q <= 0)
        return 0;
    return bolt::ranges_ws_bytes(ranges, n_ranges, M, Q, k);
}

extern "C" int bolt_scan_topk_ranges(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                                     int64_t Q, int32_t metric, int32_t k, const int64_t *ranges, int32_t n_ranges,
                                     uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(validate_topk(Q, N, k));
    Metric mt;
    BOLT_TRY(decode_metric(metric, &mt));
    BOLT_TRY(validate_ranges(ranges, n_ranges, N));
    if (Q == 0)
        return BOLT_OK;
    if (!vals || !idx || (N > 0 && (!codes || !luts_u8)))
        return fail(BOLT_ERR_INVALID, "bolt_scan_topk_ranges: null pointer");
    return scan_topk_ranges(codes, N, M, luts_u8, Q, k, mt.largest, ranges, n_ranges, vals, idx,
                            ws, ws_bytes, as_stream(stream));
}

// Test hook: 1 forces bolt_scan_topk onto the scan-then-select path.
extern "C" int bolt_debug_force_unfused_topk(int32_t on)
{
    bolt::g_force_unfused_topk = on ? 1 : 0;
    return BOLT_OK;
}

// Test hook: speculative bounds of many-query scans (-1 automatic, 0 off,
// 1 on from 2^16 rows (as -1), 2 as 1 with every bound failing: all queries are
// recomputed by the exact fallback).
extern "C" int bolt_debug_speculation(int32_t mode)
{
    if (mode < -1 || mode > 2)
        return bolt::fail(BOLT_ERR_INVALID, "speculation mode must be -1, 0, 1 or 2 (got %d)", mode);
    bolt::g_spec_mode = mode;
    return BOLT_OK;
}

// Test hook: the matrix-core tiles with the sparse (1) or the dense (0) instruction.
extern "C" int bolt_debug_sparse_mfma(int32_t on)
{
    bolt::g_sparse_mfma = on ? 1 : 0;
    return BOLT_OK;
}

// Test hook: the many-query fused kernel (-1 automatic, 2 grouped, 3 matrix cores).
extern "C" int bolt_debug_force_fused_kind(int32_t kind)
{
    if (kind != -1 && kind != 2 && kind != 3)
        return bolt::fail(BOLT_ERR_INVALID, "fused kind must be -1, 2 or 3 (got %d)", kind);
    bolt::g_force_fused_kind = kind;
    return BOLT_OK;
}
