// Declarations shared by the scan, top-k and batched translation units.
#pragma once

#include "common.hpp"

namespace bolt {

enum class OutMode { U16, F32, F32T };

// Which sums a call's queries rank by: the smallest, or the largest (through
// d = 255 M - sum).  Queries before `split` take order `lo` (1: largest) and
// those at or beyond it the other order, so that one launch can serve a
// distance metric and a similarity side by side; a call of one order has
// split = kOneOrder.
constexpr int64_t kOneOrder = INT64_MAX;

struct RankOrder {
    int64_t split;
    int lo;
    __host__ __device__ __forceinline__ bool largest(int64_t q) const { return (q >= split) != (lo != 0); }
};

__host__ __device__ __forceinline__ RankOrder one_order(bool largest) { return RankOrder{kOneOrder, largest ? 1 : 0}; }

// Queries below this count use the few-query scan (tables as 16-byte rows).
constexpr int kSmallQ = 8;

// -1 automatic, 0 generic, 1 few-query, 2 grouped (set by a test hook).
extern int g_force_scan_kernel;

// uint16 scan into out[Q][ldo] on stream s (arguments already validated).
int scan_u16(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, uint16_t *out,
             int64_t ldo, hipStream_t s);

// Fused scan + top-k (fused.hip): whether the shape has a fused kernel (vec_ok:
// codes and tables 16-byte aligned), its workspace size (0 if it has none) and
// the launch (BOLT_ERR_UNSUPPORTED if it has none).
bool fused_supported(int64_t N, int M, int64_t Q, int k, bool vec_ok);
size_t fused_ws_bytes(int64_t N, int M, int64_t Q, int k);
// The same over caller-given row ranges (host int64 [n_ranges][2]).
size_t ranges_ws_bytes(const int64_t *ranges, int n_ranges, int M, int64_t Q, int k);
int scan_topk_ranges(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                     bool largest, const int64_t *ranges, int n_ranges, uint16_t *vals, int32_t *idx, void *ws,
                     size_t ws_bytes, hipStream_t s);
int scan_topk_fused(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                    RankOrder order, uint16_t *vals, int32_t *idx, void *ws, size_t ws_bytes, hipStream_t s);
// Whether the fused plan of the shape runs on the matrix-core tiles (the
// only kind that serves queries of both orders in one launch).
bool fused_on_matrix_cores(int64_t N, int M, int64_t Q, int k, bool vec_ok);

// Few-query scans (few.hip).
bool few_supported(int M, int64_t Q);
template <OutMode OUT>
int few_scan(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, uint16_t *out,
             float *outf, int64_t ldo, float bias, float scale, hipStream_t s);
int64_t few_rows_per_block(int64_t N, int M, int nq);
size_t few_fused_lds_bytes(int M, int nq);
int few_scan_topk(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                  RankOrder order, int n_rb, uint64_t *cand, uint32_t *ccnt, uint32_t *hist, uint32_t *gthr,
                  const int64_t *tiles, uint32_t *lcnt, hipStream_t s);

// Test hook: 1 forces the unfused scan-then-select path of bolt_scan_topk.
extern int g_force_unfused_topk;
extern int g_force_fused_kind;   // -1 automatic, 2 grouped, 3 matrix cores
extern int g_spec_mode;           // speculative bounds: -1 automatic, 0 off, 1 on, 2 on and failing

// Speculative starting bounds (fused.hip): sample chunks of kSpecSpan rows,
// used from kSpecMinRows rows (kSpecMinRowsForced under test mode 1), at
// most kSpecMaxDists sample distances computed per call, kept as one
// minimum per kSpecGroup rows; spec_rank gives the smallest rank r with
// P(binomial(k, p) >= r) <= 1e-7 (at most k).
constexpr int64_t kSpecSpan = 1024;
constexpr int kSpecGroup = 16;
constexpr int kSpecGroups = (int)kSpecSpan / kSpecGroup;   // group minima per chunk
// From 2^16 rows: at 7e4 to 5e5 rows, M = 16 and 32, 1 to 1000 queries, a
// sampled call took 0.19-0.31 of the time of one without (whose tiles keep
// slots of candidates for every row block and merge them all).  Over 256
// batched databases of 1e3 to 2e6 rows the whole batch took 11.0 ms
// sampling from 2^19 rows, 9.0 from 2^17, 8.8 from 2^16 and 9.0-9.3 from
// 2^15, where a few sampled bounds (a sample of half the rows in
// 1024-row chunks) failed and were recomputed.
constexpr int64_t kSpecMinRows = 1 << 16;
constexpr int64_t kSpecMinRowsForced = 1 << 16;
constexpr int64_t kSpecMaxDists = 1 << 26;
int spec_rank(int k, double pr);

// Top-k of the rows of a uint16 matrix (arguments already validated).
int topk_u16(const uint16_t *d, int64_t Q, int64_t N, int64_t ldd, int k, int largest,
             uint16_t *vals, int32_t *idx, hipStream_t s);

// Load the M/2 code bytes of row n into dwords (MM/8 of them).
// NT: non-temporal loads, for codes that one call streams exactly once
// (one or a few queries): a plain streaming read of 4 GB on MI355X reaches
// 7.1-7.2 TB/s with the non-temporal hint and 5.6-5.7 TB/s without it.
template <int MM, bool NT = false>
__device__ __forceinline__ void load_row(const uint8_t *__restrict__ codes, int64_t n, uint32_t *cw)
{
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const uint8_t *p = codes + n * (MM / 2);
    if constexpr (MM / 2 >= 16) {
#pragma unroll
        for (int v = 0; v < MM / 32; ++v) {
            const u32x4 *a = reinterpret_cast<const u32x4 *>(p) + v;
            const u32x4 t = NT ? __builtin_nontemporal_load(a) : *a;
            cw[4 * v + 0] = t.x;
            cw[4 * v + 1] = t.y;
            cw[4 * v + 2] = t.z;
            cw[4 * v + 3] = t.w;
        }
    } else if constexpr (MM / 2 == 8) {
        const u32x2 *a = reinterpret_cast<const u32x2 *>(p);
        const u32x2 t = NT ? __builtin_nontemporal_load(a) : *a;
        cw[0] = t.x;
        cw[1] = t.y;
    } else {
        static_assert(MM / 2 == 4, "rows of 4, 8 or a multiple of 16 bytes");
        const uint32_t *a = reinterpret_cast<const uint32_t *>(p);
        cw[0] = NT ? __builtin_nontemporal_load(a) : *a;
    }
}

// Code of subspace m from the row's dwords (low nibble = even subspace).
template <int MM>
__device__ __forceinline__ uint32_t code_at(const uint32_t *cw, int m)
{
    return (cw[m >> 3] >> (4 * (m & 7))) & 15u;
}

}  // namespace bolt
