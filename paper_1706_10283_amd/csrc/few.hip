// The scan for a few queries (Q < 8), the HBM-bound case (Sec. 3.1 scan,
// Sec. 3.2 vectorised lookups), plain or fused with top-k selection.
//
// One byte of codes holds the codes of two subspaces, so each workgroup
// first expands every query's tables into pair tables: entry b of pair p is
// lut[2p][b & 15] + lut[2p+1][b >> 4], a 256-entry uint16 table (512 bytes).
// One 16-bit LDS read then performs two lookups.  A 512-byte table covers
// each of the 64 LDS banks with two dwords, so a wave read has at most a
// two-way bank conflict.  Rows are streamed with 16-byte loads, R rows per
// lane in flight, and the lookups of the R rows are interleaved so that the
// reads of different rows overlap.  LDS is sized by the actual query count,
// which keeps occupancy high for a single query.
#include <atomic>

#include "common.hpp"
#include "scan_common.hpp"
#include "tiles.hpp"

namespace {

using bolt::load_row;
using bolt::OutMode;

using bolt::build_pair_tables;
using bolt::local_key;
using bolt::PruneResult;
using bolt::read_bound;
using bolt::copy_rows;
using bolt::load_rows;
using bolt::load_rows_clamped;
using bolt::pair_sums;

// ------------------------------------------------------------------ plain

template <int MM, OutMode OUT, bool ONE>
__global__ __launch_bounds__(256) void few_scan_kernel(const uint8_t *__restrict__ codes, int64_t N,
                                                       const uint8_t *__restrict__ luts, int nq,
                                                       int64_t rows_per_block,
                                                       uint16_t *__restrict__ out,
                                                       float *__restrict__ outf, int64_t ldo,
                                                       float bias, float scale)
{
    // one query: static tables at a fixed LDS address (table offsets fold
    // into the reads); several: dynamic [nq][MM/2][256]
    extern __shared__ __attribute__((aligned(16))) uint16_t pt_dyn[];
    __shared__ __attribute__((aligned(16))) uint16_t pt_one[ONE ? (MM / 2) * 256 : 1];
    uint16_t *pt = ONE ? pt_one : pt_dyn;
    if (ONE)
        nq = 1;
    build_pair_tables<MM>(luts, nq, pt);
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    constexpr int R = bolt::few_r(MM);
    constexpr int PASS = bolt::few_pass(MM);
    uint32_t cw[R][MM / 8], nx[R][MM / 8];
    load_rows<MM, R>(codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += PASS) {
        copy_rows<MM, R>(nx, cw);
        if (base + PASS < r1)   // next pass in flight while this one is computed
            load_rows<MM, R>(codes, base + PASS, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[R];
            pair_sums<MM, R, ONE>(reinterpret_cast<const char *>(pt + q * (MM / 2) * 256), cw, s);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t n = base + threadIdx.x + 256 * r;
                if (n < r1) {
                    if (OUT == OutMode::U16) {
                        out[q * ldo + n] = (uint16_t)s[r];
                    } else {
                        const float v = ((float)s[r] + bias) * scale;
                        if (OUT == OutMode::F32)
                            outf[q * ldo + n] = v;
                        else
                            outf[n * ldo + q] = v;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ fused with top-k

template <int MM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void few_scan_topk_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int nq, uint32_t k,
    bolt::RankOrder order, int64_t rows_per_block, int n_rb, uint64_t *__restrict__ cand, uint32_t *__restrict__ ccnt,
    uint32_t *__restrict__ hist, uint32_t *__restrict__ gthr, const int64_t *__restrict__ tiles,
    uint32_t *__restrict__ lcnt)
{
    extern __shared__ __attribute__((aligned(16))) char few_lds[];
    bolt::TileJob job;
    job.codes = codes;
    job.luts = luts;
    job.cand = cand;
    job.ccnt = ccnt;
    job.hist = hist;
    job.lcnt = lcnt;
    job.hist_shift = bolt::hist_shift(MM);
    job.gthr = gthr;
    job.rb = blockIdx.x;
    if (tiles) {   // row ranges given by the caller, cut into tiles
        job.r0 = tiles[2 * job.rb];
        job.r1 = tiles[2 * job.rb + 1];
    } else {
        job.r0 = job.rb * rows_per_block;
        job.r1 = (job.r0 + rows_per_block) < N ? (job.r0 + rows_per_block) : N;
    }
    job.n_rb = n_rb;
    job.q0 = 0;
    job.nq = nq;
    job.k = k;
    job.order = order;
    bolt::few_tile<MM, false>(job, few_lds);
}

// One query (the HBM-bound case): one workgroup per tile of tile_rows rows;
// the many small tiles let the dispatcher balance the load.  Each tile
// writes its exact local top-k to cand[tile][k] (packed, count in
// ccnt[tile] and keys counted in hist, when ccnt is given), or appends it
// to the dense list cand (count in *lcnt) when lcnt is given; see
// bolt::one_query_tile.
template <int MM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void one_scan_topk_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, uint32_t k,
    int largest, int64_t tile_rows, uint64_t *__restrict__ cand, uint32_t *__restrict__ ccnt,
    uint32_t *__restrict__ hist, uint32_t *__restrict__ gthr, const int64_t *__restrict__ tiles,
    uint32_t *__restrict__ lcnt)
{
    // One tile per workgroup: a persistent grid of four workgroups per CU,
    // each building its pair tables once for several tiles, measured 5-8%
    // slower over 2.5e8 rows at M = 16 and 32.
    __shared__ __attribute__((aligned(16))) char lds[bolt::one_query_lds_bytes(MM)];
    const int64_t tile = blockIdx.x;
    const int64_t r0 = tiles ? tiles[2 * tile] : tile * tile_rows;
    const int64_t r1 = tiles ? tiles[2 * tile + 1] : ((r0 + tile_rows) < N ? (r0 + tile_rows) : N);
    if (lcnt)
        bolt::one_query_tile<MM>(codes, r0, r1, luts, k, largest, cand, nullptr, nullptr, gthr, lds, lcnt);
    else
        bolt::one_query_tile<MM>(codes, r0, r1, luts, k, largest, cand + tile * k, ccnt ? ccnt + tile : nullptr,
                                 hist, gthr, lds);
}

size_t few_lds_bytes(int M, int nq, bool fused)
{
    return fused ? bolt::few_tile_lds_bytes(M, nq) : (size_t)nq * (M / 2) * 256 * sizeof(uint16_t);
}

template <int MM, OutMode OUT>
void launch_few_scan(const uint8_t *codes, int64_t N, const uint8_t *luts, int nq, uint16_t *out,
                     float *outf, int64_t ldo, float bias, float scale, hipStream_t s)
{
    const int64_t rpb = bolt::few_rows_per_block(N, MM, nq);
    const dim3 grid((unsigned)((N + rpb - 1) / rpb));
    const size_t lds = few_lds_bytes(MM, nq, false);
    bolt::ProfScope prof_("scan_few", s);
    if (nq == 1)
        hipLaunchKernelGGL((few_scan_kernel<MM, OUT, true>), grid, dim3(256), 0, s, codes, N, luts, nq, rpb,
                           out, outf, ldo, bias, scale);
    else
        hipLaunchKernelGGL((few_scan_kernel<MM, OUT, false>), grid, dim3(256), lds, s, codes, N, luts, nq, rpb,
                           out, outf, ldo, bias, scale);
}

template <int MM>
void launch_few_scan_topk(const uint8_t *codes, int64_t N, const uint8_t *luts, int nq, int k, bolt::RankOrder order,
                          int64_t rpb, int n_rb, uint64_t *cand, uint32_t *ccnt, uint32_t *hist, uint32_t *gthr,
                          const int64_t *tiles, uint32_t *lcnt, hipStream_t s)
{
    if (nq == 1)
        hipLaunchKernelGGL(one_scan_topk_kernel<MM>, dim3(n_rb), dim3(256), 0, s, codes, N, luts, (uint32_t)k,
                           (int)order.largest(0), rpb, cand, ccnt, hist, gthr, tiles, lcnt);
    else
        hipLaunchKernelGGL(few_scan_topk_kernel<MM>, dim3(n_rb), dim3(256), few_lds_bytes(MM, nq, true), s,
                           codes, N, luts, nq, (uint32_t)k, order, rpb, n_rb, cand, ccnt, hist, gthr,
                           tiles, lcnt);
}

template <int MM>
hipError_t few_occupancy(int *per_cu, int nq, size_t lds)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, few_scan_topk_kernel<MM>, 256, lds);
}

}  // namespace

namespace bolt {

bool few_supported(int M, int64_t Q)
{
    return (M == 8 || M == 16 || M == 32 || M == 64) && Q >= 1 && Q < kSmallQ;
}

template <OutMode OUT>
int few_scan(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, uint16_t *out,
             float *outf, int64_t ldo, float bias, float scale, hipStream_t s)
{
    const int nq = (int)Q;
    switch (M) {
    case 8: launch_few_scan<8, OUT>(codes, N, luts, nq, out, outf, ldo, bias, scale, s); break;
    case 16: launch_few_scan<16, OUT>(codes, N, luts, nq, out, outf, ldo, bias, scale, s); break;
    case 32: launch_few_scan<32, OUT>(codes, N, luts, nq, out, outf, ldo, bias, scale, s); break;
    case 64: launch_few_scan<64, OUT>(codes, N, luts, nq, out, outf, ldo, bias, scale, s); break;
    default: return fail(BOLT_ERR_UNSUPPORTED, "few-query scan takes M in {8, 16, 32, 64}");
    }
    return check_launch("bolt scan (few queries)");
}

template int few_scan<OutMode::U16>(const uint8_t *, int64_t, int, const uint8_t *, int64_t,
                                    uint16_t *, float *, int64_t, float, float, hipStream_t);
template int few_scan<OutMode::F32>(const uint8_t *, int64_t, int, const uint8_t *, int64_t,
                                    uint16_t *, float *, int64_t, float, float, hipStream_t);
template int few_scan<OutMode::F32T>(const uint8_t *, int64_t, int, const uint8_t *, int64_t,
                                     uint16_t *, float *, int64_t, float, float, hipStream_t);

size_t few_fused_lds_bytes(int M, int nq) { return few_lds_bytes(M, nq, true); }

// Workgroups of the fused few-query kernel resident on the current device
// (occupancy per CU times CUs), cached per (device, M, nq).
static int few_slots(int M, int nq)
{
    static std::atomic<int> cache[16][4][8];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16)
        dev = 0;
    const int mi = M == 8 ? 0 : M == 16 ? 1 : M == 32 ? 2 : 3;
    const int qi = nq < 1 ? 1 : nq > 7 ? 7 : nq;
    int v = cache[dev][mi][qi].load(std::memory_order_relaxed);
    if (v > 0)
        return v;
    const size_t lds = few_lds_bytes(M, qi, true);
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (M) {
    case 8: e = few_occupancy<8>(&per_cu, qi, lds); break;
    case 16: e = few_occupancy<16>(&per_cu, qi, lds); break;
    case 32: e = few_occupancy<32>(&per_cu, qi, lds); break;
    case 64: e = few_occupancy<64>(&per_cu, qi, lds); break;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    (void)hipGetLastError();
    if (e != hipSuccess || per_cu < 1)
        return cus;   // not cached: no device to ask
    v = per_cu * cus;
    cache[dev][mi][qi].store(v, std::memory_order_relaxed);
    return v;
}

// Rows per workgroup.  Several queries: equal blocks, as many as whole
// rounds of resident workgroups need (so no round runs partly empty).  One
// query: tiles of at most 32768 rows, so that the last round is short and a
// small database still spreads over 2048 workgroups.  Always at most 65536
// rows (16-bit local row indices), at least two passes, a multiple of one
// pass.
int64_t few_rows_per_block(int64_t N, int M, int nq)
{
    const int64_t pass = bolt::few_pass(M);
    int64_t r;
    if (nq == 1) {
        r = (N + 2047) / 2048;
        if (r > 32768)
            r = 32768;
    } else {
        const int64_t slots = few_slots(M, nq);
        const int64_t per_round = slots * (int64_t)bolt::kTileRowsMax;
        const int64_t rounds = N > 0 ? (N + per_round - 1) / per_round : 1;
        r = (N + slots * rounds - 1) / (slots * rounds);
    }
    r = (r + pass - 1) / pass * pass;
    if (r < 2 * pass)
        r = 2 * pass;
    if (r > bolt::kTileRowsMax)
        r = bolt::kTileRowsMax;
    return r;
}

// Stage 1 of the fused few-query path: candidates [Q][n_rb][k] (packed,
// counts [Q][n_rb] in ccnt and histograms in hist, if given) and bounds.
int few_scan_topk(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                  bolt::RankOrder order, int n_rb, uint64_t *cand, uint32_t *ccnt, uint32_t *hist, uint32_t *gthr,
                  const int64_t *tiles, uint32_t *lcnt, hipStream_t s)
{
    const int nq = (int)Q;
    const int64_t rpb = few_rows_per_block(N, M, nq);
    bolt::ProfScope prof_("scan_topk_few", s);
    switch (M) {
    case 8: launch_few_scan_topk<8>(codes, N, luts, nq, k, order, rpb, n_rb, cand, ccnt, hist, gthr, tiles, lcnt,
                                    s); break;
    case 16: launch_few_scan_topk<16>(codes, N, luts, nq, k, order, rpb, n_rb, cand, ccnt, hist, gthr, tiles, lcnt,
                                    s); break;
    case 32: launch_few_scan_topk<32>(codes, N, luts, nq, k, order, rpb, n_rb, cand, ccnt, hist, gthr, tiles, lcnt,
                                    s); break;
    case 64: launch_few_scan_topk<64>(codes, N, luts, nq, k, order, rpb, n_rb, cand, ccnt, hist, gthr, tiles, lcnt,
                                    s); break;
    default: return fail(BOLT_ERR_UNSUPPORTED, "few-query scan takes M in {8, 16, 32, 64}");
    }
    return BOLT_OK;
}

}  // namespace bolt
