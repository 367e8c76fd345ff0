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
#include "common.hpp"
#include "scan_common.hpp"
#include "tiles.hpp"

namespace {

using bolt::load_row;
using bolt::OutMode;

constexpr int kPass = bolt::kFewPass;        // rows per pass
constexpr int kFewRowsMax = bolt::kTileRowsMax;

using bolt::build_pair_tables;
using bolt::copy_rows4;
using bolt::load_rows4;
using bolt::pair_sums;

// ------------------------------------------------------------------ plain

template <int MM, OutMode OUT>
__global__ __launch_bounds__(256) void few_scan_kernel(const uint8_t *__restrict__ codes, int64_t N,
                                                       const uint8_t *__restrict__ luts, int nq,
                                                       int64_t rows_per_block,
                                                       uint16_t *__restrict__ out,
                                                       float *__restrict__ outf, int64_t ldo,
                                                       float bias, float scale)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t pt[];   // [nq][MM/2][256]
    build_pair_tables<MM>(luts, nq, pt);
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    uint32_t cw[bolt::kFewR][MM / 8], nx[bolt::kFewR][MM / 8];
    load_rows4<MM>(codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += kPass) {
        copy_rows4<MM>(nx, cw);
        if (base + kPass < r1)   // next pass in flight while this one is computed
            load_rows4<MM>(codes, base + kPass, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[bolt::kFewR];
            pair_sums<MM>(pt + q * (MM / 2) * 256, cw, s);
#pragma unroll
            for (int r = 0; r < bolt::kFewR; ++r) {
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
    int largest, int64_t rows_per_block, int n_rb, uint64_t *__restrict__ cand,
    uint32_t *__restrict__ gthr)
{
    extern __shared__ __attribute__((aligned(16))) char few_lds[];
    bolt::TileJob job;
    job.codes = codes;
    job.luts = luts;
    job.cand = cand;
    job.gthr = gthr;
    job.rb = blockIdx.x;
    job.r0 = job.rb * rows_per_block;
    job.r1 = (job.r0 + rows_per_block) < N ? (job.r0 + rows_per_block) : N;
    job.n_rb = n_rb;
    job.q0 = 0;
    job.nq = nq;
    job.k = k;
    job.largest = largest;
    bolt::few_tile<MM>(job, few_lds);
}

size_t few_lds_bytes(int M, int nq, bool fused)
{
    return fused ? bolt::few_tile_lds_bytes(M, nq) : (size_t)nq * (M / 2) * 256 * sizeof(uint16_t);
}

template <int MM, OutMode OUT>
void launch_few_scan(const uint8_t *codes, int64_t N, const uint8_t *luts, int nq, uint16_t *out,
                     float *outf, int64_t ldo, float bias, float scale, hipStream_t s)
{
    const int64_t rpb = bolt::few_rows_per_block(N);
    const dim3 grid((unsigned)((N + rpb - 1) / rpb));
    {
        bolt::ProfScope prof_("scan_few", s);
        hipLaunchKernelGGL((few_scan_kernel<MM, OUT>), grid, dim3(256), few_lds_bytes(MM, nq, false), s,
                           codes, N, luts, nq, rpb, out, outf, ldo, bias, scale);
    }
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

// Rows per workgroup: enough workgroups to fill the GPU (about 4 per CU),
// at most 65536 rows (16-bit local row indices), a multiple of one pass.
size_t few_fused_lds_bytes(int M, int nq) { return few_lds_bytes(M, nq, true); }

int64_t few_rows_per_block(int64_t N)
{
    int64_t r = (N + 1023) / 1024;
    r = (r + kPass - 1) / kPass * kPass;
    if (r < 4 * kPass)
        r = 4 * kPass;
    if (r > kFewRowsMax)
        r = kFewRowsMax;
    return r;
}

// Stage 1 of the fused few-query path: candidates [Q][n_rb][k] and bounds.
int few_scan_topk(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, int k,
                  bool largest, int n_rb, uint64_t *cand, uint32_t *gthr, hipStream_t s)
{
    const int64_t rpb = few_rows_per_block(N);
    const int nq = (int)Q;
    const size_t lds = few_lds_bytes(M, nq, true);
    bolt::ProfScope prof_("scan_topk_few", s);
    switch (M) {
    case 8:
        hipLaunchKernelGGL(few_scan_topk_kernel<8>, dim3(n_rb), dim3(256), lds, s, codes, N, luts, nq,
                           (uint32_t)k, (int)largest, rpb, n_rb, cand, gthr);
        break;
    case 16:
        hipLaunchKernelGGL(few_scan_topk_kernel<16>, dim3(n_rb), dim3(256), lds, s, codes, N, luts, nq,
                           (uint32_t)k, (int)largest, rpb, n_rb, cand, gthr);
        break;
    case 32:
        hipLaunchKernelGGL(few_scan_topk_kernel<32>, dim3(n_rb), dim3(256), lds, s, codes, N, luts, nq,
                           (uint32_t)k, (int)largest, rpb, n_rb, cand, gthr);
        break;
    case 64:
        hipLaunchKernelGGL(few_scan_topk_kernel<64>, dim3(n_rb), dim3(256), lds, s, codes, N, luts, nq,
                           (uint32_t)k, (int)largest, rpb, n_rb, cand, gthr);
        break;
    default: return fail(BOLT_ERR_UNSUPPORTED, "few-query scan takes M in {8, 16, 32, 64}");
    }
    return BOLT_OK;
}

}  // namespace bolt
