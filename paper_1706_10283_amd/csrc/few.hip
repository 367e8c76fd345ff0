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
#include "topk_device.hpp"

namespace {

using bolt::load_row;
using bolt::OutMode;

constexpr int kR = 4;                       // rows per lane per pass
constexpr int kPass = 256 * kR;             // rows per pass
constexpr int kFewCap = 2 * kPass;          // candidate slots per query (fused)
constexpr int kFewRowsMax = 65536;          // rows per workgroup at most (16-bit local rows)

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

// Sums of query q for the kR rows held in cw (pair tables of q at tq).
template <int MM>
__device__ __forceinline__ void sums_for(const uint16_t *tq, const uint32_t (&cw)[kR][MM / 8],
                                         uint32_t (&s)[kR])
{
    const char *tb = reinterpret_cast<const char *>(tq);
    uint32_t part[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r)
        part[r] = 0;
    // one code dword (four pairs) per step keeps 4*kR reads in flight and the
    // register count low
#pragma unroll 1
    for (int t = 0; t < MM / 8; ++t) {
        uint32_t w[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            w[r] = cw[r][0];
#pragma unroll
            for (int v = 1; v < MM / 8; ++v)
                w[r] = (t == v) ? cw[r][v] : w[r];
        }
        const char *tt = tb + t * 4 * 512;
        uint32_t v[kR][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const uint32_t byte = (w[r] >> (8 * j)) & 0xFFu;
                v[r][j] = *reinterpret_cast<const uint16_t *>(tt + j * 512 + 2 * byte);
            }
#pragma unroll
        for (int r = 0; r < kR; ++r)
            part[r] += v[r][0] + v[r][1] + v[r][2] + v[r][3];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r)
        s[r] = part[r];
}

template <int MM>
__device__ __forceinline__ void copy_rows(const uint32_t (&a)[kR][MM / 8], uint32_t (&b)[kR][MM / 8])
{
#pragma unroll
    for (int r = 0; r < kR; ++r)
#pragma unroll
        for (int v = 0; v < MM / 8; ++v)
            b[r][v] = a[r][v];
}

template <int MM>
__device__ __forceinline__ void load_rows(const uint8_t *__restrict__ codes, int64_t base, int64_t r1,
                                          uint32_t (&cw)[kR][MM / 8])
{
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t n = base + threadIdx.x + 256 * r;
        if (n < r1)
            load_row<MM>(codes, n, cw[r]);
        else
#pragma unroll
            for (int v = 0; v < MM / 8; ++v)
                cw[r][v] = 0;
    }
}

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
    uint32_t cw[kR][MM / 8], nx[kR][MM / 8];
    load_rows<MM>(codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += kPass) {
        copy_rows<MM>(nx, cw);
        if (base + kPass < r1)   // next pass in flight while this one is computed
            load_rows<MM>(codes, base + kPass, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[kR];
            sums_for<MM>(pt + q * (MM / 2) * 256, cw, s);
#pragma unroll
            for (int r = 0; r < kR; ++r) {
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
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void few_scan_topk_kernel(const uint8_t *__restrict__ codes,
                                                            int64_t N, const uint8_t *__restrict__ luts,
                                                            int nq, uint32_t k, int largest,
                                                            int64_t rows_per_block, int n_rb,
                                                            uint64_t *__restrict__ cand,
                                                            uint32_t *__restrict__ gthr)
{
    constexpr uint32_t SMAX = 255u * MM;
    extern __shared__ __attribute__((aligned(16))) uint16_t pt[];   // tables, then buffers
    uint32_t *buf = reinterpret_cast<uint32_t *>(pt + nq * (MM / 2) * 256);   // [nq][kFewCap]
    uint32_t *cnt = buf + nq * kFewCap;                                       // [nq]
    uint32_t *bnd = cnt + nq;                                                 // [nq]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rb = blockIdx.x;
    build_pair_tables<MM>(luts, nq, pt);
    if (tid < nq) {
        cnt[tid] = 0;
        bnd[tid] = __atomic_load_n(&gthr[tid], __ATOMIC_RELAXED) + 1u;
    }
    __syncthreads();
    const int64_t r0 = (int64_t)rb * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    int pass = 0;
    uint32_t cw[kR][MM / 8], nx[kR][MM / 8];
    load_rows<MM>(codes, r0, r1, nx);
    for (int64_t base = r0; base < r1; base += kPass, ++pass) {
        copy_rows<MM>(nx, cw);
        if (base + kPass < r1)   // next pass in flight while this one is computed
            load_rows<MM>(codes, base + kPass, r1, nx);
        for (int q = 0; q < nq; ++q) {
            uint32_t s[kR];
            sums_for<MM>(pt + q * (MM / 2) * 256, cw, s);
            const uint32_t bq = bnd[q];
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int64_t n = base + tid + 256 * r;
                const uint32_t d = largest ? SMAX - s[r] : s[r];
                if (n < r1 && d < bq) {
                    const uint32_t pos = atomicAdd(&cnt[q], 1u);
                    buf[q * kFewCap + pos] = bolt::local_key(d, (uint32_t)(n - r0));
                }
            }
        }
        __syncthreads();
        const bool refresh = (pass & 7) == 7;
        for (int q = wave; q < nq; q += 4) {
            const uint32_t c = cnt[q];
            uint32_t nb = 0xFFFFFFFFu;
            if (c > kFewCap - kPass) {
                bolt::PruneResult pr = bolt::prune_local_lds<kFewCap>(buf + q * kFewCap, c, k, false);
                if (pr.count > kFewCap - kPass)
                    pr = bolt::prune_local_lds<kFewCap>(buf + q * kFewCap, pr.count, k, true);
                if (lane == 0) {
                    cnt[q] = pr.count;
                    if (pr.T <= 0xFFFFu)
                        atomicMin(&gthr[q], pr.T);
                }
                nb = pr.T;
            }
            if (lane == 0 && (nb != 0xFFFFFFFFu || refresh)) {
                uint32_t b = bnd[q];
                b = nb < b ? nb : b;
                const uint32_t gb = __atomic_load_n(&gthr[q], __ATOMIC_RELAXED) + 1u;
                bnd[q] = gb < b ? gb : b;
            }
        }
        __syncthreads();
    }
    for (int q = wave; q < nq; q += 4) {
        uint32_t n = cnt[q];
        uint32_t *bq = buf + q * kFewCap;
        if (n > k) {
            const bolt::PruneResult pr = bolt::prune_local_lds<kFewCap>(bq, n, k, true);
            n = pr.count;
            if (lane == 0)
                atomicMin(&gthr[q], pr.T);
        }
        uint64_t *dst = cand + ((int64_t)q * n_rb + rb) * (int64_t)k;
        for (uint32_t j = lane; j < k; j += 64) {
            uint64_t key = ~0ull;
            if (j < n) {
                const uint32_t lk = bq[j];
                key = ((uint64_t)(lk >> 16) << 32) | (uint64_t)(r0 + (lk & 0xFFFFu));
            }
            dst[j] = key;
        }
    }
}

size_t few_lds_bytes(int M, int nq, bool fused)
{
    size_t b = (size_t)nq * (M / 2) * 256 * sizeof(uint16_t);
    if (fused)
        b += (size_t)nq * (kFewCap + 2) * sizeof(uint32_t);
    return b;
}

template <int MM, OutMode OUT>
void launch_few_scan(const uint8_t *codes, int64_t N, const uint8_t *luts, int nq, uint16_t *out,
                     float *outf, int64_t ldo, float bias, float scale, hipStream_t s)
{
    const int64_t rpb = bolt::few_rows_per_block(N);
    const dim3 grid((unsigned)((N + rpb - 1) / rpb));
    hipLaunchKernelGGL((few_scan_kernel<MM, OUT>), grid, dim3(256), few_lds_bytes(MM, nq, false), s,
                       codes, N, luts, nq, rpb, out, outf, ldo, bias, scale);
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
