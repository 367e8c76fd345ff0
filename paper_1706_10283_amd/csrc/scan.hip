// The scan d_hat for gfx950 (Sec. 3.1: the approximate distance is the sum
// of the table entries selected by the codes; Sec. 3.2: lookups vectorised
// over many encoded vectors at once).
//
//   out[q][n] = sum over m of lut[q][m][code(n, m)]       (exact integer)
//
// Three kernels, chosen by the number of queries:
//
// * scan_grouped<MM, NG> (many queries).  The tables of 8*NG queries are
//   re-laid out in LDS so that one table entry (m, c) holds the 8 queries of
//   a group as 8 uint16 lanes (16 bytes).  A lane owns one encoded vector:
//   it computes the LDS byte address (m*16 + c_m)*16 once per subspace and
//   then, for every group g, one 16-byte LDS read at immediate offset
//   g*MM*256 returns that vector's entries for 8 queries, already widened to
//   16 bits.  Two subspaces are folded per add3, so the VALU cost is about a
//   quarter of an instruction per lookup and the kernel runs at the LDS read
//   bandwidth (2 bytes per lookup).  A uint16 lane cannot carry into its
//   neighbour because 255 * M < 65536.
// * few.hip (1..7 queries, the HBM-bound case): pair tables, one 16-bit LDS
//   read per code byte.
// * scan_generic (any even M): the plain per-row loop, used for widths
//   without a tuned kernel.
//
// Output modes: uint16 sums [Q][ldo]; fp32 rescaled sums [Q][ldo] or
// [N][ldo] for the approximate matrix product (out = (S + bias) * scale).
#include "common.hpp"
#include "scan_common.hpp"
#include "tiles.hpp"

namespace {

using bolt::OutMode;
using bolt::load_row;
using bolt::code_at;

template <OutMode OUT>
__device__ __forceinline__ void emit(uint32_t s, int64_t q, int64_t n, uint16_t *__restrict__ out,
                                     float *__restrict__ outf, int64_t ldo, float bias, float scale)
{
    if (OUT == OutMode::U16) {
        out[q * ldo + n] = (uint16_t)s;
    } else {
        float t = (float)s + bias;
        float v = t * scale;
        if (OUT == OutMode::F32)
            outf[q * ldo + n] = v;
        else
            outf[n * ldo + q] = v;
    }
}

// ---------------------------------------------------------------- many queries

template <int MM, int NG, OutMode OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MM >= 256 ? 2 : 4))) void scan_grouped_kernel(
    const uint8_t *__restrict__ codes, int64_t N, const uint8_t *__restrict__ luts, int64_t Q,
    int64_t rows_per_block, uint16_t *__restrict__ out, float *__restrict__ outf, int64_t ldo,
    float bias, float scale)
{
    constexpr int QG = 8;               // queries per group (uint16 lanes of a 16-byte read)
    constexpr int QB = QG * NG;         // queries per workgroup
    constexpr int GROUP_BYTES = MM * 16 * QG * 2;
    static_assert(NG * GROUP_BYTES <= 65536, "immediate LDS offsets are 16 bits");
    __shared__ uint4 tab[NG * GROUP_BYTES / 16];

    const int64_t q0 = (int64_t)blockIdx.y * QB;
    const int nq = (int)((Q - q0) < QB ? (Q - q0) : QB);
    // stage: tab[g][m][c][qq] = lut[q0 + 8g + qq][m][c]  (0 for missing queries)
    uint16_t *tab16 = reinterpret_cast<uint16_t *>(tab);
    for (int e = threadIdx.x; e < NG * MM * 16 * QG; e += 256) {
        const int qq = e & 7, c = (e >> 3) & 15;
        const int m = (e >> 7) % MM, g = (e >> 7) / MM;
        const int q = g * QG + qq;
        tab16[e] = q < nq ? luts[(q0 + q) * MM * 16 + m * 16 + c] : (uint16_t)0;
    }
    __syncthreads();

    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    const char *tabb = reinterpret_cast<const char *>(tab);
    constexpr int GU = NG >= 2 ? 2 : 1;   // groups per pass: the second one at an immediate offset
    constexpr int NW = MM / 8;            // code dwords per row (8 subspaces each)
    for (int64_t n = r0 + threadIdx.x; n < r1; n += 256) {
        uint32_t cw[NW];
        load_row<MM>(codes, n, cw);
#pragma unroll 1
        for (int g = 0; g < NG; g += GU) {
            if (g * QG >= nq)
                break;
            const char *tg = tabb + g * GROUP_BYTES;
            uint32_t acc[GU][4];
#pragma unroll
            for (int u = 0; u < GU; ++u)
                acc[u][0] = acc[u][1] = acc[u][2] = acc[u][3] = 0;
            // one code dword (8 subspaces) per step keeps 8*GU reads in flight
#pragma unroll 1
            for (int t = 0; t < NW; ++t) {
                uint32_t w = cw[0];
#pragma unroll
                for (int v = 1; v < NW; ++v)
                    w = (t == v) ? cw[v] : w;
                const char *tt = tg + t * 8 * 256;
#pragma unroll
                for (int k = 0; k < 8; k += 2) {
                    const uint32_t am = (uint32_t)(k * 256) + (((w >> (4 * k)) & 15u) << 4);
                    const uint32_t am1 = (uint32_t)((k + 1) * 256) + (((w >> (4 * k + 4)) & 15u) << 4);
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
            for (int u = 0; u < GU; ++u)
#pragma unroll
                for (int d = 0; d < 4; ++d)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int q = (g + u) * QG + 2 * d + h;
                        if (q < nq)
                            emit<OUT>((acc[u][d] >> (16 * h)) & 0xFFFFu, q0 + q, n, out, outf, ldo,
                                      bias, scale);
                    }
        }
    }
}

// ---------------------------------------------------------------- any even M

template <OutMode OUT>
__global__ __launch_bounds__(256) void scan_generic_kernel(
    const uint8_t *__restrict__ codes, int64_t N, int M, const uint8_t *__restrict__ luts,
    int64_t Q, int qb, int64_t rows_per_block, uint16_t *__restrict__ out,
    float *__restrict__ outf, int64_t ldo, float bias, float scale)
{
    extern __shared__ uint8_t tabg[];   // [qb][M][16]
    const int64_t q0 = (int64_t)blockIdx.y * qb;
    const int nq = (int)((Q - q0) < qb ? (Q - q0) : qb);
    for (int e = threadIdx.x; e < nq * M * 16; e += 256)
        tabg[e] = luts[q0 * M * 16 + e];
    __syncthreads();
    const int bpr = M / 2;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    for (int64_t n = r0 + threadIdx.x; n < r1; n += 256) {
        const uint8_t *row = codes + n * bpr;
        for (int q = 0; q < nq; ++q) {
            uint32_t s = 0;
            for (int t = 0; t < bpr; ++t) {
                const uint32_t byte = row[t];
                s += tabg[(q * M + 2 * t) * 16 + (byte & 15u)];
                s += tabg[(q * M + 2 * t + 1) * 16 + (byte >> 4)];
            }
            emit<OUT>(s, q0 + q, n, out, outf, ldo, bias, scale);
        }
    }
}

// ---------------------------------------------------------------- dispatch

// Rows per workgroup: about target_blocks workgroups in all, but at least
// 2048 rows so that staging the query tables stays a small part of the work.
int64_t rows_per_block_for(int64_t N, int64_t n_qblocks, int64_t target_blocks)
{
    int64_t want = (N * n_qblocks + target_blocks - 1) / target_blocks;
    want = (want + 255) / 256 * 256;
    if (want < 2048)
        want = 2048;
    return want;
}

template <int MM, int NG, OutMode OUT>
void launch_grouped(const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q, uint16_t *out,
                    float *outf, int64_t ldo, float bias, float scale, hipStream_t s)
{
    const int64_t qblocks = (Q + 8 * NG - 1) / (8 * NG);
    const int64_t rpb = rows_per_block_for(N, qblocks, 4096);
    dim3 grid((unsigned)((N + rpb - 1) / rpb), (unsigned)qblocks);
    {
        bolt::ProfScope prof_("scan_grouped", s);
        hipLaunchKernelGGL((scan_grouped_kernel<MM, NG, OUT>), grid, dim3(256), 0, s, codes, N, luts, Q,
                           rpb, out, outf, ldo, bias, scale);
    }
}

// ---------------------------------------------------------------- matrix cores

// Many queries on the int8 matrix cores (the one-hot contraction of
// tiles.hpp with tables as T - 128, so acc + 128 M is the exact sum):
// workgroup (row block, block of 32 NT queries), passes of 128 rows with
// the codes one pass ahead.  Each lane holds four runs of four consecutive
// rows of one query: written as 8-byte (uint16) or 16-byte (fp32) words
// when the layout allows (vec), else element by element; the transposed
// fp32 layout writes 32 consecutive queries of a row per store.
template <int MM, int NT, OutMode OUT, bool SP>
__global__ __launch_bounds__(256) void scan_mfma_kernel(const uint8_t *__restrict__ codes, int64_t N,
                                                        const uint8_t *__restrict__ luts, int64_t Q, int64_t rpb,
                                                        uint16_t *__restrict__ out, float *__restrict__ outf,
                                                        int64_t ldo, float bias, float scale, int vec)
{
    constexpr int NW = MM / 8;
    constexpr int OFF = 128 * MM;
    __shared__ bolt::OneHot onehot;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, col = lane & 31;
    const int64_t q0 = (int64_t)blockIdx.y * 32 * NT;
    const int nq = (int)((Q - q0) < 32 * NT ? (Q - q0) : 32 * NT);
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = (r0 + rpb) < N ? (r0 + rpb) : N;
    bolt::onehot_init(onehot);
    bolt::i32x4 tb[NT][MM / 2];
    bolt::mfma_load_tables<MM, NT>(luts, q0, nq, bolt::one_order(false), tb);
    __syncthreads();
    uint32_t nxt[NW];
    {
        const int64_t n = r0 + 32 * wave + col;
        load_row<MM>(codes, n < r1 ? n : r1 - 1, nxt);
    }
    for (int64_t base = r0; base < r1; base += bolt::kMfmaPass) {
        uint32_t cw[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v)
            cw[v] = nxt[v];
        {
            const int64_t nn = base + bolt::kMfmaPass + 32 * wave + col;
            load_row<MM>(codes, nn < r1 ? nn : r1 - 1, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);
        bolt::i32x16 acc[NT];
        bolt::mfma_pass<MM, NT, SP>(cw, onehot, tb, acc);
        const int64_t rl = base + 32 * wave + 4 * half;   // first row of this lane's runs
        const bool full = base + bolt::kMfmaPass <= r1;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t q = q0 + 32 * t + col;
            if (32 * t + col >= nq)
                continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = rl + 8 * j;
                uint32_t sv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    sv[i] = (uint32_t)(acc[t][4 * j + i] + OFF);
                if (full && vec && OUT == OutMode::U16) {
                    *reinterpret_cast<uint2 *>(out + q * ldo + row) =
                        make_uint2(sv[0] | (sv[1] << 16), sv[2] | (sv[3] << 16));
                } else if (full && vec && OUT == OutMode::F32) {
                    float f[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float tt = (float)sv[i] + bias;
                        f[i] = tt * scale;
                    }
                    *reinterpret_cast<float4 *>(outf + q * ldo + row) = make_float4(f[0], f[1], f[2], f[3]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (full || row + i < r1)
                            emit<OUT>(sv[i], q, row + i, out, outf, ldo, bias, scale);
                }
            }
        }
    }
}

template <int MM, OutMode OUT>
void launch_mfma(const uint8_t *codes, int64_t N, const uint8_t *luts, int64_t Q, uint16_t *out, float *outf,
                 int64_t ldo, float bias, float scale, hipStream_t s)
{
    constexpr int NT = 1;   // one 32-query tile per wave: half the table registers, twice the waves
    const int64_t qblocks = (Q + 32 * NT - 1) / (32 * NT);
    // about 2048 workgroups, whole passes, 512..16384 rows each
    int64_t rpb = (N * qblocks + 2047) / 2048;
    rpb = (rpb + bolt::kMfmaPass - 1) / bolt::kMfmaPass * bolt::kMfmaPass;
    rpb = rpb < 512 ? 512 : (rpb > 16384 ? 16384 : rpb);
    const int vec = OUT == OutMode::U16 ? (ldo % 4 == 0 && bolt::aligned(out, 8))
                                        : (OUT == OutMode::F32 ? (ldo % 4 == 0 && bolt::aligned(outf, 16)) : 0);
    dim3 grid((unsigned)((N + rpb - 1) / rpb), (unsigned)qblocks);
    bolt::ProfScope prof_("scan_mfma", s);
    // the dense instruction: this kernel is bound by its output writes, and
    // the sparse one measured slower here (matrix product, K = 1024: 0.23
    // against 0.19 ms)
    hipLaunchKernelGGL((scan_mfma_kernel<MM, NT, OUT, false>), grid, dim3(256), 0, s, codes, N, luts, Q, rpb, out,
                       outf, ldo, bias, scale, vec);
}

template <OutMode OUT>
int scan_dispatch(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q,
                  uint16_t *out, float *outf, int64_t ldo, float bias, float scale, hipStream_t s,
                  int force_kernel)
{
    // grid.y is at most 65535 query blocks: split very large query counts
    constexpr int64_t kMaxQ = 65535LL * 8;
    if (Q > kMaxQ) {
        for (int64_t q0 = 0; q0 < Q; q0 += kMaxQ) {
            const int64_t nq = (Q - q0) < kMaxQ ? (Q - q0) : kMaxQ;
            int st = scan_dispatch<OUT>(codes, N, M, luts + q0 * M * 16, nq,
                                        OUT == OutMode::U16 ? out + q0 * ldo : out,
                                        OUT == OutMode::F32 ? outf + q0 * ldo
                                                            : (OUT == OutMode::F32T ? outf + q0 : outf),
                                        ldo, bias, scale, s, force_kernel);
            if (st)
                return st;
        }
        return BOLT_OK;
    }
    const bool vec_ok = bolt::aligned(codes, 16) && bolt::aligned(luts, 16);
    // force_kernel: -1 automatic, 0 generic, 1 small, 2 grouped, 3 matrix cores (tests)
    int kind = force_kernel;
    const bool tuned_M = (M == 8 || M == 16 || M == 32 || M == 64 || M == 128 || M == 256);
    const bool few_M = (M == 8 || M == 16 || M == 32 || M == 64);
    if (kind < 0)
        kind = (!tuned_M || !vec_ok) ? 0 : (Q < bolt::kSmallQ ? (few_M ? 1 : 2) : (few_M && Q >= 32 ? 3 : 2));
    if ((kind == 1 && (!few_M || !vec_ok)) || (kind == 2 && (!tuned_M || !vec_ok)) ||
        (kind == 3 && (!few_M || !vec_ok)))
        return bolt::fail(BOLT_ERR_UNSUPPORTED, "tuned scan kernels need a power-of-two M (8..64 for few queries "
                                                "and the matrix cores, 8..256 otherwise) and 16-byte aligned "
                                                "codes/tables");
    if (kind == 1 && Q >= bolt::kSmallQ)
        return bolt::fail(BOLT_ERR_UNSUPPORTED, "small-Q scan handles at most %d queries", bolt::kSmallQ - 1);
    if (kind == 0) {
        int qb = 16384 / (M * 16);
        if (qb < 1)
            qb = 1;
        const int64_t qblocks = (Q + qb - 1) / qb;
        const int64_t rpb = rows_per_block_for(N, qblocks, 4096);
        dim3 grid((unsigned)((N + rpb - 1) / rpb), (unsigned)qblocks);
        {
            bolt::ProfScope prof_("scan_generic", s);
            hipLaunchKernelGGL(scan_generic_kernel<OUT>, grid, dim3(256), qb * M * 16, s, codes, N, M,
                               luts, Q, qb, rpb, out, outf, ldo, bias, scale);
        }
    } else if (kind == 1) {
        return bolt::few_scan<OUT>(codes, N, M, luts, Q, out, outf, ldo, bias, scale, s);
    } else if (kind == 3) {
        switch (M) {
        case 8: launch_mfma<8, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 16: launch_mfma<16, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 32: launch_mfma<32, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 64: launch_mfma<64, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        }
    } else {
        switch (M) {
        case 8: launch_grouped<8, 16, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 16: launch_grouped<16, 8, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 32: launch_grouped<32, 4, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 64: launch_grouped<64, 2, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 128: launch_grouped<128, 1, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        case 256: launch_grouped<256, 1, OUT>(codes, N, luts, Q, out, outf, ldo, bias, scale, s); break;
        }
    }
    return bolt::check_launch("bolt scan");
}

int scan_common(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8, int64_t Q,
                uint16_t *out, int64_t ldo, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(check_N(N, "N"));
    BOLT_TRY(check_N(Q, "Q"));
    if (ldo < N)
        return fail(BOLT_ERR_INVALID, "ldo (%lld) < N (%lld)", (long long)ldo, (long long)N);
    if (N == 0 || Q == 0)
        return BOLT_OK;
    if (!codes || !luts_u8 || !out)
        return fail(BOLT_ERR_INVALID, "bolt_scan: null pointer");
    return scan_dispatch<OutMode::U16>(codes, N, M, luts_u8, Q, out, nullptr, ldo, 0.f, 0.f,
                                       as_stream(stream), g_force_scan_kernel);
}

}  // namespace

namespace bolt {
int g_force_scan_kernel = -1;

int scan_u16(const uint8_t *codes, int64_t N, int M, const uint8_t *luts, int64_t Q, uint16_t *out,
             int64_t ldo, hipStream_t s)
{
    return scan_dispatch<OutMode::U16>(codes, N, M, luts, Q, out, nullptr, ldo, 0.f, 0.f, s,
                                       g_force_scan_kernel);
}
}  // namespace bolt

extern "C" int bolt_scan_l2(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                            int64_t Q, uint16_t *out, int64_t ldo, void *stream)
{
    return scan_common(codes, N, M, luts_u8, Q, out, ldo, stream);
}

extern "C" int bolt_scan_dot(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                             int64_t Q, uint16_t *out, int64_t ldo, void *stream)
{
    return scan_common(codes, N, M, luts_u8, Q, out, ldo, stream);
}

extern "C" int bolt_amm(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *luts_u8,
                        int64_t K, float bias, float scale, float *out, int64_t ldo,
                        int32_t transpose, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(check_N(N, "N"));
    BOLT_TRY(check_N(K, "K"));
    if (transpose != 0 && transpose != 1)
        return fail(BOLT_ERR_INVALID, "transpose must be 0 or 1");
    if ((transpose == 0 && ldo < N) || (transpose == 1 && ldo < K))
        return fail(BOLT_ERR_INVALID, "ldo too small (%lld)", (long long)ldo);
    if (N == 0 || K == 0)
        return BOLT_OK;
    if (!codes || !luts_u8 || !out)
        return fail(BOLT_ERR_INVALID, "bolt_amm: null pointer");
    hipStream_t s = as_stream(stream);
    if (transpose)
        return scan_dispatch<OutMode::F32T>(codes, N, M, luts_u8, K, nullptr, out, ldo, bias, scale,
                                            s, g_force_scan_kernel);
    return scan_dispatch<OutMode::F32>(codes, N, M, luts_u8, K, nullptr, out, ldo, bias, scale, s,
                                       g_force_scan_kernel);
}

// Test hook: pin the scan kernel choice (-1 automatic, 0 generic, 1 few-query, 2 grouped,
// 3 matrix cores).
extern "C" int bolt_debug_force_scan_kernel(int32_t kind)
{
    if (kind < -1 || kind > 3)
        return bolt::fail(BOLT_ERR_INVALID, "kind must be -1..3");
    bolt::g_force_scan_kernel = kind;
    return BOLT_OK;
}
