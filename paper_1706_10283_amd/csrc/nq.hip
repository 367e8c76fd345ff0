// Bolt No Quantize (Sec. 4.2): the scan of Sec. 3.1 with the float tables
// D instead of their uint8 quantisation, the paper's control for what the
// quantiser costs in accuracy, and top-k on the float sums.
//
// The float sum is defined in one order: acc = 0, then acc = acc + D[m][c_m]
// for m = 0, 1, ..., M-1, each add rounded to nearest in fp32 (no fused
// operations), so the result is reproducible bit for bit.
//
// Scan: a workgroup serves 8 queries as two groups of 4; its LDS holds
// entry (g, m, c) as the 4 queries' floats (16 bytes), so one 16-byte read
// per code nibble and group feeds four accumulators.  A lane owns one row;
// code dwords are read from global memory (rows of any even M).
//
// Top-k: per query the k smallest (or largest) values, ties by ascending
// index, found exactly by a four-level radix select over order-preserving
// 32-bit keys, then sorted by (key, index).
#include "common.hpp"
#include "scan_common.hpp"

namespace {

constexpr int kQB = 8;   // queries per workgroup (two groups of four)

__global__ __launch_bounds__(256) void scan_f32_kernel(const uint8_t *__restrict__ codes, int64_t N, int M,
                                                       const float *__restrict__ luts, int64_t Q,
                                                       float *__restrict__ out, int64_t ldo,
                                                       int64_t rows_per_block)
{
    extern __shared__ __attribute__((aligned(16))) float4 tab[];   // [g][m][c], g < 2
    const int tid = threadIdx.x;
    const int64_t q0 = (int64_t)blockIdx.y * kQB;
    const int nq = (int)((Q - q0) < kQB ? (Q - q0) : kQB);
    float *t = reinterpret_cast<float *>(tab);
    for (int e = tid; e < 2 * M * 16 * 4; e += 256) {
        const int qq = e & 3, c = (e >> 2) & 15;
        const int m = (e >> 6) % M, g = (e >> 6) / M;
        const int q = g * 4 + qq;
        t[e] = q < nq ? luts[((q0 + q) * M + m) * 16 + c] : 0.0f;
    }
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block) < N ? (r0 + rows_per_block) : N;
    const int bpr = M >> 1;
    for (int64_t n = r0 + tid; n < r1; n += 256) {
        const uint8_t *row = codes + n * bpr;
        float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int b0 = 0; b0 < bpr; b0 += 4) {
            uint32_t w;
            if (b0 + 4 <= bpr && ((reinterpret_cast<uintptr_t>(row) & 3) == 0)) {
                w = *reinterpret_cast<const uint32_t *>(row + b0);
            } else {
                w = 0;
                for (int b = 0; b < 4 && b0 + b < bpr; ++b)
                    w |= (uint32_t)row[b0 + b] << (8 * b);
            }
            const int nb = (bpr - b0) < 4 ? (bpr - b0) : 4;
            for (int j = 0; j < 2 * nb; ++j) {
                const int m = 2 * b0 + j;
                const uint32_t c = (w >> (4 * j)) & 15u;
                const float4 x = tab[(0 * M + m) * 16 + c];
                const float4 y = tab[(1 * M + m) * 16 + c];
                a[0] = a[0] + x.x;
                a[1] = a[1] + x.y;
                a[2] = a[2] + x.z;
                a[3] = a[3] + x.w;
                a[4] = a[4] + y.x;
                a[5] = a[5] + y.y;
                a[6] = a[6] + y.z;
                a[7] = a[7] + y.w;
            }
        }
#pragma unroll
        for (int q = 0; q < kQB; ++q)
            if (q < nq)
                out[(q0 + q) * ldo + n] = a[q];
    }
}

// Order-preserving map of a finite float to 32 bits (ascending).
__device__ __forceinline__ uint32_t fkey(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float fkey_inv(uint32_t k)
{
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

constexpr int kT = 256;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *wave_sums, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += y;
    }
    if (lane == 63)
        wave_sums[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kT / 64; ++w) {
        const uint32_t s = wave_sums[w];
        before += (w < wave) ? s : 0;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// One workgroup per row of dists.  flip = 0: k smallest; ~0: k largest
// (keys are complemented, so the k smallest keys are wanted either way).
__global__ __launch_bounds__(kT) void topk_f32_kernel(const float *__restrict__ d, int64_t N, int64_t ldd, int k,
                                                      uint32_t flip, float *__restrict__ vals,
                                                      int32_t *__restrict__ idx)
{
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sel[BOLT_TOPK_MAX_K];
    __shared__ uint32_t wave_sums[kT / 64];
    __shared__ uint32_t sh_prefix, sh_lt, sh_nlt;
    const int tid = threadIdx.x;
    const int64_t q = blockIdx.x;
    const float *row = d + q * ldd;
    const int kk = ((int64_t)k < N) ? k : (int)N;

    uint32_t T = 0, count_lt = 0, need_eq = 0;
    bool take_all = (int64_t)kk == N;
    if (!take_all) {
        // four levels of 8 bits, high to low: the k-th smallest key T
        uint32_t prefix = 0, lt = 0;
        for (int level = 0; level < 4; ++level) {
            const int shift = 24 - 8 * level;
            const uint32_t hmask = level == 0 ? 0u : (0xFFFFFFFFu << (shift + 8));
            hist[tid] = 0;
            __syncthreads();
            for (int64_t i = tid; i < N; i += kT) {
                const uint32_t key = fkey(row[i]) ^ flip;
                if ((key & hmask) == prefix)
                    atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t cum = lt;
                int B = 0;
                for (; B < 255; ++B) {
                    if (cum + hist[B] >= (uint32_t)k)
                        break;
                    cum += hist[B];
                }
                sh_prefix = prefix | ((uint32_t)B << shift);
                sh_lt = cum;
            }
            __syncthreads();
            prefix = sh_prefix;
            lt = sh_lt;
            __syncthreads();
        }
        T = prefix;
        count_lt = lt;
        need_eq = (uint32_t)k - count_lt;
    }

    // collect: every key below T, then the first need_eq keys equal to T in index order
    if (tid == 0)
        sh_nlt = 0;
    __syncthreads();
    uint32_t eq_base = 0;
    for (int64_t c0 = 0; c0 < N; c0 += (int64_t)kT * 8) {
        const int64_t i0 = c0 + (int64_t)tid * 8;
        uint32_t key[8];
        uint32_t my_eq = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            key[e] = 0;
            if (i0 + e < N) {
                key[e] = fkey(row[i0 + e]) ^ flip;
                if (take_all || key[e] < T) {
                    const uint32_t pos = atomicAdd(&sh_nlt, 1u);
                    sel[pos] = ((uint64_t)key[e] << 32) | (uint64_t)(i0 + e);
                } else if (key[e] == T) {
                    ++my_eq;
                }
            }
        }
        uint32_t total;
        uint32_t r = eq_base + block_exclusive_scan(my_eq, wave_sums, &total);
        if (my_eq) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (i0 + e < N && !take_all && key[e] == T) {
                    if (r < need_eq)
                        sel[count_lt + r] = ((uint64_t)T << 32) | (uint64_t)(i0 + e);
                    ++r;
                }
            }
        }
        eq_base += total;
        if (!take_all && eq_base >= need_eq && sh_nlt == count_lt)
            break;
        __syncthreads();
    }
    __syncthreads();

    int P = 1;
    while (P < kk)
        P <<= 1;
    for (int i = kk + tid; i < P; i += kT)
        sel[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P / 2; t += kT) {
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
    for (int r = tid; r < k; r += kT) {
        if (r < kk) {
            vals[q * k + r] = fkey_inv((uint32_t)(sel[r] >> 32) ^ flip);
            idx[q * k + r] = (int32_t)(sel[r] & 0xFFFFFFFFu);
        } else {
            vals[q * k + r] = flip ? -__builtin_inff() : __builtin_inff();
            idx[q * k + r] = -1;
        }
    }
}

}  // namespace

extern "C" int bolt_scan_f32(const uint8_t *codes, int64_t N, int32_t M, const float *luts_f32, int64_t Q,
                             float *out, int64_t ldo, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_M(M));
    BOLT_TRY(check_N(N, "N"));
    BOLT_TRY(check_N(Q, "Q"));
    if (ldo < N)
        return fail(BOLT_ERR_INVALID, "ldo (%lld) < N (%lld)", (long long)ldo, (long long)N);
    if (N == 0 || Q == 0)
        return BOLT_OK;
    if (!codes || !luts_f32 || !out)
        return fail(BOLT_ERR_INVALID, "bolt_scan_f32: null pointer");
    hipStream_t s = as_stream(stream);
    const int64_t n_qb = (Q + kQB - 1) / kQB;
    if (n_qb > 65535)
        return fail(BOLT_ERR_UNSUPPORTED, "bolt_scan_f32 takes at most %d queries per call", 65535 * kQB);
    // enough row blocks to fill the GPU, at least 1024 rows each
    int64_t rpb = (N * n_qb + 2047) / 2048;
    rpb = rpb < 1024 ? 1024 : (rpb + 255) / 256 * 256;
    const int64_t n_rb = (N + rpb - 1) / rpb;
    const size_t lds = (size_t)2 * M * 16 * sizeof(float4);
    {
        bolt::ProfScope prof_("scan_f32", s);
        hipLaunchKernelGGL(scan_f32_kernel, dim3((unsigned)n_rb, (unsigned)n_qb), dim3(256), lds, s, codes, N, M,
                           luts_f32, Q, out, ldo, rpb);
    }
    return check_launch("bolt_scan_f32");
}

extern "C" int bolt_topk_f32(const float *dists, int64_t Q, int64_t N, int64_t ldd, int32_t k, int32_t largest,
                             float *vals, int32_t *idx, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_N(Q, "Q"));
    BOLT_TRY(check_N(N, "N"));
    if (k < 1)
        return fail(BOLT_ERR_INVALID, "k must be >= 1 (got %d)", k);
    if (k > BOLT_TOPK_MAX_K)
        return fail(BOLT_ERR_UNSUPPORTED, "k must be <= %d (got %d)", BOLT_TOPK_MAX_K, k);
    if (ldd < N)
        return fail(BOLT_ERR_INVALID, "ldd (%lld) < N (%lld)", (long long)ldd, (long long)N);
    if (Q == 0)
        return BOLT_OK;
    if (!vals || !idx || (N > 0 && !dists))
        return fail(BOLT_ERR_INVALID, "bolt_topk_f32: null pointer");
    hipStream_t s = as_stream(stream);
    {
        bolt::ProfScope prof_("topk_f32", s);
        hipLaunchKernelGGL(topk_f32_kernel, dim3((unsigned)Q), dim3(kT), 0, s, dists, N, ldd, k,
                           largest ? 0xFFFFFFFFu : 0u, vals, idx);
    }
    return check_launch("bolt_topk_f32");
}
