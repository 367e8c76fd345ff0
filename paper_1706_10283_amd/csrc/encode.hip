// Data encoding h for gfx950: for every row and subspace, the index of the
// nearest of 16 centroids in squared Euclidean distance (Sec. 3.1, the
// encoding function h; K = 16 per Sec. 3.2).
//
// Design: a workgroup of 4 waves owns a tile of 64 rows.  The tile is staged
// in LDS with coalesced 16-byte loads (row stride padded to 4 mod 64 dwords,
// so that 64 lanes reading the same column of 64 different rows hit distinct
// banks).  Each lane then owns one row; each wave walks a disjoint set of
// subspaces, so the subspace index is wave-uniform and the centroids are read
// through the scalar cache as SGPR operands of the VALU instructions.  The
// distance is the direct form (x - c)^2 accumulated with fma in ascending
// dimension order, the same order the definition fixes, so the fp32 argmin
// (ties to the lowest index) is reproducible; the expanded form
// |x|^2 - 2 x.c + |c|^2 would cancel badly.  Codes are gathered per row in
// LDS (M bytes per row, dynamic) and written back as packed bytes with
// coalesced dword stores.  Rows are staged 32 dimensions at a time (64 for
// subspaces wider than 8), and the next chunk's loads are issued into
// registers before the current chunk is computed, so a workgroup waits for
// HBM once (its first chunk) instead of once per chunk; it holds about 11 KB
// of LDS (J = 128, M = 32) and eight workgroups per CU keep the VALU busy.
#include "common.hpp"

namespace {

constexpr int kRows = 64;                 // rows per tile = lanes per wave
constexpr int kWaves = 4;
constexpr int kThreads = kRows * kWaves;

// Dimensions staged per pass: 32 (9 KB of rows) while that holds at least
// four subspaces, one per wave; 64 for wider subspaces.
template <int SUB>
constexpr int chunk_dims() { return SUB <= 8 ? 32 : 64; }

template <int SUB>
__device__ __forceinline__ int nearest(const float *x, const float *__restrict__ c)
{
    float best = __builtin_inff();
    int bi = 0;
#pragma unroll
    for (int i = 0; i < bolt::kCentroids; ++i) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < SUB; ++j) {
            float t = x[j] - c[i * SUB + j];
            acc = __builtin_fmaf(t, t, acc);
        }
        if (acc < best) {
            best = acc;
            bi = i;
        }
    }
    return bi;
}

// Pack the per-row nibbles gathered in LDS (cs[row][m], one byte each) and
// store rows [n0, n0+rows) of the code matrix.
__device__ __forceinline__ void store_codes(const uint8_t *cs, int cs_stride, int rows, int M,
                                            uint8_t *__restrict__ dst, int byte_store)
{
    const int bpr = M >> 1;
    const int tile_bytes = rows * bpr;
    // bytes per row a power of two (every M the kernels are tuned for): a
    // shift and a mask instead of a division per byte
    const bool pow2 = (bpr & (bpr - 1)) == 0;
    const int sh = pow2 ? __builtin_ctz((unsigned)bpr) : 0;
    if (!byte_store) {
        for (int e = threadIdx.x; 4 * e < tile_bytes; e += kThreads) {
            uint32_t w = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                int byte = 4 * e + b;
                if (byte < tile_bytes) {
                    const int r = pow2 ? byte >> sh : byte / bpr;
                    const int t = byte - r * bpr;
                    uint32_t v = cs[r * cs_stride + 2 * t] | (cs[r * cs_stride + 2 * t + 1] << 4);
                    w |= v << (8 * b);
                }
            }
            if (4 * e + 3 < tile_bytes) {
                *reinterpret_cast<uint32_t *>(dst + 4 * e) = w;
            } else {
                for (int b = 0; b < 4 && 4 * e + b < tile_bytes; ++b)
                    dst[4 * e + b] = (uint8_t)(w >> (8 * b));
            }
        }
    } else {
        for (int byte = threadIdx.x; byte < tile_bytes; byte += kThreads) {
            int r = byte / bpr, t = byte - r * bpr;
            dst[byte] = (uint8_t)(cs[r * cs_stride + 2 * t] | (cs[r * cs_stride + 2 * t + 1] << 4));
        }
    }
}

// SUB = J / M, the subspace width.  G consecutive subspaces are handled per
// lane step so that every LDS read is a full 16 bytes.
template <int SUB>
__global__ __launch_bounds__(kThreads) void encode_lds_kernel(
    const float *__restrict__ X, int64_t N, int64_t ldx, const float *__restrict__ C, int M,
    uint8_t *__restrict__ codes, int vec4, int byte_store)
{
    constexpr int G = SUB >= 4 ? 1 : 4 / SUB;
    constexpr int kChunkDims = chunk_dims<SUB>();
    constexpr int kStride = kChunkDims + 4;   // LDS row stride in floats (4 mod 64 banks)
    constexpr int kChunkM = kChunkDims / SUB;
    static_assert(kChunkM >= 1 && kChunkM % G == 0, "chunk must hold whole lane steps");
    __shared__ __attribute__((aligned(16))) float xs[kRows * kStride];
    extern __shared__ uint8_t cs[];   // [kRows][M]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n0 = (int64_t)blockIdx.x * kRows;
    const int rows = (int)((N - n0) < kRows ? (N - n0) : kRows);

    constexpr int d4 = kChunkDims / 4;
    constexpr int PF = kRows * d4 / kThreads;   // float4 per thread of a full chunk
    float4 pf[PF];
    bool have_pf = false;
    // the float4 loads of a full chunk into registers (rows clamped: unconditional)
    auto prefetch = [&](int64_t jj) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            const int e = tid + p * kThreads;
            const int r0 = e / d4, c4 = e % d4;
            const int r = r0 < rows ? r0 : rows - 1;
            pf[p] = __builtin_bit_cast(float4, __builtin_nontemporal_load(
                reinterpret_cast<const float __attribute__((ext_vector_type(4))) *>(X + (n0 + r) * ldx + jj + 4 * c4)));
        }
    };
    for (int m0 = 0; m0 < M; m0 += kChunkM) {
        const int mc = (M - m0) < kChunkM ? (M - m0) : kChunkM;
        const int dims = mc * SUB;
        const int64_t j0 = (int64_t)m0 * SUB;
        if (m0)
            __syncthreads();
        if (vec4 && dims == kChunkDims) {   // a full chunk: d4 float4 per row, no division
            if (!have_pf)
                prefetch(j0);
#pragma unroll
            for (int p = 0; p < PF; ++p) {
                const int e = tid + p * kThreads;
                const int r = e / d4, c4 = e % d4;
                if (r < rows)
                    *reinterpret_cast<float4 *>(&xs[r * kStride + 4 * c4]) = pf[p];
            }
            // the next full chunk's loads fly while this one is computed
            const int mn = m0 + kChunkM;
            have_pf = mn < M && (M - mn) * SUB >= kChunkDims;
            if (have_pf)
                prefetch((int64_t)mn * SUB);
        } else if (vec4) {
            const int dq = dims >> 2;
            for (int e = tid; e < rows * dq; e += kThreads) {
                int r = e / dq, c4 = e - r * dq;
                // streamed once: non-temporal loads (about 4% faster here)
                float4 v = __builtin_bit_cast(float4, __builtin_nontemporal_load(
                    reinterpret_cast<const float __attribute__((ext_vector_type(4))) *>(X + (n0 + r) * ldx + j0 + 4 * c4)));
                *reinterpret_cast<float4 *>(&xs[r * kStride + 4 * c4]) = v;
            }
        } else {
            for (int e = tid; e < rows * dims; e += kThreads) {
                int r = e / dims, c = e - r * dims;
                xs[r * kStride + c] = X[(n0 + r) * ldx + j0 + c];
            }
        }
        __syncthreads();
        const int steps = (mc + G - 1) / G;
        for (int s = wave; s < steps; s += kWaves) {
            float x[G * SUB];
            const float4 *xr = reinterpret_cast<const float4 *>(&xs[lane * kStride + s * G * SUB]);
#pragma unroll
            for (int v = 0; v < G * SUB / 4; ++v) {
                float4 t = xr[v];
                x[4 * v + 0] = t.x;
                x[4 * v + 1] = t.y;
                x[4 * v + 2] = t.z;
                x[4 * v + 3] = t.w;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int m = m0 + s * G + g;
                if (m < M) {
                    const float *cm = C + (int64_t)m * bolt::kCentroids * SUB;
                    cs[lane * M + m] = (uint8_t)nearest<SUB>(x + g * SUB, cm);
                }
            }
        }
    }
    __syncthreads();
    store_codes(cs, M, rows, M, codes + n0 * (M >> 1), byte_store);
}

// Any subspace width: one thread per (row, subspace pair), reading X and the
// centroids straight from global memory.  Used for widths without a tuned
// kernel (odd widths, or wider than the LDS tile).
__global__ __launch_bounds__(256) void encode_generic_kernel(
    const float *__restrict__ X, int64_t N, int64_t ldx, const float *__restrict__ C, int M,
    int sub, uint8_t *__restrict__ codes)
{
    const int bpr = M >> 1;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * bpr)
        return;
    const int64_t n = e / bpr;
    const int t = (int)(e - n * bpr);
    uint32_t byte = 0;
    for (int h = 0; h < 2; ++h) {
        const int m = 2 * t + h;
        const float *x = X + n * ldx + (int64_t)m * sub;
        float best = __builtin_inff();
        int bi = 0;
        for (int i = 0; i < bolt::kCentroids; ++i) {
            const float *c = C + ((int64_t)m * bolt::kCentroids + i) * sub;
            float acc = 0.0f;
            for (int j = 0; j < sub; ++j) {
                float d = x[j] - c[j];
                acc = __builtin_fmaf(d, d, acc);
            }
            if (acc < best) {
                best = acc;
                bi = i;
            }
        }
        byte |= (uint32_t)bi << (4 * h);
    }
    codes[e] = (uint8_t)byte;
}

template <int SUB>
void launch_lds(const float *X, int64_t N, int64_t ldx, const float *C, int M, uint8_t *codes,
                int vec4, int byte_store, hipStream_t s)
{
    dim3 grid((unsigned)((N + kRows - 1) / kRows));
    {
        bolt::ProfScope prof_("encode", s);
        hipLaunchKernelGGL(encode_lds_kernel<SUB>, grid, dim3(kThreads), (size_t)kRows * M, s, X, N, ldx, C, M,
                           codes, vec4, byte_store);
    }
}

}  // namespace

extern "C" int bolt_encode(const float *X, int64_t N, int32_t J, int64_t ldx,
                           const float *centroids, int32_t M, uint8_t *codes, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    BOLT_TRY(check_N(N, "N"));
    if (ldx < J)
        return fail(BOLT_ERR_INVALID, "ldx (%lld) < J (%d)", (long long)ldx, J);
    if (N == 0)
        return BOLT_OK;
    if (!X || !centroids || !codes)
        return fail(BOLT_ERR_INVALID, "bolt_encode: null pointer");
    hipStream_t s = as_stream(stream);
    const int sub = J / M;
    const int vec4 = (J % 4 == 0) && (ldx % 4 == 0) && aligned(X, 16);
    const int byte_store = !aligned(codes, 4);
    switch (sub) {
    case 1: launch_lds<1>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    case 2: launch_lds<2>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    case 4: launch_lds<4>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    case 8: launch_lds<8>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    case 16: launch_lds<16>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    case 32: launch_lds<32>(X, N, ldx, centroids, M, codes, vec4, byte_store, s); break;
    default: {
        const int64_t work = N * (M / 2);
        {
            bolt::ProfScope prof_("encode", s);
            hipLaunchKernelGGL(encode_generic_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                               s, X, N, ldx, centroids, M, sub, codes);
        }
    }
    }
    return check_launch("bolt_encode");
}
