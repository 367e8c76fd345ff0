// Codebook learning on the GPU (the offline phase of Sec. 1.2; K = 16
// centroids per subspace, Sec. 3.2): Lloyd's k-means on every subspace.
//
// Iteration t: every (row, subspace) is assigned to its nearest centroid by
// the squared distance in fp64, accumulated in ascending dimension order,
// ties to the lowest index (the same fp64 operations in the same order as
// the definition, so the assignment is reproducible); the total error of
// the assignment is the objective; each centroid becomes the fp64 mean of
// its rows, rounded to fp32, and an empty cluster keeps its centroid.
//
// The means are sums over rows in parallel order: bit-identical to the
// ascending-row definition whenever the sums are exact in fp64 (for example
// integer-valued data), otherwise within the last bit of the fp32 result.
//
// Kernels: assign + accumulate (per-workgroup sums in LDS, one fp64 atomic
// per workgroup and entry), then finalise (means, empty clusters, clearing
// the sums for the next iteration).  All state lives in the caller's
// workspace; the call synchronises its stream once at the end to return the
// objective to the host.
#include "common.hpp"

namespace {

constexpr int kK = bolt::kCentroids;

// Centroid i of subspace m starts at row init_rows[i] of X.
struct InitRows {
    int64_t r[kK];
};

// Initial centroids: one thread per (m, i, j) of the [M][16][sub] layout.
__global__ __launch_bounds__(256) void kmeans_seed_kernel(const float *__restrict__ X, int64_t ldx, int M,
                                                          int sub, InitRows init, float *__restrict__ C)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= M * kK * sub)
        return;
    const int j = e % sub, i = (e / sub) % kK, m = e / (sub * kK);
    C[e] = X[init.r[i] * ldx + (int64_t)m * sub + j];
}

// Assignment of every (row, subspace) and, unless last, the per-cluster sums
// and counts.  LDS: sums [M][16][sub] fp64 and counts [M][16].
__global__ __launch_bounds__(256) void kmeans_assign_kernel(const float *__restrict__ X, int64_t n, int64_t ldx,
                                                            int M, int sub, const float *__restrict__ C,
                                                            int accumulate, double *__restrict__ sums,
                                                            unsigned long long *__restrict__ counts,
                                                            double *__restrict__ objective, int64_t per_block)
{
    extern __shared__ __attribute__((aligned(16))) double lsum[];   // [M * 16 * sub], then counts
    const int J = M * sub;
    unsigned int *lcnt = reinterpret_cast<unsigned int *>(lsum + (int64_t)J * kK);
    __shared__ double wobj[4];
    const int tid = threadIdx.x;
    if (accumulate) {
        for (int e = tid; e < J * kK; e += 256)
            lsum[e] = 0.0;
        for (int e = tid; e < M * kK; e += 256)
            lcnt[e] = 0;
    }
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * per_block;
    const int64_t e1 = (e0 + per_block) < n * M ? (e0 + per_block) : n * M;
    double obj = 0.0;
    for (int64_t e = e0 + tid; e < e1; e += 256) {
        const int64_t r = e / M;
        const int m = (int)(e - r * M);
        const float *x = X + r * ldx + (int64_t)m * sub;
        const float *cm = C + (int64_t)m * kK * sub;
        double best = __builtin_inf();
        int bi = 0;
        for (int i = 0; i < kK; ++i) {
            double s = 0.0;
            for (int j = 0; j < sub; ++j) {
                const double d = (double)x[j] - (double)cm[i * sub + j];
                s = s + d * d;
            }
            if (s < best) {
                best = s;
                bi = i;
            }
        }
        obj += best;
        if (accumulate) {
            for (int j = 0; j < sub; ++j)
                atomicAdd(&lsum[((int64_t)m * kK + bi) * sub + j], (double)x[j]);
            atomicAdd(&lcnt[m * kK + bi], 1u);
        }
    }
    // objective: wave sums, then one atomic per workgroup
    for (int off = 32; off > 0; off >>= 1)
        obj += __shfl_down(obj, off, 64);
    if ((tid & 63) == 0)
        wobj[tid >> 6] = obj;
    __syncthreads();
    if (tid == 0)
        atomicAdd(objective, wobj[0] + wobj[1] + wobj[2] + wobj[3]);
    if (accumulate) {
        for (int e = tid; e < J * kK; e += 256)
            if (lsum[e] != 0.0)
                atomicAdd(&sums[e], lsum[e]);
        for (int e = tid; e < M * kK; e += 256)
            if (lcnt[e])
                atomicAdd(&counts[e], (unsigned long long)lcnt[e]);
    }
}

// Means (fp64, rounded to fp32), empty clusters unchanged; sums and counts
// cleared for the next iteration.
__global__ __launch_bounds__(256) void kmeans_finalize_kernel(int M, int sub, float *__restrict__ C,
                                                              double *__restrict__ sums,
                                                              unsigned long long *__restrict__ counts)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= M * kK * sub)
        return;
    const int mi = e / sub;   // (m, i)
    const unsigned long long c = counts[mi];
    if (c > 0)
        C[e] = (float)(sums[e] / (double)c);
    sums[e] = 0.0;
}

__global__ void kmeans_clear_kernel(unsigned long long *__restrict__ counts, int n_counts,
                                    double *__restrict__ sums, int n_sums, double *__restrict__ obj, int n_obj)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n_counts)
        counts[e] = 0;
    if (e < n_sums)
        sums[e] = 0.0;
    if (e < n_obj)
        obj[e] = 0.0;
}

__global__ void kmeans_clear_counts_kernel(unsigned long long *__restrict__ counts, int n_counts)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n_counts)
        counts[e] = 0;
}

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" size_t bolt_kmeans_ws_bytes(int32_t J, int32_t M, int32_t iters)
{
    if (M <= 0 || J <= 0 || iters < 0)
        return 0;
    return a256((size_t)J * kK * sizeof(double)) + a256((size_t)M * kK * sizeof(unsigned long long)) +
           a256((size_t)(iters + 1) * sizeof(double));
}

extern "C" int bolt_kmeans(const float *X, int64_t n, int32_t J, int64_t ldx, int32_t M, int32_t iters,
                           const int64_t *init_rows, float *centroids, double *objective, void *ws,
                           size_t ws_bytes, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    BOLT_TRY(check_N(n, "n"));
    if (ldx < J)
        return fail(BOLT_ERR_INVALID, "ldx (%lld) < J (%d)", (long long)ldx, J);
    if (iters < 0 || iters > 10000)
        return fail(BOLT_ERR_INVALID, "iters must be in [0, 10000] (got %d)", iters);
    if (n < kK)
        return fail(BOLT_ERR_SHAPE, "k-means needs at least %d rows (got %lld)", kK, (long long)n);
    if (!X || !init_rows || !centroids)
        return fail(BOLT_ERR_INVALID, "bolt_kmeans: null pointer");
    InitRows init;
    for (int i = 0; i < kK; ++i) {
        if (init_rows[i] < 0 || init_rows[i] >= n)
            return fail(BOLT_ERR_INVALID, "init_rows[%d] = %lld outside [0, %lld)", i, (long long)init_rows[i],
                        (long long)n);
        init.r[i] = init_rows[i];
    }
    const size_t need = bolt_kmeans_ws_bytes(J, M, iters);
    if (ws_bytes < need || !ws || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "k-means needs a 256-byte aligned workspace of %zu bytes", need);
    const int sub = J / M;
    const size_t lds = (size_t)J * kK * sizeof(double) + (size_t)M * kK * sizeof(unsigned int);
    if (lds > 150 * 1024)
        return fail(BOLT_ERR_UNSUPPORTED, "k-means keeps J * 16 fp64 sums in LDS: J = %d is too large", J);
    char *w = reinterpret_cast<char *>(ws);
    double *sums = reinterpret_cast<double *>(w);
    unsigned long long *counts = reinterpret_cast<unsigned long long *>(w + a256((size_t)J * kK * sizeof(double)));
    double *obj = reinterpret_cast<double *>(w + a256((size_t)J * kK * sizeof(double)) +
                                             a256((size_t)M * kK * sizeof(unsigned long long)));
    hipStream_t s = as_stream(stream);
    const int n_c = M * kK, n_s = J * kK;
    const int big = n_s > n_c ? (n_s > iters + 1 ? n_s : iters + 1) : (n_c > iters + 1 ? n_c : iters + 1);
    hipLaunchKernelGGL(kmeans_clear_kernel, dim3((big + 255) / 256), dim3(256), 0, s, counts, n_c, sums, n_s, obj,
                       iters + 1);
    hipLaunchKernelGGL(kmeans_seed_kernel, dim3((n_s + 255) / 256), dim3(256), 0, s, X, ldx, M, sub, init,
                       centroids);
    // about 1024 workgroups over the n * M (row, subspace) pairs
    const int64_t pairs = n * M;
    int64_t per_block = (pairs + 1023) / 1024;
    per_block = per_block < 1024 ? 1024 : per_block;
    const unsigned blocks = (unsigned)((pairs + per_block - 1) / per_block);
    {
        bolt::ProfScope prof_("kmeans", s);
        for (int t = 0; t <= iters; ++t) {
            const int acc = t < iters;
            hipLaunchKernelGGL(kmeans_assign_kernel, dim3(blocks), dim3(256), acc ? lds : 0, s, X, n, ldx, M, sub,
                               centroids, acc, sums, counts, obj + t, per_block);
            if (acc) {
                hipLaunchKernelGGL(kmeans_finalize_kernel, dim3((n_s + 255) / 256), dim3(256), 0, s, M, sub,
                                   centroids, sums, counts);
                hipLaunchKernelGGL(kmeans_clear_counts_kernel, dim3((n_c + 255) / 256), dim3(256), 0, s, counts,
                                   n_c);
            }
        }
    }
    BOLT_TRY(check_launch("bolt_kmeans"));
    if (objective) {
        if (hipMemcpyAsync(objective, obj, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost, s) != hipSuccess)
            return check_launch("bolt_kmeans (objective copy)");
    }
    if (hipStreamSynchronize(s) != hipSuccess)
        return check_launch("bolt_kmeans (synchronise)");
    return BOLT_OK;
}
