// Learning the uint8 quantiser on the GPU (Sec. 3.2): the shared scale a and
// the per-table offsets b_m, chosen over a grid of tail fractions alpha.
//
// The distribution of table m is the multiset of D_m[h(x)_m](q) over pairs
// (training query q, training vector x): for a fixed q it depends on x only
// through the code, so it is the value D_m[i](q) weighted by the number of
// training vectors whose code in subspace m is i.  For each alpha:
//   b_m   = the alpha-quantile of table m's multiset
//   a     = 255 / the (1 - alpha)-quantile of y - b_m pooled over all tables
//           (a = 1 if that quantile is not positive)
//   b'_m  = fp32(a32 * b_m), a32 = fp32(a)
//   loss  = weighted mean of (y_hat - y)^2, y_hat = (clamp(floor(a32 y - b'_m),
//           0, 255) + b'_m) / a32
// and the alpha with the smallest loss wins, ties to the smaller alpha.
// Quantiles interpolate linearly between order statistics (position
// (total - 1) p of the sorted multiset).
//
// Kernels: (1) the fp64 tables of the training queries, one thread per
// entry, in the definition's order; (2) the code counts per subspace;
// (3) per table a bitonic sort of its entries in LDS (up to 16384, i.e.
// 1024 training queries) and the running sum of their weights; (4) one
// workgroup per alpha: b_m by binary search over the running sums, the
// pooled quantile by bisection over the ordered fp64 bit patterns (the
// number of pooled values at or below v is a sum over tables of one binary
// search each, with y - b_m rounded exactly as the definition rounds it),
// then a, b' and the loss.  Every value that decides a or b' uses the
// definition's fp64 operations in its order, so for the chosen alpha they
// are bit-identical to a sequential implementation; the losses are summed
// in parallel order (within the last bits of a sequential sum).
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace {

constexpr int kK = bolt::kCentroids;
constexpr int kMaxAlphas = 64;
constexpr int kSortThreads = 1024;
constexpr int kMaxSort = 16384;   // entries per table sorted in LDS: 1024 training queries

struct Alphas {
    double v[kMaxAlphas];
};

inline size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// Entries per table, padded to a power of two for the bitonic sort, at
// least one per sorting thread.
int64_t sort_size(int64_t nq)
{
    int64_t s = kSortThreads;
    while (s < nq * kK)
        s *= 2;
    return s;
}

__device__ inline uint64_t order_key(double d)
{
    const uint64_t u = (uint64_t)__double_as_longlong(d);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double key_value(uint64_t k)
{
    const uint64_t u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)u);
}

// (1) fp64 table entry of training query q, table m, centroid i (padding: +inf).
__global__ __launch_bounds__(256) void qtab_kernel(const float *__restrict__ Qt, int64_t nq, int64_t ldq,
                                                   const float *__restrict__ C, int M, int sub, int kind, int p,
                                                   int64_t S, double *__restrict__ tab, uint8_t *__restrict__ pay)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)M * S)
        return;
    const int m = (int)(e / S);
    const int64_t r = e - (int64_t)m * S;
    if (r >= nq * kK) {
        tab[e] = __builtin_inf();
        pay[e] = 0;
        return;
    }
    const int64_t q = r / kK;
    const int i = (int)(r % kK);
    const float *qv = Qt + q * ldq;
    const float *c = C + ((int64_t)m * kK + i) * sub;
    double qn = 0.0;
    if (kind == BOLT_METRIC_COSINE) {
        for (int j = 0; j < M * sub; ++j)
            qn += (double)qv[j] * (double)qv[j];
        qn = sqrt(qn);
    }
    double s = 0.0;
    for (int j = 0; j < sub; ++j) {
        const double x = (double)qv[(int64_t)m * sub + j], y = (double)c[j];
        switch (kind) {
        case BOLT_METRIC_L2: {
            const double t = x - y;
            s += t * t;
            break;
        }
        case BOLT_METRIC_L1: s += fabs(x - y); break;
        case 3: {   // |x - y|^p by repeated products
            const double t = fabs(x - y);
            double w = t;
            for (int e2 = 1; e2 < p; ++e2)
                w = w * t;
            s += w;
            break;
        }
        case BOLT_METRIC_COSINE: s += (qn > 0.0 ? x / qn : 0.0) * y; break;
        default: s += x * y;
        }
    }
    tab[e] = s;
    pay[e] = (uint8_t)i;
}

// (2) counts[m][i]: training rows whose code in subspace m is i.
__global__ __launch_bounds__(256) void code_count_kernel(const uint8_t *__restrict__ codes, int64_t n, int M,
                                                         unsigned long long *__restrict__ counts)
{
    extern __shared__ unsigned int lcnt[];   // [M][16]
    for (int e = threadIdx.x; e < M * kK; e += 256)
        lcnt[e] = 0;
    __syncthreads();
    const int half = M / 2;
    const int64_t total = n * half;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int t = (int)(e % half);
        const uint8_t b = codes[e];
        atomicAdd(&lcnt[(2 * t) * kK + (b & 15)], 1u);
        atomicAdd(&lcnt[(2 * t + 1) * kK + (b >> 4)], 1u);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M * kK; e += 256)
        if (lcnt[e])
            atomicAdd(&counts[e], (unsigned long long)lcnt[e]);
}

// (3) sort table m's entries ascending (with their centroid index) and write
// the running sum of their weights.
__global__ __launch_bounds__(kSortThreads) void table_sort_kernel(double *__restrict__ tab, uint8_t *__restrict__ pay,
                                                                  int64_t *__restrict__ cum, int64_t S, int64_t used,
                                                                  const unsigned long long *__restrict__ counts)
{
    extern __shared__ __attribute__((aligned(16))) uint64_t keys[];   // [S], then payload [S]
    uint8_t *lpay = reinterpret_cast<uint8_t *>(keys + S);
    const int m = blockIdx.x;
    const int tid = threadIdx.x;
    double *t = tab + (int64_t)m * S;
    uint8_t *pm = pay + (int64_t)m * S;
    for (int64_t r = tid; r < S; r += kSortThreads) {
        keys[r] = order_key(t[r]);
        lpay[r] = pm[r];
    }
    __syncthreads();
    for (int64_t k = 2; k <= S; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t x = tid; x < S / 2; x += kSortThreads) {
                const int64_t i = (x / j) * 2 * j + (x % j);
                const int64_t l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t a = keys[i], b = keys[l];
                if ((a > b) == up) {
                    keys[i] = b;
                    keys[l] = a;
                    const uint8_t pa = lpay[i];
                    lpay[i] = lpay[l];
                    lpay[l] = pa;
                }
            }
            __syncthreads();
        }
    // running weights: each thread sums a contiguous run, then a scan of the runs
    const int64_t per = S / kSortThreads;
    const unsigned long long *cm = counts + (int64_t)m * kK;
    int64_t local = 0;
    for (int64_t r = tid * per; r < (tid + 1) * per; ++r)
        local += r < used ? (int64_t)cm[lpay[r]] : 0;
    __shared__ int64_t run[kSortThreads];
    run[tid] = local;
    __syncthreads();
    for (int off = 1; off < kSortThreads; off <<= 1) {
        const int64_t v = tid >= off ? run[tid - off] : 0;
        __syncthreads();
        run[tid] += v;
        __syncthreads();
    }
    int64_t acc = run[tid] - local;
    for (int64_t r = tid * per; r < (tid + 1) * per; ++r) {
        acc += r < used ? (int64_t)cm[lpay[r]] : 0;
        cum[(int64_t)m * S + r] = acc;
        t[r] = key_value(keys[r]);
        pm[r] = lpay[r];
    }
}

// The value at 0-based position pos of table m's expanded multiset.
__device__ inline double table_at(const double *t, const int64_t *cum, int64_t used, int64_t pos)
{
    int64_t lo = 0, hi = used - 1;   // smallest r with cum[r] > pos
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (cum[mid] > pos)
            hi = mid;
        else
            lo = mid + 1;
    }
    return t[lo];
}

// Number of pooled values y - b at or below v in one table (y - b rounded
// once, as the definition computes it; monotone in y).
__device__ inline int64_t table_count_le(const double *t, const int64_t *cum, int64_t used, double b, double v)
{
    int64_t lo = 0, hi = used;   // first r with t[r] - b > v
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (t[mid] - b > v)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo > 0 ? cum[lo - 1] : 0;
}

__device__ int64_t block_sum_i64(int64_t v, int64_t *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            red[tid] += red[tid + off];
        __syncthreads();
    }
    const int64_t r = red[0];
    __syncthreads();
    return r;
}

// The pooled value at position pos: the first ordered key whose count of
// pooled values at or below it exceeds pos.
__device__ double pool_at(const double *tab, const int64_t *cum, int64_t S, int64_t used, int M, const double *b,
                          int64_t pos, uint64_t klo, uint64_t khi, int64_t *red)
{
    const int tid = threadIdx.x;
    while (klo < khi) {
        const uint64_t mid = klo + (khi - klo) / 2;
        const double v = key_value(mid);
        int64_t c = 0;
        for (int m = tid; m < M; m += 256)
            c += table_count_le(tab + (int64_t)m * S, cum + (int64_t)m * S, used, b[m], v);
        if (block_sum_i64(c, red) > pos)
            khi = mid;
        else
            klo = mid + 1;
    }
    return key_value(khi);
}

// (4) one workgroup per alpha: b_m, a, b'_m and the loss.
__global__ __launch_bounds__(256) void alpha_kernel(const double *__restrict__ tab, const uint8_t *__restrict__ pay,
                                                    const int64_t *__restrict__ cum, int64_t S, int64_t used,
                                                    int M, int64_t n_train, int64_t nq,
                                                    const unsigned long long *__restrict__ counts, Alphas alphas,
                                                    float *__restrict__ a_out, float *__restrict__ boff_out,
                                                    double *__restrict__ loss_out)
{
    __shared__ double b[256];
    __shared__ float boff[256];
    __shared__ int64_t red[256];
    __shared__ double dred[256];
    __shared__ double lo_hi[2];
    const int tid = threadIdx.x;
    const double alpha = alphas.v[blockIdx.x];
    const int64_t total = nq * n_train;   // multiset size of one table
    for (int m = tid; m < M; m += 256) {
        const double *t = tab + (int64_t)m * S;
        const int64_t *c = cum + (int64_t)m * S;
        const double h = (double)(total - 1) * alpha;
        const int64_t lo = (int64_t)floor(h);
        const double frac = h - (double)lo;
        const double vlo = table_at(t, c, used, lo);
        b[m] = lo + 1 >= total ? vlo : vlo + frac * (table_at(t, c, used, lo + 1) - vlo);
    }
    __syncthreads();
    // pooled (1 - alpha)-quantile of y - b_m over all tables
    if (tid == 0) {
        double vmin = __builtin_inf(), vmax = -__builtin_inf();
        for (int m = 0; m < M; ++m) {
            const double *t = tab + (int64_t)m * S;
            const double x0 = t[0] - b[m], x1 = t[used - 1] - b[m];
            vmin = x0 < vmin ? x0 : vmin;
            vmax = x1 > vmax ? x1 : vmax;
        }
        lo_hi[0] = vmin;
        lo_hi[1] = vmax;
    }
    __syncthreads();
    const uint64_t klo = order_key(lo_hi[0]), khi = order_key(lo_hi[1]);
    const int64_t ptotal = total * M;
    const double h = (double)(ptotal - 1) * (1.0 - alpha);
    const int64_t lo = (int64_t)floor(h);
    const double frac = h - (double)lo;
    const double vlo = pool_at(tab, cum, S, used, M, b, lo, klo, khi, red);
    double top = vlo;
    if (lo + 1 < ptotal)
        top = vlo + frac * (pool_at(tab, cum, S, used, M, b, lo + 1, klo, khi, red) - vlo);
    const double a = top > 0.0 ? 255.0 / top : 1.0;
    const float a32 = (float)a;
    for (int m = tid; m < M; m += 256)
        boff[m] = (float)((double)a32 * b[m]);
    __syncthreads();
    // weighted squared reconstruction error over every (table, entry)
    double se = 0.0;
    for (int64_t e = tid; e < (int64_t)M * used; e += 256) {
        const int m = (int)(e / used);
        const int64_t r = e - (int64_t)m * used;
        const double v = tab[(int64_t)m * S + r];
        const double w = (double)counts[(int64_t)m * kK + pay[(int64_t)m * S + r]];
        double t = floor((double)a32 * v - (double)boff[m]);
        t = t < 0.0 ? 0.0 : (t > 255.0 ? 255.0 : t);
        const double yh = (t + (double)boff[m]) / (double)a32;
        se += w * (yh - v) * (yh - v);
    }
    dred[tid] = se;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            dred[tid] += dred[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        const double wsum = (double)ptotal;
        loss_out[blockIdx.x] = wsum > 0.0 ? dred[0] / wsum : 0.0;
        a_out[blockIdx.x] = a32;
    }
    for (int m = tid; m < M; m += 256)
        boff_out[(int64_t)blockIdx.x * M + m] = boff[m];
}

struct QuantWs {
    double *tab;
    int64_t *cum;
    uint8_t *pay;
    unsigned long long *counts;
    float *a;
    float *boff;
    double *loss;
};

size_t quant_layout(int64_t nq, int M, int nalpha, char *base, QuantWs *w)
{
    const int64_t S = sort_size(nq);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += a256(bytes);
        return p;
    };
    QuantWs l;
    l.tab = reinterpret_cast<double *>(take((size_t)M * S * sizeof(double)));
    l.cum = reinterpret_cast<int64_t *>(take((size_t)M * S * sizeof(int64_t)));
    l.pay = reinterpret_cast<uint8_t *>(take((size_t)M * S));
    l.counts = reinterpret_cast<unsigned long long *>(take((size_t)M * kK * sizeof(unsigned long long)));
    l.a = reinterpret_cast<float *>(take((size_t)nalpha * sizeof(float)));
    l.boff = reinterpret_cast<float *>(take((size_t)nalpha * M * sizeof(float)));
    l.loss = reinterpret_cast<double *>(take((size_t)nalpha * sizeof(double)));
    if (w)
        *w = l;
    return off;
}

__global__ void clear_u64_kernel(unsigned long long *p, int n)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n)
        p[e] = 0;
}

}  // namespace

extern "C" size_t bolt_learn_quantizer_ws_bytes(int64_t nq, int32_t M, int32_t nalpha)
{
    if (nq < 1 || nq * kK > kMaxSort || M < 2 || M > 256 || nalpha < 1 || nalpha > kMaxAlphas)
        return 0;
    return quant_layout(nq, M, nalpha, nullptr, nullptr);
}

extern "C" int bolt_learn_quantizer(const float *Qt, int64_t nq, int32_t J, int64_t ldq, const uint8_t *codes,
                                    int64_t n, const float *centroids, int32_t M, int32_t metric,
                                    const double *alphas, int32_t nalpha, float *a, float *offsets,
                                    int32_t *alpha_idx, double *losses, void *ws, size_t ws_bytes, void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    BOLT_TRY(check_N(n, "n"));
    Metric mt;
    BOLT_TRY(decode_metric(metric, &mt));
    if (nq < 1 || n < 1 || ldq < J)
        return fail(BOLT_ERR_INVALID, "need nq >= 1, n >= 1 and ldq >= J");
    if (nq * kK > kMaxSort)
        return fail(BOLT_ERR_UNSUPPORTED, "at most %d training queries (got %lld)", kMaxSort / kK, (long long)nq);
    if (nalpha < 1 || nalpha > kMaxAlphas)
        return fail(BOLT_ERR_INVALID, "need 1 <= nalpha <= %d", kMaxAlphas);
    if (!Qt || !codes || !centroids || !alphas || !a || !offsets)
        return fail(BOLT_ERR_INVALID, "bolt_learn_quantizer: null pointer");
    Alphas al;
    std::memset(&al, 0, sizeof(al));
    for (int i = 0; i < nalpha; ++i) {
        if (!(alphas[i] >= 0.0 && alphas[i] < 0.5))
            return fail(BOLT_ERR_INVALID, "alpha must be in [0, 0.5)");
        al.v[i] = alphas[i];
    }
    const size_t need = quant_layout(nq, M, nalpha, nullptr, nullptr);
    if (ws_bytes < need || !ws || !aligned(ws, 256))
        return fail(BOLT_ERR_NOMEM, "the quantiser search needs a 256-byte aligned workspace of %zu bytes", need);
    QuantWs w;
    quant_layout(nq, M, nalpha, reinterpret_cast<char *>(ws), &w);
    const int64_t S = sort_size(nq), used = nq * kK;
    hipStream_t s = as_stream(stream);
    {
        bolt::ProfScope prof_("quantizer", s);
        hipLaunchKernelGGL(clear_u64_kernel, dim3((M * kK + 255) / 256), dim3(256), 0, s, w.counts, M * kK);
        hipLaunchKernelGGL(qtab_kernel, dim3((unsigned)((M * S + 255) / 256)), dim3(256), 0, s, Qt, nq, ldq,
                           centroids, M, J / M, mt.kind, mt.p, S, w.tab, w.pay);
        const int64_t cells = n * (M / 2);
        int64_t blocks = (cells + 255) / 256;
        blocks = blocks > 1024 ? 1024 : blocks;
        hipLaunchKernelGGL(code_count_kernel, dim3((unsigned)blocks), dim3(256), M * kK * sizeof(unsigned int), s,
                           codes, n, M, w.counts);
        hipLaunchKernelGGL(table_sort_kernel, dim3((unsigned)M), dim3(kSortThreads),
                           (size_t)S * (sizeof(uint64_t) + 1), s, w.tab, w.pay, w.cum, S, used, w.counts);
        hipLaunchKernelGGL(alpha_kernel, dim3((unsigned)nalpha), dim3(256), 0, s, w.tab, w.pay, w.cum, S, used, M,
                           n, nq, w.counts, al, w.a, w.boff, w.loss);
    }
    BOLT_TRY(check_launch("bolt_learn_quantizer"));
    std::vector<double> loss(nalpha);
    std::vector<float> av(nalpha);
    if (hipMemcpyAsync(loss.data(), w.loss, sizeof(double) * nalpha, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(av.data(), w.a, sizeof(float) * nalpha, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return check_launch("bolt_learn_quantizer (results)");
    int best = 0;
    for (int i = 1; i < nalpha; ++i)
        if (loss[i] < loss[best])
            best = i;
    if (hipMemcpyAsync(offsets, w.boff + (int64_t)best * M, sizeof(float) * M, hipMemcpyDeviceToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return check_launch("bolt_learn_quantizer (offsets)");
    *a = av[best];
    if (alpha_idx)
        *alpha_idx = best;
    if (losses)
        std::memcpy(losses, loss.data(), sizeof(double) * nalpha);
    return BOLT_OK;
}
