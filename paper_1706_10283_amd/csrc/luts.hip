// Query encoding g and its uint8 quantisation for gfx950 (Sec. 3.1, the
// matrix D of a query; Sec. 3.2, the learned quantiser beta_m), for every
// per-dimension term of eq. distFuncForm the library serves, and unit rows
// for cosine similarity (Sec. 1.1).
//
// One thread per table entry (query q, table m, entry i).  The 16 threads of
// one table read the same query subvector (a broadcast) and neighbouring
// centroids.  Each entry is accumulated sequentially in ascending dimension
// order with fma, and quantised with a single fma, floor and clamp, so the
// uint8 value is reproducible bit for bit.  The work is Theta(K J) per query
// (Sec. 3.1) and tiny next to the scan.
#include "common.hpp"

namespace {

// Unit-norm scale of row x: |x| with the sum of squares accumulated by fma in
// ascending order and a correctly rounded square root.
__device__ inline float row_norm(const float *__restrict__ x, int J)
{
    float s = 0.0f;
    for (int j = 0; j < J; ++j)
        s = __builtin_fmaf(x[j], x[j], s);
    return __fsqrt_rn(s);
}

__global__ __launch_bounds__(256) void luts_kernel(
    const float *__restrict__ Qv, int64_t Q, int64_t ldq, const float *__restrict__ C, int M,
    int sub, int kind, int p, float a, const float *__restrict__ offsets, float *__restrict__ lf,
    uint8_t *__restrict__ l8)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= Q * M * bolt::kCentroids)
        return;
    const int i = (int)(e & 15);
    const int64_t qm = e >> 4;
    const int64_t q = qm / M;
    const int m = (int)(qm - q * M);
    const float *qv = Qv + q * ldq + (int64_t)m * sub;
    const float *c = C + ((int64_t)m * bolt::kCentroids + i) * sub;
    float acc = 0.0f;
    if (kind == BOLT_METRIC_L2) {
        for (int j = 0; j < sub; ++j) {
            float t = qv[j] - c[j];
            acc = __builtin_fmaf(t, t, acc);
        }
    } else if (kind == BOLT_METRIC_L1 || (kind == 3 && p == 1)) {
        for (int j = 0; j < sub; ++j)
            acc = acc + __builtin_fabsf(qv[j] - c[j]);
    } else if (kind == 3) {
        for (int j = 0; j < sub; ++j) {
            const float t = __builtin_fabsf(qv[j] - c[j]);
            float w = t;
            for (int r = 2; r < p; ++r)
                w = w * t;
            acc = __builtin_fmaf(w, t, acc);
        }
    } else if (kind == BOLT_METRIC_COSINE) {
        // every entry of the query recomputes its norm: J fma per entry, a
        // few microseconds for a thousand queries
        const float n = row_norm(Qv + q * ldq, M * sub);
        for (int j = 0; j < sub; ++j)
            acc = __builtin_fmaf(n > 0.0f ? __fdiv_rn(qv[j], n) : 0.0f, c[j], acc);
    } else {
        for (int j = 0; j < sub; ++j)
            acc = __builtin_fmaf(qv[j], c[j], acc);
    }
    if (lf)
        lf[e] = acc;
    if (l8) {
        float y = __builtin_fmaf(a, acc, -offsets[m]);
        float f = __builtin_floorf(y);
        f = f > 0.0f ? f : 0.0f;
        f = f < 255.0f ? f : 255.0f;
        l8[e] = (uint8_t)f;
    }
}

// One thread per row: the canonical sum of squares is sequential in j.
__global__ __launch_bounds__(256) void normalize_kernel(const float *X, int64_t N, int J, int64_t ldx, float *Y,
                                                        int64_t ldy)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    const float *x = X + r * ldx;
    const float n = row_norm(x, J);
    float *y = Y + r * ldy;
    for (int j = 0; j < J; ++j)
        y[j] = n > 0.0f ? __fdiv_rn(x[j], n) : 0.0f;
}

}  // namespace

extern "C" int bolt_build_luts(const float *Qv, int64_t Q, int32_t J, int64_t ldq,
                               const float *centroids, int32_t M, int32_t metric, float a,
                               const float *offsets, float *luts_f32, uint8_t *luts_u8,
                               void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    BOLT_TRY(check_N(Q, "Q"));
    Metric mt;
    BOLT_TRY(decode_metric(metric, &mt));
    if (ldq < J)
        return fail(BOLT_ERR_INVALID, "ldq (%lld) < J (%d)", (long long)ldq, J);
    if (luts_u8 && !(a > 0.0f))
        return fail(BOLT_ERR_INVALID, "scale a must be positive (got %g)", (double)a);
    if (Q == 0)
        return BOLT_OK;
    if (!Qv || !centroids || (luts_u8 && !offsets))
        return fail(BOLT_ERR_INVALID, "bolt_build_luts: null pointer");
    const int64_t work = Q * M * kCentroids;
    {
        bolt::ProfScope prof_("luts", as_stream(stream));
        hipLaunchKernelGGL(luts_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                           as_stream(stream), Qv, Q, ldq, centroids, M, J / M, mt.kind, mt.p, a, offsets,
                           luts_f32, luts_u8);
    }
    return check_launch("bolt_build_luts");
}

extern "C" int bolt_normalize_rows(const float *X, int64_t N, int32_t J, int64_t ldx, float *Y, int64_t ldy,
                                   void *stream)
{
    using namespace bolt;
    BOLT_TRY(check_N(N, "N"));
    if (J <= 0 || ldx < J || ldy < J)
        return fail(BOLT_ERR_INVALID, "need J > 0, ldx >= J and ldy >= J (J=%d)", J);
    if (N == 0)
        return BOLT_OK;
    if (!X || !Y)
        return fail(BOLT_ERR_INVALID, "bolt_normalize_rows: null pointer");
    if (X != Y && ((Y < X + N * ldx && X < Y + N * ldy)))
        return fail(BOLT_ERR_INVALID, "bolt_normalize_rows: Y overlaps X without being X");
    if (X == Y && ldx != ldy)
        return fail(BOLT_ERR_INVALID, "bolt_normalize_rows: in place needs ldy == ldx");
    {
        bolt::ProfScope prof_("normalize", as_stream(stream));
        hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, as_stream(stream), X,
                           N, J, ldx, Y, ldy);
    }
    return check_launch("bolt_normalize_rows");
}
