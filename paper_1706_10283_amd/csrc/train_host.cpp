// Offline phase on the host (Sec. 1.2: codebooks and the query quantiser are
// learned before the online phase).  Codebooks are k-means with K = 16 per
// subspace (Sec. 3.1, Sec. 3.2); the quantiser is the alpha grid search of
// Sec. 3.2.  Subspaces are independent, so they are spread over host threads.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.hpp"

namespace {

constexpr int K = bolt::kCentroids;

int n_threads(int work)
{
    unsigned hw = std::thread::hardware_concurrency();
    int t = hw ? (int)hw : 4;
    if (t > 16)
        t = 16;
    return std::max(1, std::min(t, work));
}

template <class F>
void parallel_for(int count, F f)
{
    const int nt = n_threads(count);
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int i = t; i < count; i += nt)
                f(i);
        });
    for (auto &th : pool)
        th.join();
}

// Lloyd's algorithm on subspace m.  Assignment in double precision with ties
// to the lowest index; update = mean of the members in ascending row order;
// a cluster left empty keeps its previous centroid.
void kmeans_subspace(const float *X, int64_t n, int64_t ldx, int sub, int m, int iters,
                     const int64_t *init_rows, float *Cm)
{
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < sub; ++j)
            Cm[i * sub + j] = X[init_rows[i] * ldx + (int64_t)m * sub + j];
    std::vector<int> owner(n > 0 ? n : 1);
    std::vector<double> acc((size_t)K * sub);
    std::vector<int64_t> members(K);
    std::vector<double> c64((size_t)K * sub);
    for (int it = 0; it < iters; ++it) {
        for (int e = 0; e < K * sub; ++e)
            c64[e] = Cm[e];
        for (int64_t r = 0; r < n; ++r) {
            const float *x = X + r * ldx + (int64_t)m * sub;
            int best = 0;
            double bestd = INFINITY;
            for (int i = 0; i < K; ++i) {
                double s = 0.0;
                for (int j = 0; j < sub; ++j) {
                    double t = (double)x[j] - c64[i * sub + j];
                    s += t * t;
                }
                if (s < bestd) {
                    bestd = s;
                    best = i;
                }
            }
            owner[r] = best;
        }
        std::fill(acc.begin(), acc.end(), 0.0);
        std::fill(members.begin(), members.end(), 0);
        for (int64_t r = 0; r < n; ++r) {
            const float *x = X + r * ldx + (int64_t)m * sub;
            const int o = owner[r];
            members[o] += 1;
            for (int j = 0; j < sub; ++j)
                acc[o * sub + j] += (double)x[j];
        }
        for (int i = 0; i < K; ++i)
            if (members[i])
                for (int j = 0; j < sub; ++j)
                    Cm[i * sub + j] = (float)(acc[i * sub + j] / (double)members[i]);
    }
}

struct Weighted {
    double value;
    int64_t count;
};

// Quantile by linear interpolation between order statistics (numpy's
// default) of the multiset in which `value` appears `count` times; `s` is
// sorted by value and `prefix[e]` is the number of elements before s[e].
struct WeightedSample {
    std::vector<Weighted> s;
    std::vector<int64_t> prefix;
    int64_t total = 0;

    void finish()
    {
        std::sort(s.begin(), s.end(), [](const Weighted &a, const Weighted &b) { return a.value < b.value; });
        prefix.resize(s.size());
        int64_t c = 0;
        for (size_t e = 0; e < s.size(); ++e) {
            prefix[e] = c;
            c += s[e].count;
        }
        total = c;
    }
    double at(int64_t pos) const
    {
        // last entry whose prefix <= pos
        size_t lo = 0, hi = s.size();
        while (hi - lo > 1) {
            size_t mid = (lo + hi) / 2;
            if (prefix[mid] <= pos)
                lo = mid;
            else
                hi = mid;
        }
        while (lo + 1 < s.size() && s[lo].count == 0)
            ++lo;
        return s[lo].value;
    }
    double quantile(double p) const
    {
        const double h = (double)(total - 1) * p;
        const int64_t i = (int64_t)std::floor(h);
        const double f = h - (double)i;
        const double v0 = at(i);
        if (i + 1 >= total)
            return v0;
        return v0 + f * (at(i + 1) - v0);
    }
};

int learn_quantizer(const float *Qt, int64_t nq, int J, int64_t ldq, const uint8_t *codes, int64_t n,
                    const float *C, int M, const bolt::Metric &mt, const double *alphas, int nalpha, float *a_out,
                    float *offsets, int32_t *alpha_idx)
{
    const int sub = J / M;
    // per query the fp64 scale of the cosine tables: its norm
    std::vector<double> qnorm((size_t)nq, 1.0);
    if (mt.kind == BOLT_METRIC_COSINE)
        for (int64_t q = 0; q < nq; ++q) {
            double s = 0.0;
            for (int j = 0; j < J; ++j)
                s += (double)Qt[q * ldq + j] * (double)Qt[q * ldq + j];
            qnorm[q] = std::sqrt(s);
        }
    // how many training vectors carry each code in each subspace
    std::vector<int64_t> count((size_t)M * K, 0);
    for (int64_t r = 0; r < n; ++r)
        for (int t = 0; t < M / 2; ++t) {
            const uint8_t b = codes[r * (M / 2) + t];
            count[(2 * t) * K + (b & 15)] += 1;
            count[(2 * t + 1) * K + (b >> 4)] += 1;
        }
    // table m's sample: D_m[i](q) weighted by count[m][i], over queries q
    std::vector<WeightedSample> table(M);
    parallel_for(M, [&](int m) {
        WeightedSample &ws = table[m];
        ws.s.reserve((size_t)nq * K);
        for (int64_t q = 0; q < nq; ++q)
            for (int i = 0; i < K; ++i) {
                double d = 0.0;
                for (int j = 0; j < sub; ++j) {
                    const double qv = Qt[q * ldq + (int64_t)m * sub + j];
                    const double cv = C[((int64_t)m * K + i) * sub + j];
                    switch (mt.kind) {
                    case BOLT_METRIC_L2: d += (qv - cv) * (qv - cv); break;
                    case BOLT_METRIC_L1: d += std::fabs(qv - cv); break;
                    case 3: d += std::pow(std::fabs(qv - cv), (double)mt.p); break;
                    case BOLT_METRIC_COSINE: d += (qnorm[q] > 0.0 ? qv / qnorm[q] : 0.0) * cv; break;
                    default: d += qv * cv;
                    }
                }
                ws.s.push_back({d, count[(size_t)m * K + i]});
            }
        ws.finish();
    });
    double best_loss = INFINITY;
    int best = -1;
    std::vector<double> b(M);
    std::vector<float> boff(M);
    for (int ai = 0; ai < nalpha; ++ai) {
        const double alpha = alphas[ai];
        for (int m = 0; m < M; ++m)
            b[m] = table[m].quantile(alpha);
        WeightedSample pool;
        pool.s.reserve((size_t)M * nq * K);
        for (int m = 0; m < M; ++m)
            for (const Weighted &w : table[m].s)
                pool.s.push_back({w.value - b[m], w.count});
        pool.finish();
        const double top = pool.quantile(1.0 - alpha);
        const float a = top > 0.0 ? (float)(255.0 / top) : 1.0f;
        for (int m = 0; m < M; ++m)
            boff[m] = (float)((double)a * b[m]);
        double err = 0.0, wsum = 0.0;
        for (int m = 0; m < M; ++m)
            for (const Weighted &w : table[m].s) {
                double beta = std::floor((double)a * w.value - (double)boff[m]);
                beta = std::min(255.0, std::max(0.0, beta));
                const double rec = (beta + (double)boff[m]) / (double)a;
                err += (double)w.count * (rec - w.value) * (rec - w.value);
                wsum += (double)w.count;
            }
        const double loss = wsum > 0.0 ? err / wsum : 0.0;
        if (loss < best_loss) {
            best_loss = loss;
            best = ai;
            *a_out = a;
            std::memcpy(offsets, boff.data(), sizeof(float) * M);
        }
    }
    if (alpha_idx)
        *alpha_idx = best;
    if (best < 0)
        return bolt::fail(BOLT_ERR_INVALID, "quantiser learning found no finite loss");
    return BOLT_OK;
}

// Host-side encoding of the training set (the same rule as bolt_encode, in
// double precision; only the code histogram of the training set is used).
void encode_host(const float *X, int64_t n, int J, int64_t ldx, const float *C, int M, uint8_t *codes)
{
    const int sub = J / M;
    // one writer per code byte: thread t owns subspaces 2t and 2t+1
    parallel_for(M / 2, [&](int t) {
        for (int64_t r = 0; r < n; ++r) {
            uint8_t byte = 0;
            for (int h = 0; h < 2; ++h) {
                const int m = 2 * t + h;
                int best = 0;
                double bestd = INFINITY;
                for (int i = 0; i < K; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < sub; ++j) {
                        const double d = (double)X[r * ldx + (int64_t)m * sub + j] -
                                         (double)C[((int64_t)m * K + i) * sub + j];
                        s += d * d;
                    }
                    if (s < bestd) {
                        bestd = s;
                        best = i;
                    }
                }
                byte |= (uint8_t)(best << (4 * h));
            }
            codes[r * (M / 2) + t] = byte;
        }
    });
}

}  // namespace

extern "C" int bolt_learn_quantizer_host(const float *Qt, int64_t nq, int32_t J, int64_t ldq,
                                         const uint8_t *codes, int64_t n, const float *centroids,
                                         int32_t M, int32_t metric, const double *alphas,
                                         int32_t nalpha, float *a, float *offsets, int32_t *alpha_idx)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    Metric mt;
    BOLT_TRY(decode_metric(metric, &mt));
    if (nq < 1 || n < 1 || nalpha < 1 || ldq < J)
        return fail(BOLT_ERR_INVALID, "need nq >= 1, n >= 1, nalpha >= 1 and ldq >= J");
    if (!Qt || !codes || !centroids || !alphas || !a || !offsets)
        return fail(BOLT_ERR_INVALID, "bolt_learn_quantizer_host: null pointer");
    for (int i = 0; i < nalpha; ++i)
        if (!(alphas[i] >= 0.0 && alphas[i] < 0.5))
            return fail(BOLT_ERR_INVALID, "alpha must be in [0, 0.5)");
    return learn_quantizer(Qt, nq, J, ldq, codes, n, centroids, M, mt, alphas, nalpha, a, offsets,
                           alpha_idx);
}

extern "C" int bolt_train_host(const float *X, int64_t n, int32_t J, int64_t ldx, int32_t M,
                               int32_t iters, const int64_t *init_rows, const float *Qt, int64_t nq,
                               int64_t ldq, int32_t metric, const double *alphas, int32_t nalpha,
                               float *centroids, float *a, float *offsets, int32_t *alpha_idx)
{
    using namespace bolt;
    BOLT_TRY(check_JM(J, M));
    if (n < K || iters < 0 || ldx < J)
        return fail(BOLT_ERR_INVALID, "need n >= 16 training rows, iters >= 0, ldx >= J");
    if (!X || !init_rows || !centroids)
        return fail(BOLT_ERR_INVALID, "bolt_train_host: null pointer");
    for (int i = 0; i < K; ++i)
        if (init_rows[i] < 0 || init_rows[i] >= n)
            return fail(BOLT_ERR_INVALID, "init_rows[%d] out of range", i);
    const int sub = J / M;
    parallel_for(M, [&](int m) {
        kmeans_subspace(X, n, ldx, sub, m, iters, init_rows, centroids + (int64_t)m * K * sub);
    });
    std::vector<uint8_t> codes((size_t)n * (M / 2));
    encode_host(X, n, J, ldx, centroids, M, codes.data());
    return bolt_learn_quantizer_host(Qt, nq, J, ldq, codes.data(), n, centroids, M, metric, alphas,
                                     nalpha, a, offsets, alpha_idx);
}
