/*
 * Plain CPU oracle for the Bolt hot path (Blalock & Guttag, "Bolt:
 * Accelerated Data Mining with Fast Vector Compression", KDD 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what every step of the hot
 * path computes, as slowly and as plainly as possible: scalar loops, no
 * blocking, no intrinsics, no reordering.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the GPU library, and the GPU library never
 * calls it.
 *
 * Compiled with -O2 -ffp-contract=off so that every fp32 operation is
 * rounded exactly where it is written; fmaf() is the correctly rounded
 * fused multiply-add.
 *
 * Layouts (the paper fixes none of them; these are the conventions of the
 * whole project):
 *   X          fp32 [N][ldx], first J columns used
 *   centroids  fp32 [M][16][J/M]      (codebook m, centroid i, sub-dimension)
 *   codes      uint8 [N][M/2]          byte t: subspace 2t in bits 0-3,
 *                                      subspace 2t+1 in bits 4-7
 *   luts       [Q][M][16]
 *   scan out   uint16 [Q][N]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define K 16 /* centroids per codebook: Sec. 3.2, change (1) */

static int code_of(const uint8_t *codes, int64_t n, int M, int m)
{
    uint8_t byte = codes[n * (M / 2) + m / 2];
    return (m % 2 == 0) ? (byte & 0x0F) : (byte >> 4);
}

/*
 * Data encoding h(x) (Sec. 3.1, definition of h; K = 16 per Sec. 3.2):
 * for every subspace m, the index of the centroid nearest to x^(m).
 * Subspaces are J/M consecutive dimensions (Sec. 3.1).  The distance used
 * is squared Euclidean whatever the task metric, and ties go to the lowest
 * index.  The decision is taken in fp32 with the canonical order
 *     acc = 0; for j ascending: t = x_j - c_j; acc = fmaf(t, t, acc)
 * which is the precision and order the GPU kernel uses.
 * If dist32 is not NULL it receives the 16 fp32 distances [N][M][16].
 */
void orc_encode(const float *X, int64_t N, int32_t J, int64_t ldx,
                const float *C, int32_t M, uint8_t *codes, float *dist32)
{
    int sub = J / M;
    memset(codes, 0, (size_t)N * (size_t)(M / 2));
    for (int64_t n = 0; n < N; n++) {
        const float *x = X + n * ldx;
        for (int m = 0; m < M; m++) {
            float best = INFINITY;
            int best_i = 0;
            for (int i = 0; i < K; i++) {
                const float *c = C + ((int64_t)m * K + i) * sub;
                float acc = 0.0f;
                for (int jj = 0; jj < sub; jj++) {
                    float t = x[m * sub + jj] - c[jj];
                    acc = fmaf(t, t, acc);
                }
                if (dist32)
                    dist32[(n * M + m) * K + i] = acc;
                if (acc < best) {
                    best = acc;
                    best_i = i;
                }
            }
            codes[n * (M / 2) + m / 2] |= (uint8_t)(best_i << (4 * (m % 2)));
        }
    }
}

/*
 * Exact (fp64) squared distances from every subvector to every centroid,
 * [N][M][16].  Used to report the relative gap of any encoding that
 * differs from the fp32 decision.
 */
void orc_subspace_dists_f64(const float *X, int64_t N, int32_t J, int64_t ldx,
                            const float *C, int32_t M, double *out)
{
    int sub = J / M;
    for (int64_t n = 0; n < N; n++)
        for (int m = 0; m < M; m++)
            for (int i = 0; i < K; i++) {
                double s = 0.0;
                for (int jj = 0; jj < sub; jj++) {
                    double t = (double)X[n * ldx + m * sub + jj] -
                               (double)C[((int64_t)m * K + i) * sub + jj];
                    s += t * t;
                }
                out[(n * M + m) * K + i] = s;
            }
}

/*
 * Unit-norm rows, for cosine similarity (Sec. 1.1 names it among the
 * similarities the method serves; with unit vectors it is the dot product):
 *   s = 0; for j ascending: s = fmaf(x_j, x_j, s);  n = sqrtf(s);
 *   y_j = x_j / n          (each operation correctly rounded in fp32)
 * A zero row stays zero.
 */
void orc_normalize_rows(const float *X, int64_t N, int32_t J, int64_t ldx, float *Y, int64_t ldy)
{
    for (int64_t r = 0; r < N; r++) {
        const float *x = X + r * ldx;
        float s = 0.0f;
        for (int j = 0; j < J; j++)
            s = fmaf(x[j], x[j], s);
        float n = sqrtf(s);
        for (int j = 0; j < J; j++)
            Y[r * ldy + j] = n > 0.0f ? x[j] / n : 0.0f;
    }
}

/*
 * Query encoding g(q) (Sec. 3.1, definition of the matrix D) followed by
 * the learned quantisation beta_m (Sec. 3.2).
 *
 *   D[m][i] = sum over j in p_m of delta(q_j, c_ij)   (eq. distFuncForm)
 *       metric 0, squared Euclidean:  delta = (q - c)^2
 *       metric 1, dot product:        delta = q * c
 *       metric 2, L1:                 delta = |q - c|
 *       metric 3, L_p (integer p):    delta = |q - c|^p, the L_p distance
 *                                     raised to the p (f the p-th root)
 *       metric 4, cosine similarity:  delta = (q / |q|) * c, the dot
 *                                     product with the unit query (the
 *                                     database side encodes unit rows)
 *
 *   lut64: the entries in fp64 (the "true" table).
 *   lut32: the entries in fp32, canonical order, acc = 0 then j ascending,
 *          L2: t = q_j - c_j; acc = fmaf(t, t, acc)
 *          dot: acc = fmaf(q_j, c_j, acc)
 *          L1:  acc = acc + |q_j - c_j|
 *          L_p: t = |q_j - c_j|; p = 1: acc = acc + t; p >= 2:
 *               w = t, then w = w * t (p - 2 times), acc = fmaf(w, t, acc)
 *               (so L_1 and L_2 give exactly the L1 and L2 tables)
 *          cosine: u = the unit query (orc_normalize_rows), then as dot
 *   lut8:  beta = max(0, min(255, floor(a*y - b'_m))), with a*y - b'_m
 *          evaluated as one fmaf(a, lut32, -offsets[m]).  offsets[m] is
 *          b'_m = a * F^-1(alpha) for table m, i.e. the offset in
 *          quantised units, so the alpha-quantile maps to 0.
 * Any of the three outputs may be NULL.  p is used by metric 3 only.
 */
void orc_luts(const float *Qv, int64_t Q, int32_t J, int64_t ldq,
              const float *C, int32_t M, int32_t metric, int32_t p, float a,
              const float *offsets, double *lut64, float *lut32, uint8_t *lut8)
{
    int sub = J / M;
    float *unit = (float *)malloc(sizeof(float) * (size_t)(J > 0 ? J : 1));
    for (int64_t q = 0; q < Q; q++) {
        double qn64 = 0.0;
        if (metric == 4) {
            orc_normalize_rows(Qv + q * ldq, 1, J, ldq, unit, J);
            for (int j = 0; j < J; j++)
                qn64 += (double)Qv[q * ldq + j] * (double)Qv[q * ldq + j];
            qn64 = sqrt(qn64);
        }
        for (int m = 0; m < M; m++)
            for (int i = 0; i < K; i++) {
                const float *qv = Qv + q * ldq + m * sub;
                const float *c = C + ((int64_t)m * K + i) * sub;
                double s64 = 0.0;
                float s32 = 0.0f;
                for (int jj = 0; jj < sub; jj++) {
                    if (metric == 0) {
                        double t = (double)qv[jj] - (double)c[jj];
                        s64 += t * t;
                        float t32 = qv[jj] - c[jj];
                        s32 = fmaf(t32, t32, s32);
                    } else if (metric == 2) {
                        s64 += fabs((double)qv[jj] - (double)c[jj]);
                        s32 = s32 + fabsf(qv[jj] - c[jj]);
                    } else if (metric == 3) {
                        s64 += pow(fabs((double)qv[jj] - (double)c[jj]), (double)p);
                        float t = fabsf(qv[jj] - c[jj]);
                        if (p == 1) {
                            s32 = s32 + t;
                        } else {
                            float w = t;
                            for (int e = 2; e < p; e++)
                                w = w * t;
                            s32 = fmaf(w, t, s32);
                        }
                    } else if (metric == 4) {
                        s64 += (qn64 > 0.0 ? (double)qv[jj] / qn64 : 0.0) * (double)c[jj];
                        s32 = fmaf(unit[m * sub + jj], c[jj], s32);
                    } else {
                        s64 += (double)qv[jj] * (double)c[jj];
                        s32 = fmaf(qv[jj], c[jj], s32);
                    }
                }
                int64_t e = (q * M + m) * K + i;
                if (lut64)
                    lut64[e] = s64;
                if (lut32)
                    lut32[e] = s32;
                if (lut8) {
                    float y = fmaf(a, s32, -offsets[m]);
                    float f = floorf(y);
                    if (!(f > 0.0f))
                        f = 0.0f;
                    if (f > 255.0f)
                        f = 255.0f;
                    lut8[e] = (uint8_t)f;
                }
            }
    }
    free(unit);
}

/*
 * The scan (Sec. 3.1, the approximate distance as a sum of table entries):
 *   out[q][n] = sum over m of lut8[q][m][h(x_n)_m]
 * summed exactly as an integer; M <= 256 keeps it below 65536.
 * The monotone f of the distance form (Sec. 1.1) is not applied.
 */
void orc_scan(const uint8_t *codes, int64_t N, int32_t M, const uint8_t *lut8,
              int64_t Q, uint16_t *out)
{
    for (int64_t q = 0; q < Q; q++)
        for (int64_t n = 0; n < N; n++) {
            uint32_t s = 0;
            for (int m = 0; m < M; m++)
                s += lut8[(q * M + m) * K + code_of(codes, n, M, m)];
            out[q * N + n] = (uint16_t)s;
        }
}

/* Same sums, for an arbitrary list of (query, row) pairs. */
void orc_scan_pairs(const uint8_t *codes, int32_t M, const uint8_t *lut8,
                    const int64_t *qs, const int64_t *ns, int64_t P,
                    uint32_t *out)
{
    for (int64_t p = 0; p < P; p++) {
        uint32_t s = 0;
        for (int m = 0; m < M; m++)
            s += lut8[(qs[p] * M + m) * K + code_of(codes, ns[p], M, m)];
        out[p] = s;
    }
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Top-k retrieval (Sec. 1.2, "the k closest vectors"; Sec. 4.5 ranks by
 * smallest approximate distance).  For squared L2 the k smallest sums, for
 * the dot product (a similarity, maximum inner product search) the k
 * largest.  Equal sums are ordered by ascending row index, which makes the
 * answer unique: the key (s << 32 | n), or ((65535 - s) << 32 | n) for
 * largest, is sorted ascending and the first k kept.  Missing entries
 * (k > N) are vals = 65535 (L2) or 0 (dot), idx = -1.
 */
void orc_topk(const uint16_t *d, int64_t Q, int64_t N, int64_t ldd, int32_t k,
              int32_t largest, uint16_t *vals, int32_t *idx)
{
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(N > 0 ? N : 1));
    for (int64_t q = 0; q < Q; q++) {
        for (int64_t n = 0; n < N; n++) {
            uint64_t s = d[q * ldd + n];
            if (largest)
                s = 65535u - s;
            keys[n] = (s << 32) | (uint64_t)n;
        }
        qsort(keys, (size_t)N, sizeof(uint64_t), cmp_u64);
        for (int32_t r = 0; r < k; r++) {
            if (r < N) {
                uint64_t s = keys[r] >> 32;
                vals[q * k + r] = (uint16_t)(largest ? 65535u - s : s);
                idx[q * k + r] = (int32_t)(keys[r] & 0xFFFFFFFFu);
            } else {
                vals[q * k + r] = largest ? 0 : 65535;
                idx[q * k + r] = -1;
            }
        }
    }
    free(keys);
}

/*
 * Bolt No Quantize (Sec. 4.2): the sum of the float table entries selected
 * by the codes.  The paper fixes no order for it; this project's reading is
 * ascending m with every add rounded to fp32:
 *   acc = 0;  acc = acc + D[q][m][code(n, m)]  for m = 0 .. M-1.
 */
void orc_scan_f32(const uint8_t *codes, int64_t N, int32_t M, const float *lutf,
                  int64_t Q, float *out)
{
    for (int64_t q = 0; q < Q; q++)
        for (int64_t n = 0; n < N; n++) {
            float acc = 0.0f;
            for (int m = 0; m < M; m++)
                acc = acc + lutf[(q * M + m) * K + code_of(codes, n, M, m)];
            out[q * N + n] = acc;
        }
}

/* One (value, index) candidate of a float top-k. */
struct fcand {
    float v;
    int64_t i;
};

static int cmp_fcand_small(const void *a, const void *b)
{
    const struct fcand *x = (const struct fcand *)a, *y = (const struct fcand *)b;
    if (x->v != y->v)
        return x->v < y->v ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

static int cmp_fcand_large(const void *a, const void *b)
{
    const struct fcand *x = (const struct fcand *)a, *y = (const struct fcand *)b;
    if (x->v != y->v)
        return x->v > y->v ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

/*
 * Top-k of float rows (Sec. 1.2, the k closest): the k smallest values
 * (largest = 0) or the k largest, equal values by ascending index; rows with
 * fewer than k values are padded with +inf / -inf and index -1.
 */
void orc_topk_f32(const float *d, int64_t Q, int64_t N, int64_t ldd, int32_t k,
                  int32_t largest, float *vals, int32_t *idx)
{
    struct fcand *c = (struct fcand *)malloc(sizeof(struct fcand) * (size_t)(N > 0 ? N : 1));
    for (int64_t q = 0; q < Q; q++) {
        for (int64_t n = 0; n < N; n++) {
            c[n].v = d[q * ldd + n];
            c[n].i = n;
        }
        qsort(c, (size_t)N, sizeof(struct fcand), largest ? cmp_fcand_large : cmp_fcand_small);
        for (int32_t r = 0; r < k; r++) {
            if (r < N) {
                vals[q * k + r] = c[r].v;
                idx[q * k + r] = (int32_t)c[r].i;
            } else {
                vals[q * k + r] = largest ? -INFINITY : INFINITY;
                idx[q * k + r] = -1;
            }
        }
    }
    free(c);
}

/*
 * Reconstruction of a quantised sum (Sec. 3.2: y_hat = (beta + b) / a,
 * summed over the M tables whose offsets add up to one bias):
 *   S_hat = (S + sum_m b'_m) / a          in fp64.
 */
void orc_rescale_f64(const uint16_t *S, int64_t count, float a,
                     const float *offsets, int32_t M, double *out)
{
    double bias = 0.0;
    for (int m = 0; m < M; m++)
        bias += (double)offsets[m];
    for (int64_t e = 0; e < count; e++)
        out[e] = ((double)S[e] + bias) / (double)a;
}

/*
 * The fp32 rescale of the approximate matrix product: out = fp32(fp32(S +
 * bias) * scale), two roundings, with bias and scale given in fp32
 * (scale = 1/a, bias = sum of the offsets).
 */
void orc_rescale_f32(const uint16_t *S, int64_t count, float bias, float scale,
                     float *out)
{
    for (int64_t e = 0; e < count; e++) {
        float t = (float)S[e] + bias;
        out[e] = t * scale;
    }
}

/* ------------------------------------------------------------------ */
/* Offline training (Sec. 1.2 offline phase; k-means per Sec. 3.1;     */
/* quantiser learning per Sec. 3.2).  Host only, not a parity subject. */
/* ------------------------------------------------------------------ */

/*
 * k-means with K = 16 on every subspace, Lloyd iterations.
 * init_rows: 16 row indices; centroid i of every subspace starts at row
 * init_rows[i].  Assignment in fp64, ties to the lowest index; the update
 * is the fp64 mean in ascending row order; an empty cluster keeps its
 * previous centroid.  objective (optional, [iters+1]) receives the total
 * squared error of the assignment made before each update and after the
 * last one.
 */
void orc_kmeans(const float *X, int64_t n, int32_t J, int64_t ldx, int32_t M,
                int32_t iters, const int64_t *init_rows, float *C,
                double *objective)
{
    int sub = J / M;
    double *sum = (double *)malloc(sizeof(double) * K * (size_t)sub);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * K);
    int *assign = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (objective)
        for (int t = 0; t <= iters; t++)
            objective[t] = 0.0;
    for (int m = 0; m < M; m++) {
        float *Cm = C + (int64_t)m * K * sub;
        for (int i = 0; i < K; i++)
            for (int jj = 0; jj < sub; jj++)
                Cm[i * sub + jj] = X[init_rows[i] * ldx + m * sub + jj];
        for (int t = 0; t <= iters; t++) {
            double obj = 0.0;
            for (int64_t r = 0; r < n; r++) {
                double best = INFINITY;
                int bi = 0;
                for (int i = 0; i < K; i++) {
                    double s = 0.0;
                    for (int jj = 0; jj < sub; jj++) {
                        double d = (double)X[r * ldx + m * sub + jj] - (double)Cm[i * sub + jj];
                        s += d * d;
                    }
                    if (s < best) {
                        best = s;
                        bi = i;
                    }
                }
                assign[r] = bi;
                obj += best;
            }
            if (objective)
                objective[t] += obj;
            if (t == iters)
                break;
            memset(sum, 0, sizeof(double) * K * (size_t)sub);
            memset(cnt, 0, sizeof(int64_t) * K);
            for (int64_t r = 0; r < n; r++) {
                cnt[assign[r]]++;
                for (int jj = 0; jj < sub; jj++)
                    sum[assign[r] * sub + jj] += (double)X[r * ldx + m * sub + jj];
            }
            for (int i = 0; i < K; i++)
                if (cnt[i] > 0)
                    for (int jj = 0; jj < sub; jj++)
                        Cm[i * sub + jj] = (float)(sum[i * sub + jj] / (double)cnt[i]);
        }
    }
    free(sum);
    free(cnt);
    free(assign);
}

/* A weighted sample: value v repeated w times. */
typedef struct {
    double v;
    int64_t w;
} wsample;

static int cmp_ws(const void *a, const void *b)
{
    double x = ((const wsample *)a)->v, y = ((const wsample *)b)->v;
    return (x > y) - (x < y);
}

/* Element at 0-based position pos of the expanded sorted multiset. */
static double ws_at(const wsample *s, int64_t ns, int64_t pos)
{
    int64_t c = 0;
    for (int64_t e = 0; e < ns; e++) {
        c += s[e].w;
        if (pos < c)
            return s[e].v;
    }
    return s[ns - 1].v;
}

/* Linear-interpolation quantile (numpy's default, "type 7") of the
 * expanded multiset; s must be sorted by value. */
static double ws_quantile(const wsample *s, int64_t ns, int64_t total, double p)
{
    double h = (double)(total - 1) * p;
    int64_t lo = (int64_t)floor(h);
    double frac = h - (double)lo;
    double vlo = ws_at(s, ns, lo);
    if (lo + 1 >= total)
        return vlo;
    double vhi = ws_at(s, ns, lo + 1);
    return vlo + frac * (vhi - vlo);
}

/*
 * Learning the quantiser (Sec. 3.2): b_m = F_m^-1(alpha) per table,
 * a = 255 / F^-1(1 - alpha) of the offset distances pooled over all tables,
 * alpha from a grid, chosen to minimise E[(y_hat - y)^2].
 *
 * The distribution Y of table m is taken over pairs (training query q,
 * training vector x) of the value the scan adds, D_m[h(x)_m](q).  For a
 * fixed q that value depends on x only through h(x)_m, so Y_m is the
 * multiset {D_m[i](q) repeated count_m[i] times : q, i}, where count_m[i]
 * is the number of training vectors with code i in subspace m.
 *
 * Qt: training queries [nq][ldq]; codes: packed codes of the n training
 * vectors.  D is evaluated in fp64.  For each alpha:
 *   b_m   = quantile_alpha(Y_m)
 *   a     = 255 / quantile_{1-alpha}(pool of y - b_m),  a = 1 if that is <= 0
 *   b'_m  = fp32(a * b_m)
 *   beta  = clamp(floor(a*y - b'_m), 0, 255),  y_hat = (beta + b'_m) / a
 *   loss  = weighted mean over all samples of (y_hat - y)^2
 * The alpha with the smallest loss wins (ties: the smaller alpha).
 * Outputs: a, offsets[M] = b'_m, the chosen alpha index, and the loss of
 * every alpha (losses[nalpha], optional).
 */
int orc_learn_quantizer(const float *Qt, int64_t nq, int32_t J, int64_t ldq,
                        const uint8_t *codes, int64_t n, const float *C, int32_t M,
                        int32_t metric, int32_t p, const double *alphas, int32_t nalpha,
                        float *a_out, float *offsets_out, double *losses)
{
    int64_t per_table = nq * K;
    int64_t *count = (int64_t *)calloc((size_t)M * K, sizeof(int64_t));
    wsample *y = (wsample *)malloc(sizeof(wsample) * (size_t)(M * per_table));
    wsample *pool = (wsample *)malloc(sizeof(wsample) * (size_t)(M * per_table));
    double *b = (double *)malloc(sizeof(double) * (size_t)M);
    float *boff = (float *)malloc(sizeof(float) * (size_t)M);
    for (int64_t r = 0; r < n; r++)
        for (int m = 0; m < M; m++)
            count[m * K + code_of(codes, r, M, m)]++;
    double *tab = (double *)malloc(sizeof(double) * (size_t)M * K);
    for (int64_t q = 0; q < nq; q++) {
        /* the fp64 table of training query q, as orc_luts defines it */
        orc_luts(Qt + q * ldq, 1, J, ldq, C, M, metric, p, 1.0f, NULL, tab, NULL, NULL);
        for (int m = 0; m < M; m++)
            for (int i = 0; i < K; i++) {
                wsample *e = &y[m * per_table + q * K + i];
                e->v = tab[m * K + i];
                e->w = count[m * K + i];
            }
    }
    free(tab);
    int64_t total_m = nq * n; /* multiset size of one table */
    for (int m = 0; m < M; m++)
        qsort(y + m * per_table, (size_t)per_table, sizeof(wsample), cmp_ws);

    double best_loss = INFINITY;
    int best = -1;
    for (int ai = 0; ai < nalpha; ai++) {
        double alpha = alphas[ai];
        for (int m = 0; m < M; m++)
            b[m] = ws_quantile(y + m * per_table, per_table, total_m, alpha);
        for (int m = 0; m < M; m++)
            for (int64_t e = 0; e < per_table; e++) {
                pool[m * per_table + e].v = y[m * per_table + e].v - b[m];
                pool[m * per_table + e].w = y[m * per_table + e].w;
            }
        qsort(pool, (size_t)(M * per_table), sizeof(wsample), cmp_ws);
        double top = ws_quantile(pool, M * per_table, total_m * M, 1.0 - alpha);
        double a = top > 0.0 ? 255.0 / top : 1.0;
        float a32 = (float)a;
        for (int m = 0; m < M; m++)
            boff[m] = (float)((double)a32 * b[m]);
        double se = 0.0;
        double wsum = 0.0;
        for (int m = 0; m < M; m++)
            for (int64_t e = 0; e < per_table; e++) {
                double v = y[m * per_table + e].v;
                double w = (double)y[m * per_table + e].w;
                double t = floor((double)a32 * v - (double)boff[m]);
                if (t < 0.0)
                    t = 0.0;
                if (t > 255.0)
                    t = 255.0;
                double yh = (t + (double)boff[m]) / (double)a32;
                se += w * (yh - v) * (yh - v);
                wsum += w;
            }
        double loss = wsum > 0.0 ? se / wsum : 0.0;
        if (losses)
            losses[ai] = loss;
        if (loss < best_loss) {
            best_loss = loss;
            best = ai;
            *a_out = a32;
            memcpy(offsets_out, boff, sizeof(float) * (size_t)M);
        }
    }
    free(count);
    free(y);
    free(pool);
    free(b);
    free(boff);
    return best;
}
