// Internal helpers of the Bolt HIP library: error reporting and argument checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "bolt.h"

namespace bolt {

// Record a message for bolt_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// BOLT_OK, or BOLT_ERR_DEVICE with the runtime's message.
int check_launch(const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Shape rules shared by every entry point (see bolt.h).
inline int check_M(int32_t M)
{
    if (M < 2 || M > 256 || (M & 1))
        return fail(BOLT_ERR_SHAPE, "M must be even and in [2, 256] (got %d)", M);
    return BOLT_OK;
}

inline int check_JM(int32_t J, int32_t M)
{
    int st = check_M(M);
    if (st)
        return st;
    if (J <= 0 || J % M)
        return fail(BOLT_ERR_SHAPE, "J must be a positive multiple of M (J=%d, M=%d)", J, M);
    return BOLT_OK;
}

inline int check_N(int64_t N, const char *name)
{
    if (N < 0 || N > INT32_MAX)
        return fail(BOLT_ERR_SHAPE, "%s must be in [0, 2^31-1] (got %lld)", name, (long long)N);
    return BOLT_OK;
}

constexpr int kCentroids = 16;  // K = 16 centroids per codebook (4-bit codes)

// A decoded metric code (bolt.h): kind BOLT_METRIC_L2, _DOT, _L1, 3 (L_p with
// exponent p) or _COSINE; similarities (dot, cosine) retrieve the largest sums.
struct Metric {
    int kind = 0;
    int p = 0;
    bool largest = false;
};

inline int decode_metric(int32_t code, Metric *m)
{
    if (code == BOLT_METRIC_L2 || code == BOLT_METRIC_DOT || code == BOLT_METRIC_L1 || code == BOLT_METRIC_COSINE) {
        m->kind = code;
        m->p = code == BOLT_METRIC_L1 ? 1 : (code == BOLT_METRIC_L2 ? 2 : 0);
    } else if (code >= 3 + 256 && (code - 3) % 256 == 0 && (code - 3) / 256 <= 16) {
        m->kind = 3;
        m->p = (code - 3) / 256;
    } else {
        return fail(BOLT_ERR_INVALID, "unknown metric code %d (0 L2, 1 dot, 2 L1, 4 cosine, 3 + 256 p for L_p "
                                      "with 1 <= p <= 16)", code);
    }
    m->largest = code == BOLT_METRIC_DOT || code == BOLT_METRIC_COSINE;
    return BOLT_OK;
}

// Times the launches enqueued during its lifetime on stream s under `name`
// when timing is enabled (bolt_prof_enable); otherwise does nothing.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    const char *name_;
    hipStream_t s_;
    void *start_;
};

}  // namespace bolt

#define BOLT_TRY(expr)          \
    do {                        \
        int _st = (expr);       \
        if (_st != BOLT_OK)     \
            return _st;         \
    } while (0)
