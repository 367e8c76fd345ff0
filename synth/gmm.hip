// Device implementation of the seeded Gaussian-mixture input generator of
// synth/__init__.py (same definition, exact integer arithmetic), so that
// workloads of billions of rows can be generated in HBM while any row can
// still be regenerated bit for bit on the host.  Input generation only: no
// part of the Bolt method lives here.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__host__ __device__ inline uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void gmm_kernel(uint64_t b_comp, uint64_t b_mean, uint64_t b_noise,
                                                  int64_t row0, int64_t nrows, int J, int64_t ld,
                                                  float *__restrict__ out, uint64_t n_comp)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nrows * J)
        return;
    const int64_t r = e / J;
    const int j = (int)(e - r * J);
    const uint64_t row = (uint64_t)(row0 + r);
    const uint64_t comp = ((splitmix64(b_comp + row) >> 32) * n_comp) >> 32;
    const int64_t mean = (int64_t)(splitmix64(b_mean + comp * (uint64_t)J + (uint64_t)j) >> 40) * 100;
    const uint64_t elem = row * (uint64_t)J + (uint64_t)j;
    int64_t S = 0;
    for (int k = 0; k < 3; ++k) {
        const uint64_t h = splitmix64(b_noise + elem * 3u + (uint64_t)k);
        for (int t = 0; t < 4; ++t)
            S += (int64_t)((h >> (16 * t)) & 0xFFFFu);
    }
    const int64_t v = mean + 10 * (S - 393210) * 256;
    int64_t q = v >> 24;
    const int64_t rem = v - (q << 24);
    if (rem > (1 << 23) || (rem == (1 << 23) && (q & 1)))
        q += 1;
    q = q < 0 ? 0 : (q > 255 ? 255 : q);
    out[r * ld + j] = (float)q;
}

uint64_t stream_base(uint64_t seed, uint64_t s) { return splitmix64(seed * 16u + s); }

}  // namespace

// Rows row0 .. row0+nrows-1 of the mixture sample into out[nrows][ld] (device).
extern "C" int synth_gmm_rows(uint64_t mix_seed, uint64_t draw_seed, int64_t row0, int64_t nrows,
                              int32_t J, int64_t ld, float *out, void *stream)
{
    if (nrows <= 0)
        return 0;
    if (J <= 0 || ld < J || !out)
        return -1;
    const int64_t work = nrows * J;
    hipLaunchKernelGGL(gmm_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), stream_base(draw_seed, 1),
                       stream_base(mix_seed, 2), stream_base(draw_seed, 3), row0, nrows, J, ld, out,
                       (uint64_t)256);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
