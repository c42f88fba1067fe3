// fill.hip -- device-side texel fill of the seeded input generator.
//
// Writes level 0 of every edge texture with the same values as
// htexgen/texels.py (splitmix64-based counter hash; uniform or smooth lattice
// noise; mirrored content on boundary edges).  Input generation only: no part
// of the sampling arithmetic lives here.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash5(uint64_t seed, uint64_t a, uint64_t b, uint64_t c,
                                          uint64_t d)
{
    uint64_t x = splitmix64(seed);
    x = splitmix64(x ^ a);
    x = splitmix64(x ^ b);
    x = splitmix64(x ^ c);
    return splitmix64(x ^ d);
}

__constant__ int32_t kRamp[8] = {1, 6, 14, 25, 39, 50, 58, 63};

__global__ void k_fill(int kind, uint64_t seed, int32_t E, const uint8_t *log2res,
                       const int64_t *base, const uint8_t *boundary, float *tex, int channels)
{
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int k = log2res[e];
        const int64_t n = int64_t(1) << k;
        const bool bnd = boundary[e] != 0;
        for (int64_t t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int64_t i = t & (n - 1), j = t >> k;
            int64_t si = i, sj = j;
            if (bnd && i + j > n - 1) {
                si = n - 1 - j;
                sj = n - 1 - i;
            }
            float vals[4];
            for (int c = 0; c < channels; ++c) {
                if (kind == 0) {
                    const uint64_t hv = hash5(seed, (uint64_t)e, (uint64_t)(sj * n + si), (uint64_t)c, 0);
                    vals[c] = (float)(int32_t)(hv >> 40) * 0x1p-24f;
                } else {
                    const int64_t a = si >> 3, b = sj >> 3;
                    const int32_t rx1 = kRamp[si & 7], ry1 = kRamp[sj & 7];
                    const int32_t rx0 = 64 - rx1, ry0 = 64 - ry1;
                    auto lat = [&](int64_t aa, int64_t bb) -> int32_t {
                        return (int32_t)(hash5(seed, (uint64_t)e, (uint64_t)c, (uint64_t)aa, (uint64_t)bb) % 63u) + 1;
                    };
                    const int32_t num = rx0 * ry0 * lat(a, b) + rx1 * ry0 * lat(a + 1, b) +
                                        rx0 * ry1 * lat(a, b + 1) + rx1 * ry1 * lat(a + 1, b + 1);
                    vals[c] = (float)num * 0x1p-18f;
                }
            }
            for (int c = 0; c < channels; ++c) tex[channels * (base[e] + t) + c] = vals[c];
        }
    }
}

}  // namespace

// texels: float32 [total][channels]; a one-channel pool receives channel 0
// of the four-channel values.
extern "C" int htexgen_fill_level0(int kind, uint64_t seed, int32_t E, const uint8_t *log2res,
                                   const int64_t *base, const uint8_t *boundary, float *texels,
                                   int channels, void *stream)
{
    if (E <= 0) return 0;
    if (kind != 0 && kind != 1) return -1;
    if (channels != 1 && channels != 4) return -1;
    const uint32_t grid = (uint32_t)(E < (1 << 20) ? E : (1 << 20));
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), kind,
                       seed, E, log2res, base, boundary, texels, channels);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
