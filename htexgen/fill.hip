// fill.hip -- device-side texel fill of the seeded input generator.
//
// Writes level 0 of every edge texture with the same values as
// htexgen/texels.py (splitmix64-based counter hash; uniform, smooth lattice
// noise or Perlin gradient noise; mirrored content on boundary edges).  Input generation only: no part
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

// Perlin's quintic fade at t = (2f + 1) / 16, times 2^20, and the eight
// lattice gradients (see htexgen/texels.py)
__constant__ int64_t kFade[8] = {2326, 51138, 188750, 402682, 645894, 859826, 997438, 1046250};
__constant__ int32_t kGrad[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1},
                                    {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};

// Perlin gradient noise texel of edge e, channel c, at source texel (si, sj),
// in exact integer arithmetic: (2^18 + 31 M) 2^-24 with
// M = clamp(floor(N / 2^26) + 2^18, 0, 2^19) and N / 2^44 the noise.
__device__ __forceinline__ float perlin_texel(uint64_t seed, int64_t e, int c, int64_t si,
                                              int64_t sj)
{
    const int64_t a = si >> 3, b = sj >> 3;
    const int64_t x = 2 * (si & 7) + 1, y = 2 * (sj & 7) + 1;
    const int64_t wx1 = kFade[si & 7], wy1 = kFade[sj & 7];
    const int64_t wx0 = (int64_t(1) << 20) - wx1, wy0 = (int64_t(1) << 20) - wy1;
    auto corner = [&](int64_t da, int64_t db) -> int64_t {
        const int g = (int)(hash5(seed, (uint64_t)e, (uint64_t)c, (uint64_t)(a + da),
                                  (uint64_t)(b + db)) & 7u);
        return kGrad[g][0] * (x - 16 * da) + kGrad[g][1] * (y - 16 * db);
    };
    const int64_t N = wx0 * wy0 * corner(0, 0) + wx1 * wy0 * corner(1, 0) +
                      wx0 * wy1 * corner(0, 1) + wx1 * wy1 * corner(1, 1);
    int64_t M = (N >> 26) + (int64_t(1) << 18);
    M = M < 0 ? 0 : (M > (int64_t(1) << 19) ? (int64_t(1) << 19) : M);
    return (float)(int32_t)((int64_t(1) << 18) + 31 * M) * 0x1p-24f;
}

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
                } else if (kind == 2) {
                    vals[c] = perlin_texel(seed, e, c, si, sj);
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
    if (kind < 0 || kind > 2) return -1;
    if (channels != 1 && channels != 4) return -1;
    const uint32_t grid = (uint32_t)(E < (1 << 20) ? E : (1 << 20));
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), kind,
                       seed, E, log2res, base, boundary, texels, channels);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
