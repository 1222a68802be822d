// contrast.hip -- contrast variables (AddContrastVariables, section "Package functions
// introduction": variables known to be irrelevant, on which the distribution of IG_max is
// fitted, left out of the p-value adjustment).  The paper cites the construction without
// defining it; here contrast variable c is a copy of original variable src(c) with its objects
// permuted by a keyed pseudo-random permutation, so it keeps that variable's distribution and
// loses any relation to the decision.
//
//   src(c)  = SplitMix64 draw (seed, c) mod n_var
//   perm_c  : a 4-round balanced Feistel network on 2h-bit indices (2^(2h) >= n_obj, h >= 1),
//             round function = the SplitMix64 finaliser of (round key + right half), keys drawn
//             from (seed, c, round); indices >= n_obj are walked along their cycle until they
//             fall below n_obj (a bijection of [0, n_obj), no storage needed).
//   out[n_var + c][n] = data[src(c)][perm_c(n)]
#include "mdfs_internal.h"

namespace mdfs {

namespace {

__host__ __device__ inline uint64_t cv_fin(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// one SplitMix64 draw keyed by (seed, a, b): absorb each component with one step
__host__ __device__ inline uint64_t cv_draw(uint64_t seed, uint64_t a, uint64_t b)
{
    const uint64_t g = 0x9e3779b97f4a7c15ull;
    uint64_t h = cv_fin(seed + g);
    h = cv_fin(h + (a + 1) * g);
    return cv_fin(h + (b + 1) * g);
}

constexpr uint64_t SRC_TAG = 0x5352434ull;   // draw index of the source choice ("SRC")

__host__ __device__ inline int64_t contrast_src(uint64_t seed, int64_t c, int64_t n_var)
{
    return (int64_t)(cv_draw(seed, (uint64_t)c, SRC_TAG) % (uint64_t)n_var);
}

// half width h of the Feistel domain: smallest h >= 1 with 2^(2h) >= n
__host__ __device__ inline int feistel_half(int64_t n)
{
    int h = 1;
    while ((int64_t(1) << (2 * h)) < n) ++h;
    return h;
}

__device__ inline uint32_t feistel(uint32_t x, int h, const uint64_t (&key)[4])
{
    const uint32_t mask = (1u << h) - 1u;
    uint32_t L = x >> h, R = x & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t F = (uint32_t)cv_fin(key[r] + R) & mask;
        const uint32_t nL = R;
        R = L ^ F;
        L = nL;
    }
    return (L << h) | R;
}

__global__ __launch_bounds__(256) void k_contrast(const float *__restrict__ data, int64_t n_obj, int64_t n_var,
                                                  uint64_t seed, float *__restrict__ out)
{
    const int64_t c = blockIdx.x;
    const int64_t src = contrast_src(seed, c, n_var);
    const int h = feistel_half(n_obj);
    uint64_t key[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) key[r] = cv_draw(seed, (uint64_t)c, (uint64_t)r);
    const float *x = data + src * n_obj;
    float *o = out + (n_var + c) * n_obj;
    const uint32_t dom = 1u << (2 * h);
    for (int64_t n = threadIdx.x; n < n_obj; n += blockDim.x) {
        uint32_t j = feistel((uint32_t)n, h, key);
        // cycle walk; the cycle through n returns to [0, n_obj) within dom steps
        for (uint32_t step = 0; j >= (uint32_t)n_obj && step < dom; ++step) j = feistel(j, h, key);
        o[n] = x[j < (uint32_t)n_obj ? j : 0];
    }
}

}  // namespace

int64_t contrast_source(uint64_t seed, int64_t c, int64_t n_var) { return contrast_src(seed, c, n_var); }

hipError_t launch_contrast(const float *data, int64_t n_obj, int64_t n_var, int64_t n_contrast, uint64_t seed,
                           float *out, hipStream_t stream)
{
    hipError_t e = hipMemcpyAsync(out, data, sizeof(float) * (size_t)n_obj * (size_t)n_var, hipMemcpyDeviceToDevice,
                                  stream);
    if (e != hipSuccess) return e;
    if (n_contrast == 0) return hipSuccess;
    hipLaunchKernelGGL(k_contrast, dim3((unsigned)n_contrast), dim3(256), 0, stream, data, n_obj, n_var, seed, out);
    return hipGetLastError();
}

}  // namespace mdfs
