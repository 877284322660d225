// Jittered-grid node builder.  One thread per node; the random draws come
// from SplitMix64 (Steele, Lea and Flood, 2014) used as a counter-based
// generator: output k of stream `seed` is mix(seed + (k+1)*GAMMA), so every
// thread computes its own draws without a sequential state.  Built with
// -ffp-contract=off: each product and sum is rounded separately.
#include "rbf_internal.h"

namespace rbf {
namespace {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_build_nodes(int dim, int64_t side, int64_t N, double h, double t, uint64_t seed,
                              double *__restrict__ xyz, int8_t *__restrict__ type) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= N) return;
    int64_t g[3] = {0, 0, 0};
    int64_t rem = id;
    bool boundary = false;
    for (int a = 0; a < dim; ++a) {
        g[a] = rem % side;
        rem /= side;
        boundary |= (g[a] == 0) || (g[a] == side - 1);
    }
    for (int a = 0; a < dim; ++a) {
        const double base = (double)g[a] * h;
        double x = base;
        if (!boundary) {
            const uint64_t z = splitmix64_at(seed, (uint64_t)id * (uint64_t)dim + (uint64_t)a);
            const double U = (double)(z >> 11) * 0x1p-53;
            const double v = 2.0 * U - 1.0;
            const double off = v * t;
            x = base + off;
        }
        xyz[a * N + id] = x;
    }
    type[id] = boundary ? 1 : 0;
}

}  // namespace

hipError_t launch_build_nodes(hipStream_t s, int dim, int64_t side, double h, double t, uint64_t seed, double *xyz,
                              int8_t *type) {
    int64_t N = 1;
    for (int a = 0; a < dim; ++a) N *= side;
    hipLaunchKernelGGL(k_build_nodes, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, dim, side, N, h, t, seed,
                       xyz, type);
    return hipGetLastError();
}

}  // namespace rbf
