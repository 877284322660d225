// Host side of the null-space weight solver: which systems it takes, their
// LDS size, the launch grid, and dispatch to the compiled sizes (the kernel
// templates are in weights_ns_impl.h, instantiated by k_weights_ns_*.hip).
#include "weights_ns_impl.h"

namespace rbf {

RBF_NS_SIZES(RBF_NS_DECL)

namespace {

// A compiled size as one key: 1000 * MB + KB.
constexpr int ns_key(int mb, int kb) { return 1000 * mb + kb; }

const void *ns_kernel(int dim, int key) {
#define RBF_NS_K(D, MBB, KBB) \
    if (dim == D && key == ns_key(MBB, KBB)) return ns_kernel_##D##_##MBB##_##KBB();
    RBF_NS_SIZES(RBF_NS_K)
#undef RBF_NS_K
    return nullptr;
}

}  // namespace

// Compiled size for (n, M): the first (in the order of RBF_NS_SIZES) whose
// LU rows hold M entries and Cholesky rows K + 1, as the key 1000 MB + KB,
// with n + 1 rows on the workgroup's lanes; 0 if none (1D systems are small
// enough for the elimination paths).
int ns_bucket(int dim, int n, int M) {
    const int K = n - M;
    if (K < 1 || M < 2 || n + 1 > kLT) return 0;
#define RBF_NS_B(D, MBB, KBB) \
    if (dim == D && M <= MBB && K + 1 <= KBB) return ns_key(MBB, KBB);
    RBF_NS_SIZES(RBF_NS_B)
#undef RBF_NS_B
    return 0;
}

int ns_lds_doubles(int n, int M, int bucket) { return lu_layout(n, M, bucket / 1000, bucket % 1000).total; }

bool ns_fits(int dim, int n, int M, size_t lds_limit) {
    const int b = ns_bucket(dim, n, M);
    if (b == 0) return false;
    return (size_t)ns_lds_doubles(n, M, b) * sizeof(double) <= lds_limit;
}

// Workgroups of the null-space launch (every resident one at this LDS size), or 0.
int weights_ns_grid(int dim, int bucket, size_t lds_bytes) {
    const void *kern = ns_kernel(dim, bucket);
    if (!kern) return 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kLT, lds_bytes) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_weights_ns(hipStream_t s, int dim, int bucket, int64_t N, const double *xyz, const int32_t *sten,
                             const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                             const int8_t *type, const double *normals, double *w_out, DevStatus *status,
                             const void *items, int64_t nitems, int32_t *counter, size_t lds_bytes, int grid) {
    const void *kern = ns_kernel(dim, bucket);
    if (grid <= 0 || !kern) return hipErrorInvalidConfiguration;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
#define RBF_NS_L(D, MBB, KBB)                                                                                  \
    if (dim == D && bucket == ns_key(MBB, KBB))                                                                \
        return ns_launch_##D##_##MBB##_##KBB(s, grid, lds_bytes, N, xyz, sten, nrow, n_max, rows, mrow, type,     \
                                             normals, w_out, status, items, nitems, counter);
    RBF_NS_SIZES(RBF_NS_L)
#undef RBF_NS_L
    return hipErrorInvalidConfiguration;
}

}  // namespace rbf
