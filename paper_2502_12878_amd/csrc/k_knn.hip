// Exact n-nearest-neighbour supports (Sec. II: a node's support is its n
// nearest nodes, the node itself included) on a uniform cell grid.
//
// Binning: cell of a node = floor((x - lo)/edge) per axis, cells numbered x
// fastest; a counting sort puts node ids and their coordinates in cell order
// (ids ascending within a cell), so the nodes of a run of x-adjacent cells
// are one contiguous range.
//
// Query (one wavefront per node): take the block of cells within r cells of
// the query's cell, gather every node in it whose d2 is below the squared
// distance from the query to the nearest block face that is not a grid edge
// (minus a small safety margin), and grow r until at least n such nodes are
// found.  Every node outside that ball - inside or outside the block - is
// farther than all of them, so the n smallest keys (d2, id) among them are
// the exact answer.  Candidates are sorted by a bitonic network in LDS.
//
// d2 = (dx*dx + dy*dy) + dz*dz, dx = x_j - x_c, every operation rounded
// separately (this file is built with -ffp-contract=off), so keys and ties are
// bit-identical to the definition.
#include "rbf_internal.h"

namespace rbf {
namespace {

constexpr int kCap = 1024;      // candidate capacity per query
constexpr int kMaxRows = 1024;  // cell rows (y,z pairs) per block
constexpr int kMaxRing = 15;

__global__ __launch_bounds__(256) void k_bbox(int dim, int64_t N, const double *__restrict__ xyz,
                                              double *__restrict__ partials) {
    __shared__ double smin[3][256], smax[3][256];
    for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = INFINITY;
        smax[a][threadIdx.x] = -INFINITY;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < dim; ++a) {
            const double x = xyz[a * N + i];
            smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], x);
            smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], x);
        }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + w]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            partials[blockIdx.x * 6 + 2 * a] = smin[a][0];
            partials[blockIdx.x * 6 + 2 * a + 1] = smax[a][0];
        }
}

// Candidate capacity exceeded at query q: the status records EOVERFLOW and
// the lowest such node id (deterministic whatever order workgroups run in).
__device__ void report_overflow(DevStatus *st, int64_t q) {
    atomicCAS(&st->code, 0, (int)RBF_EOVERFLOW);
    atomicMin((unsigned long long *)&st->info, (unsigned long long)q);
}

__device__ __forceinline__ int cell_coord(double x, double lo, double edge, int nc) {
    double t = (x - lo) / edge;
    int c = (int)t;
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

__global__ void k_cell_of(CellGrid g, int64_t N, const double *__restrict__ xyz, int32_t *__restrict__ cell_of,
                          int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t c = 0, stride = 1;
    for (int a = 0; a < g.dim; ++a) {
        c += stride * cell_coord(xyz[a * N + i], g.lo[a], g.edge[a], g.nc[a]);
        stride *= g.nc[a];
    }
    cell_of[i] = (int32_t)c;
    atomicAdd(count + c, 1);
}

// Exclusive scan of n ints in three passes (block sums, scan of block sums by
// one workgroup, per-block scan plus offset).  out has n+1 entries.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(256) void k_scan_blocksum(int64_t n, const int32_t *__restrict__ in,
                                                       int32_t *__restrict__ bsum) {
    __shared__ int32_t s[256];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    int32_t a = 0;
    for (int q = 0; q < kScanBlock / 256; ++q) {
        const int64_t i = base + q * 256 + threadIdx.x;
        if (i < n) a += in[i];
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_scan_single(int64_t nb, int32_t *__restrict__ bsum) {
    __shared__ int32_t s[1024];
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < nb ? bsum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;  // exclusive
        const int32_t total = s[1023];
        __syncthreads();
        carry += total;
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(int64_t n, const int32_t *__restrict__ in,
                                                     const int32_t *__restrict__ boff, int32_t *__restrict__ out) {
    __shared__ int32_t s[1024];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int32_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = boff[blockIdx.x] + s[threadIdx.x] - v;
    if (i == n - 1) out[n] = boff[blockIdx.x] + s[threadIdx.x];
}

__global__ void k_scatter_cells(int64_t N, const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t c = cell_of[i];
    ids[start[c] + atomicAdd(cursor + c, 1)] = (int32_t)i;
}

// Sort each cell's ids ascending (cells hold a handful of nodes).
__global__ void k_sort_cells(int64_t ncells, const int32_t *__restrict__ start, int32_t *__restrict__ ids) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int32_t b = start[c], e = start[c + 1];
    for (int32_t p = b + 1; p < e; ++p) {
        const int32_t v = ids[p];
        int32_t q = p - 1;
        while (q >= b && ids[q] > v) {
            ids[q + 1] = ids[q];
            --q;
        }
        ids[q + 1] = v;
    }
}

// ids_by_cell also carries the coordinates in cell order: xyz_c[a][pos].
__global__ void k_coords_by_cell(int dim, int64_t N, const double *__restrict__ xyz, const int32_t *__restrict__ ids,
                                 double *__restrict__ xyz_c) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int32_t j = ids[p];
    for (int a = 0; a < dim; ++a) xyz_c[a * N + p] = xyz[a * N + j];
}

__device__ __forceinline__ double sq_dist(int dim, const double *xq, double x0, double x1, double x2) {
    double t = x0 - xq[0];
    double s = t * t;
    if (dim > 1) {
        t = x1 - xq[1];
        const double t2 = t * t;
        s = s + t2;
    }
    if (dim > 2) {
        t = x2 - xq[2];
        const double t2 = t * t;
        s = s + t2;
    }
    return s;
}

__device__ __forceinline__ bool key_less(unsigned long long da, int32_t ia, unsigned long long db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

// One 64-thread workgroup per query node.
__global__ __launch_bounds__(64) void k_knn(CellGrid g, int64_t N, const double *__restrict__ xyz,
                                            const double *__restrict__ xyz_c, const int32_t *__restrict__ cell_of,
                                            const int32_t *__restrict__ cstart, const int32_t *__restrict__ ids_c,
                                            int32_t n_uniform, const int16_t *__restrict__ n_per_node, int32_t n_max,
                                            double ball_coef, double margin, int32_t *__restrict__ sten,
                                            int16_t *__restrict__ nrow_out, const int8_t *__restrict__ type,
                                            DevStatus *status) {
    __shared__ unsigned long long kd[kCap];
    __shared__ int32_t kid[kCap];
    __shared__ int32_t row_p0[kMaxRows];
    __shared__ int32_t row_off[kMaxRows + 1];
    __shared__ int32_t s_count;

    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x;
    const int dim = g.dim;
    const int n = n_per_node ? (int)n_per_node[q] : n_uniform;
    // a Neumann node (type 2) draws its support from itself and interior nodes
    const bool interior_only = type[q] == 2;
    double xq[3] = {0.0, 0.0, 0.0};
    int qc[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        xq[a] = xyz[a * N + q];
        qc[a] = cell_coord(xq[a], g.lo[a], g.edge[a], g.nc[a]);
    }
    double min_edge = g.edge[0];
    for (int a = 1; a < dim; ++a) min_edge = fmin(min_edge, g.edge[a]);
    // radius of a ball expected to hold n nodes, in cells
    const double rn = dim == 1 ? n * ball_coef : (dim == 2 ? sqrt(n * ball_coef) : cbrt(n * ball_coef));
    int r = (int)(rn / min_edge) + 1;
    if (r < 1) r = 1;

    int count = 0;
    for (;;) {
        int lo_c[3] = {0, 0, 0}, hi_c[3] = {0, 0, 0};
        double bound = INFINITY;
        bool whole = true;
        for (int a = 0; a < dim; ++a) {
            lo_c[a] = qc[a] - r;
            hi_c[a] = qc[a] + r;
            if (lo_c[a] > 0) {
                bound = fmin(bound, xq[a] - (g.lo[a] + lo_c[a] * g.edge[a]));
                whole = false;
            } else {
                lo_c[a] = 0;
            }
            if (hi_c[a] < g.nc[a] - 1) {
                bound = fmin(bound, (g.lo[a] + (hi_c[a] + 1) * g.edge[a]) - xq[a]);
                whole = false;
            } else {
                hi_c[a] = g.nc[a] - 1;
            }
        }
        double bound2 = INFINITY;
        if (!whole) {
            bound -= margin;
            bound2 = bound > 0.0 ? bound * bound : 0.0;
        }
        // rows of x-adjacent cells in the block
        const int ny = dim > 1 ? hi_c[1] - lo_c[1] + 1 : 1;
        const int nz = dim > 2 ? hi_c[2] - lo_c[2] + 1 : 1;
        const int nrows = ny * nz;
        if (nrows > kMaxRows || r > kMaxRing) {
            if (lane == 0) report_overflow(status, q);
            return;
        }
        for (int t = lane; t < nrows; t += 64) {
            const int cy = (dim > 1 ? lo_c[1] + t % ny : 0);
            const int cz = (dim > 2 ? lo_c[2] + t / ny : 0);
            const int64_t rowbase = ((int64_t)cz * g.nc[1] + cy) * (int64_t)g.nc[0];
            const int32_t p0 = cstart[rowbase + lo_c[0]];
            const int32_t p1 = cstart[rowbase + hi_c[0] + 1];
            row_p0[t] = p0;
            row_off[t + 1] = p1 - p0;
        }
        if (lane == 0) {
            row_off[0] = 0;
            s_count = 0;
        }
        __syncthreads();
        if (lane == 0)
            for (int t = 0; t < nrows; ++t) row_off[t + 1] += row_off[t];
        __syncthreads();
        const int total = row_off[nrows];
        for (int t = lane; t < total; t += 64) {
            int lo = 0, hi = nrows - 1;  // row containing candidate t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (row_off[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int64_t p = row_p0[lo] + (t - row_off[lo]);
            const double d2 = sq_dist(dim, xq, xyz_c[p], dim > 1 ? xyz_c[N + p] : 0.0,
                                      dim > 2 ? xyz_c[2 * N + p] : 0.0);
            if (d2 < bound2) {
                const int32_t j = ids_c[p];
                if (!interior_only || j == q || type[j] == 0) {
                    const int slot = atomicAdd(&s_count, 1);
                    if (slot < kCap) {
                        kd[slot] = (unsigned long long)__double_as_longlong(d2);
                        kid[slot] = j;
                    }
                }
            }
        }
        __syncthreads();
        count = s_count;
        __syncthreads();
        if (count > kCap) {
            if (lane == 0) report_overflow(status, q);
            return;
        }
        if (count >= n) break;
        ++r;
    }

    // bitonic sort of the candidates by (d2, id)
    int P = 1;
    while (P < count) P <<= 1;
    for (int t = count + lane; t < P; t += 64) {
        kd[t] = ~0ull;
        kid[t] = 0x7fffffff;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P; t += 64) {
                const int o = t ^ j;
                if (o > t) {
                    const bool up = (t & k) == 0;
                    const unsigned long long da = kd[t], db = kd[o];
                    const int32_t ia = kid[t], ib = kid[o];
                    const bool sw = up ? key_less(db, ib, da, ia) : key_less(da, ia, db, ib);
                    if (sw) {
                        kd[t] = db;
                        kd[o] = da;
                        kid[t] = ib;
                        kid[o] = ia;
                    }
                }
            }
            __syncthreads();
        }
    }
    int32_t *out = sten + q * (int64_t)n_max;
    for (int t = lane; t < n_max; t += 64) out[t] = t < n ? kid[t] : -1;
    if (lane == 0) nrow_out[q] = (int16_t)n;
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_bbox_partials(hipStream_t s, int dim, int64_t N, const double *xyz, double *partials, int nblk) {
    hipLaunchKernelGGL(k_bbox, dim3(nblk), dim3(256), 0, s, dim, N, xyz, partials);
    return hipGetLastError();
}

hipError_t launch_bin_nodes(hipStream_t s, const CellGrid &g, int64_t N, const double *xyz, int32_t *cell_of,
                            int32_t *cell_count, int32_t *cell_start, int32_t *ids_by_cell, int32_t *cursor,
                            int32_t *scan_tmp) {
    hipError_t e;
    hipLaunchKernelGGL(k_cell_of, dim3(grid1d(N, 256)), dim3(256), 0, s, g, N, xyz, cell_of, cell_count);
    const int64_t nb = (g.ncells + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_blocksum, dim3((unsigned)nb), dim3(256), 0, s, g.ncells, cell_count, scan_tmp);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, nb, scan_tmp);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(1024), 0, s, g.ncells, cell_count, scan_tmp,
                       cell_start);
    hipLaunchKernelGGL(k_scatter_cells, dim3(grid1d(N, 256)), dim3(256), 0, s, N, cell_of, cell_start, cursor,
                       ids_by_cell);
    hipLaunchKernelGGL(k_sort_cells, dim3(grid1d(g.ncells, 256)), dim3(256), 0, s, g.ncells, cell_start,
                       ids_by_cell);
    e = hipGetLastError();
    return e;
}

hipError_t launch_coords_by_cell(hipStream_t s, int dim, int64_t N, const double *xyz, const int32_t *ids,
                                 double *xyz_c) {
    hipLaunchKernelGGL(k_coords_by_cell, dim3(grid1d(N, 256)), dim3(256), 0, s, dim, N, xyz, ids, xyz_c);
    return hipGetLastError();
}

hipError_t launch_knn_query(hipStream_t s, const CellGrid &g, int64_t N, const double *xyz, const double *xyz_c,
                            const int32_t *cell_of, const int32_t *cell_start, const int32_t *ids_by_cell,
                            int32_t n_uniform, const int16_t *n_per_node, int32_t n_max, double ball_coef,
                            double margin, int32_t *sten, int16_t *nrow_out, const int8_t *type,
                            DevStatus *status) {
    hipLaunchKernelGGL(k_knn, dim3((unsigned)N), dim3(64), 0, s, g, N, xyz, xyz_c, cell_of, cell_start, ids_by_cell,
                       n_uniform, n_per_node, n_max, ball_coef, margin, sten, nrow_out, type, status);
    return hipGetLastError();
}

}  // namespace rbf
