// Transposed operator for the adjoint sweep.  The adjoint of the explicit
// step needs (L_II^T v)_c = sum over interior rows r with c in the support of
// r of w_rc v_r.  Instead of scattering with atomics every step, the transpose
// is built once (counting sort of the support entries by column, each
// column's list sorted by row so the result is deterministic) and packed in
// the same sliced layout as the forward operator; an adjoint step is then a
// gather sweep with the same memory behaviour as a forward step.
#include "rbf_internal.h"

namespace rbf {
namespace {

// Thread per (canonical row R, entry k): count entries per interior column.
__global__ void k_tcount(int64_t N, int32_t n_max, int64_t N_int, const int8_t *__restrict__ type,
                         const int32_t *__restrict__ iperm, const int32_t *__restrict__ sten,
                         const int16_t *__restrict__ nrow, int32_t *__restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = t / n_max;
    const int k = (int)(t - R * n_max);
    if (R >= N || type[R] != 0 || k >= nrow[R]) return;
    const int32_t c = iperm[sten[R * n_max + k]];
    if (c < N_int) atomicAdd(cnt + c, 1);
}

// Same mapping: place (internal row, weight) into the column's segment.
__global__ void k_tfill(int64_t N, int32_t n_max, int64_t N_int, const int8_t *__restrict__ type,
                        const int32_t *__restrict__ iperm, const int32_t *__restrict__ sten,
                        const int16_t *__restrict__ nrow, const double *__restrict__ w_can,
                        const int64_t *__restrict__ start, int32_t *__restrict__ cursor, int32_t *__restrict__ rows_t,
                        double *__restrict__ w_t) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = t / n_max;
    const int k = (int)(t - R * n_max);
    if (R >= N || type[R] != 0 || k >= nrow[R]) return;
    const int32_t c = iperm[sten[R * n_max + k]];
    if (c >= N_int) return;
    const int64_t pos = start[c] + atomicAdd(cursor + c, 1);
    rows_t[pos] = iperm[R];
    w_t[pos] = w_can[R * n_max + k];
}

__device__ __forceinline__ int64_t pair_pos(int64_t base, int k, int lane) {
    return base + (int64_t)(k >> 1) * (2 * kSlice) + 2 * lane + (k & 1);
}

// Thread per lane of every slice: the lane's column c (lmeta: lanes ordered
// by decreasing row length; null: c = 64 s + lane) has its entries sorted by
// row, then written into the sliced layout; padding entries point at c itself
// with weight 0.
__global__ void k_tpack(int64_t N_int, int64_t nslices, const int64_t *__restrict__ start,
                        int32_t *__restrict__ rows_t, double *__restrict__ w_t, const int64_t *__restrict__ slice_ptr,
                        const int32_t *__restrict__ slice_len, const uint16_t *__restrict__ lmeta,
                        int32_t *__restrict__ idx, double *__restrict__ w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslices * kSlice) return;
    const int64_t s = t / kSlice;
    const int lane = (int)(t - s * kSlice);
    const int64_t c = lmeta ? s * kSlice + (lmeta[t] & (kSlice - 1)) : t;
    const int len = slice_len[s];
    const int64_t base = slice_ptr[s];
    int cnt = 0;
    if (c < N_int) {
        const int64_t b = start[c];
        cnt = (int)(start[c + 1] - b);
        for (int p = 1; p < cnt; ++p) {  // insertion sort by row id
            const int32_t r = rows_t[b + p];
            const double ww = w_t[b + p];
            int q = p - 1;
            while (q >= 0 && rows_t[b + q] > r) {
                rows_t[b + q + 1] = rows_t[b + q];
                w_t[b + q + 1] = w_t[b + q];
                --q;
            }
            rows_t[b + q + 1] = r;
            w_t[b + q + 1] = ww;
        }
        for (int k = 0; k < cnt; ++k) {
            idx[pair_pos(base, k, lane)] = rows_t[b + k];
            w[pair_pos(base, k, lane)] = w_t[b + k];
        }
    }
    const int32_t self = c < N_int ? (int32_t)c : 0;
    for (int k = cnt; k < len; ++k) {
        idx[pair_pos(base, k, lane)] = self;
        w[pair_pos(base, k, lane)] = 0.0;
    }
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_tcount(hipStream_t s, int64_t N, int32_t n_max, int64_t N_int, const int8_t *type,
                         const int32_t *iperm, const int32_t *sten, const int16_t *nrow, int32_t *cnt) {
    const int64_t total = N * (int64_t)n_max;
    hipLaunchKernelGGL(k_tcount, dim3(grid1d(total, 256)), dim3(256), 0, s, N, n_max, N_int, type, iperm, sten, nrow,
                       cnt);
    return hipGetLastError();
}

hipError_t launch_tfill(hipStream_t s, int64_t N, int32_t n_max, int64_t N_int, const int8_t *type,
                        const int32_t *iperm, const int32_t *sten, const int16_t *nrow, const double *w_can,
                        const int64_t *start, int32_t *cursor, int32_t *rows_t, double *w_t) {
    const int64_t total = N * (int64_t)n_max;
    hipLaunchKernelGGL(k_tfill, dim3(grid1d(total, 256)), dim3(256), 0, s, N, n_max, N_int, type, iperm, sten, nrow,
                       w_can, start, cursor, rows_t, w_t);
    return hipGetLastError();
}

hipError_t launch_tpack(hipStream_t s, int64_t N_int, const int64_t *start, int32_t *rows_t, double *w_t,
                        const Ell &e) {
    if (!e.nslices) return hipSuccess;
    hipLaunchKernelGGL(k_tpack, dim3(grid1d(e.nslices * kSlice, 256)), dim3(256), 0, s, N_int, e.nslices, start,
                       rows_t, w_t, e.slice_ptr, e.slice_len, e.lmeta, e.idx, e.w);
    return hipGetLastError();
}

}  // namespace rbf
