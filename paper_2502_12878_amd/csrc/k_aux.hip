// Kernels around the sweeps: the packed-operator builder and its 16-bit
// column codes, the Neumann boundary update (Sec. II-C, enforcing the Neumann
// condition before each step), the transposed scatter and update of the
// adjoint, error norms and reductions, and permutes and fills between the
// caller's node order and the internal one.
#include "row_dot.h"

namespace rbf {
namespace {

// Transpose scatter: out[c] += w_rc v_r for interior rows r and interior c.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_transpose_scatter(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t nslices, int64_t N_int, const double *__restrict__ v,
    double *__restrict__ out, int layout) {
    const int64_t slice = (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int64_t row = slice * kSlice + lane;
    if (row >= N_int) return;
    const double vr = v[row];
    const int64_t base = slice_ptr[slice];
    const int len = slice_len[slice];
    for (int k = 0; k < len; ++k) {
        const int32_t c = ld_stream(idx + ell_pos(layout, base, k, lane));
        const double ww = ld_stream(w + ell_pos(layout, base, k, lane));
        if (c < N_int && ww != 0.0) unsafeAtomicAdd(out + c, ww * vr);
    }
}

__global__ void k_adjoint_update(int64_t N_int, double dt, double *__restrict__ lam, double *__restrict__ acc,
                                 double *__restrict__ tmp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N_int) return;
    const double l = lam[i] + dt * tmp[i];
    lam[i] = l;
    acc[i] += l;
    tmp[i] = 0.0;
}

__global__ void k_add_correction(int64_t N_int, double *__restrict__ u, const float *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N_int) u[i] += (double)e[i];
}

// max |u - uref| into slot and per-block partial sums of |u - uref|.
__global__ __launch_bounds__(256) void k_err_norm(int64_t N, const double *__restrict__ u,
                                                  const double *__restrict__ uref, double *__restrict__ partials,
                                                  unsigned long long *max_slot) {
    __shared__ double ssum[4];
    unsigned long long bits = 0;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = fabs(u[i] - uref[i]);
        const unsigned long long b = (unsigned long long)__double_as_longlong(d);
        bits = b > bits ? b : bits;
        s += d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) ssum[threadIdx.x >> 6] = s;
    block_max_to_slot<4>(bits, max_slot);  // contains __syncthreads
    if (threadIdx.x == 0) partials[blockIdx.x] = (ssum[0] + ssum[1]) + (ssum[2] + ssum[3]);
}

__global__ void k_sum_partials(const double *__restrict__ p, int n, double *out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += p[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Packed-operator builder: thread per (internal row, slot k < kmax).  Entry
// k of canonical row r goes to the slot of its rank among the row's internal
// column ids; slots past the row's size hold the row itself with weight 0;
// rows past N_int (tail of the last slice) hold column 0 with weight 0.
// The packed rows are internal rows row0 .. row0 + nrows - 1.  With
// zero_self, a row's own entry keeps its slot with weight 0 and its weight is
// written to wself[i] instead (the Neumann rows, solved for their own value).
// The internal column ids of the rows a workgroup touches are staged in LDS
// first (a 256-thread block spans at most 256 / kmax + 2 rows), so each rank
// is counted from LDS instead of re-reading the row's ids from memory.
constexpr int kPackThreads = 256;

__global__ __launch_bounds__(kPackThreads) void k_pack_ell(
    int64_t row0, int64_t nrows, int32_t n_max, int32_t kmax, int64_t nslices, int layout,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm, const int32_t *__restrict__ sten,
    const int16_t *__restrict__ nrow, const double *__restrict__ w_can, const int64_t *__restrict__ slice_ptr,
    const int32_t *__restrict__ slice_len, int32_t *__restrict__ idx, double *__restrict__ w, float *__restrict__ w32,
    double *__restrict__ wself, int32_t *__restrict__ foreign) {
    extern __shared__ int32_t pk_cols[];  // [rows of this block][kmax]
    const int64_t t0 = (int64_t)blockIdx.x * kPackThreads;
    const int64_t t = t0 + threadIdx.x;
    const int64_t irow0 = t0 / kmax;
    const int64_t irows = nslices * kSlice;
    const int nblk = (int)((t0 + kPackThreads - 1) / kmax - irow0 + 1);
    // stage: entry q of block row b holds the internal id of support entry q
    for (int e = threadIdx.x; e < nblk * kmax; e += kPackThreads) {
        const int b = e / kmax, q = e - b * kmax;
        const int64_t ii = irow0 + b;
        int32_t v = -1;
        if (ii < nrows && ii < irows) {
            const int64_t r = perm[row0 + ii];
            if (q < nrow[r]) v = iperm[sten[r * (int64_t)n_max + q]];
        }
        pk_cols[e] = v;
    }
    __syncthreads();
    const int64_t i = t / kmax;
    const int k = (int)(t - i * kmax);
    if (i >= irows) return;
    const int64_t s = i / kSlice;
    const int lane = (int)(i - s * kSlice);
    const int len = slice_len[s];
    if (k >= len) return;
    const int64_t base = slice_ptr[s];
    const int64_t gi = row0 + i;
    int32_t col = 0;
    double wk = 0.0;
    int slot = k;
    if (i < nrows) {
        const int64_t r = perm[gi];
        const int n = nrow[r];
        if (k >= n) {
            col = (int32_t)gi;
        } else {
            const int32_t *cr = pk_cols + (i - irow0) * kmax;
            col = cr[k];
            int rank = 0;
            for (int q = 0; q < n; ++q) rank += (cr[q] < col) ? 1 : 0;
            slot = rank;
            wk = w_can[r * (int64_t)n_max + k];
            if (wself && col == gi) {
                wself[i] = wk;
                wk = 0.0;
            }
            // a support entry that is neither interior (internal id < row0)
            // nor the row itself
            if (foreign && col >= row0 && col != gi) *foreign = 1;
        }
    }
    const int64_t pos = ell_pos(layout, base, slot, lane);
    idx[pos] = col;
    w[pos] = wk;
    if (w32) w32[pos] = (float)wk;
}

// Neumann update, first half: nb[j] = (g_j - sum_{k != self} w_jk u_k) / w_jj
// for Neumann row j (internal row N_int + j), all from the current iterate.
// The Neumann rows are few (one face layer), so each slice gets a workgroup
// of kNeuWaves wavefronts: wavefront q sums the q-th part of the slice's
// entries, loading index and weight pairs as vectors and issuing a batch of
// them before its gathers, and the partial sums are added in a fixed order.
// With u_cur / u_next (supports of interior nodes and the row itself only, so
// no Neumann row reads another's value) the new value goes straight into both
// iterate buffers.  With g null, nb[N_int + j] = (D u)_j instead (the
// derivative).  The update is bound by its chain of dependent loads, so the
// chain is kept short: with ulen > 0 (every slice that long) the slice's
// place is computed instead of read, and the row's own values (g, its own
// weight) are requested before the stream loads.
constexpr int kNeuWaves = 8;
constexpr int kNeuBatch = 8;  // entry pairs per batch

template <int LAYOUT>
__global__ __launch_bounds__(kNeuWaves * 64) void k_neumann_eval(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t N_int, int64_t N_neu, const double *__restrict__ wself,
    const double *__restrict__ g, const double *u, double *__restrict__ nb, double *u_cur, double *u_next,
    int ulen) {
    __shared__ double part[kNeuWaves][kSlice];
    const int64_t slice = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t jr = slice * kSlice + lane;
    double own = 0.0, ws = 1.0;  // g (or u) and the own weight of row jr, requested first
    if (wave == 0 && jr < N_neu) {
        ws = wself[jr];
        own = g ? g[N_int + jr] : u[N_int + jr];
    }
    const int len = ulen > 0 ? ulen : slice_len[slice];
    const int64_t base = ulen > 0 ? slice * (int64_t)ulen * kSlice : slice_ptr[slice];
    double acc = 0.0;
    if (LAYOUT == 1) {
        // entry pairs as vectors (len is even): wavefront q takes pairs [p0, p1)
        const int npair = len >> 1;
        const int chunk = (npair + kNeuWaves - 1) / kNeuWaves;
        const int p0 = min(npair, wave * chunk), p1 = min(npair, p0 + chunk);
        const i32x2 *ip = (const i32x2 *)(idx + base) + lane;
        const f64x2 *wp = (const f64x2 *)(w + base) + lane;
        for (int pb = p0; pb < p1; pb += kNeuBatch) {
            i32x2 j[kNeuBatch];
            f64x2 ww[kNeuBatch];
#pragma unroll
            for (int q = 0; q < kNeuBatch; ++q) {
                const int pq = pb + q < p1 ? pb + q : p0;
                j[q] = ld_stream(ip + (int64_t)pq * kSlice);
                ww[q] = ld_stream(wp + (int64_t)pq * kSlice);
            }
            double xx[2 * kNeuBatch];
#pragma unroll
            for (int q = 0; q < kNeuBatch; ++q) {
                xx[2 * q] = u[j[q].x];
                xx[2 * q + 1] = u[j[q].y];
            }
#pragma unroll
            for (int q = 0; q < kNeuBatch; ++q)
                if (pb + q < p1) {
                    acc = fma(ww[q].x, xx[2 * q], acc);
                    acc = fma(ww[q].y, xx[2 * q + 1], acc);
                }
        }
    } else {
        const int chunk = (len + kNeuWaves - 1) / kNeuWaves;
        const int k0 = min(len, wave * chunk), k1 = min(len, k0 + chunk);
        for (int k = k0; k < k1; ++k) {
            const int64_t pos = ell_pos(0, base, k, lane);
            acc = fma(ld_stream(w + pos), u[ld_stream(idx + pos)], acc);
        }
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave) return;
    acc = 0.0;
#pragma unroll
    for (int q = 0; q < kNeuWaves; ++q) acc += part[q][lane];
    if (jr >= N_neu) return;
    if (g) {
        const double v = (own - acc) / ws;
        if (u_cur) {
            u_cur[N_int + jr] = v;
            u_next[N_int + jr] = v;
        } else {
            nb[jr] = v;
        }
    } else {
        nb[N_int + jr] = acc + ws * own;
    }
}

// near[r] = 1 for an interior row whose support holds a Neumann node, else 0.
__global__ void k_flag_near(int64_t N, int32_t n_max, const int32_t *__restrict__ sten,
                            const int16_t *__restrict__ nrow, const int8_t *__restrict__ type,
                            int8_t *__restrict__ near) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    int8_t f = 0;
    if (type[r] == 0) {
        const int n = nrow[r];
        for (int k = 0; k < n; ++k) f |= type[sten[r * (int64_t)n_max + k]] == 2;
    }
    near[r] = f;
}

// Neumann update, second half: store the new values in both iterate buffers.
__global__ void k_neumann_store(int64_t N_int, int64_t N_neu, const double *__restrict__ nb, double *__restrict__ ua,
                                double *__restrict__ ub) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N_neu) return;
    ua[N_int + j] = nb[j];
    ub[N_int + j] = nb[j];
}

__global__ void k_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src,
                         double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}
__global__ void k_scatter(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}
template <typename T>
__global__ void k_fill(int64_t n, T v, T *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_scale_interior(int64_t N, int64_t N_int, double a, const double *__restrict__ src,
                                 double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[i] = i < N_int ? a * src[i] : 0.0;
}

}  // namespace

hipError_t launch_pack_ell(hipStream_t s, int64_t row0, int64_t nrows, int32_t n_max, const int32_t *perm,
                           const int32_t *iperm, const int32_t *sten, const int16_t *nrow, const double *w_can,
                           const Ell &e, double *wself, int32_t *foreign) {
    const int32_t kmax = e.max_len;
    const int64_t total = e.nslices * kSlice * (int64_t)kmax;
    if (!total) return hipSuccess;
    const size_t lds = sizeof(int32_t) * (size_t)(kPackThreads / kmax + 2) * kmax;
    hipLaunchKernelGGL(k_pack_ell, dim3(grid1d(total, kPackThreads)), dim3(kPackThreads), lds, s, row0, nrows, n_max,
                       kmax, e.nslices, e.layout, perm, iperm, sten, nrow, w_can, e.slice_ptr, e.slice_len, e.idx,
                       e.w, e.w32, wself, foreign);
    return hipGetLastError();
}

// Segment codes of one slice per workgroup (one wavefront): the distinct
// aligned 4096-id blocks touched by any entry of the slice (padding entries
// included, so every stored column stays encodable) are found in ascending
// order by repeated wavefront minima; with at most kSegs of them the slice
// gets codes (cmode 1), else it keeps only its 32-bit ids (cmode 0).  The
// block numbers of a slice are staged in LDS when its rows hold at most
// kMaxSupport entries (every forward operator); longer slices (rows of the
// transposed operator, whose length is a column's in-degree and has no such
// bound) read them from the id stream on every pass.
__global__ __launch_bounds__(64) void k_encode_codes(const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ slice_len,
                                                     const int32_t *__restrict__ idx, int64_t nslices,
                                                     const int64_t *__restrict__ cptr, uint16_t *__restrict__ code,
                                                     int32_t *__restrict__ segbase, int8_t *__restrict__ cmode,
                                                     const double *__restrict__ w, float *__restrict__ w32q) {
    __shared__ uint16_t blk[kMaxSupport * kSlice];
    __shared__ int32_t list[kSegs];
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int len = slice_len[s];
    const int64_t base = slice_ptr[s];
    const bool staged = len <= kMaxSupport;
    if (staged)
        for (int k = 0; k < len; ++k) blk[k * kSlice + lane] = (uint16_t)(idx[ell_pos(1, base, k, lane)] >> 12);
    __syncthreads();
    int cnt = 0, cur = -1;
    bool over = false;
    for (int it = 0; it <= kSegs; ++it) {
        int mn = 0x7fffffff;
        for (int k = 0; k < len; ++k) {
            const int v = staged ? (int)blk[k * kSlice + lane] : (int)(idx[ell_pos(1, base, k, lane)] >> 12);
            if (v > cur && v < mn) mn = v;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const int o = __shfl_xor(mn, off, 64);
            mn = o < mn ? o : mn;
        }
        if (mn == 0x7fffffff) break;
        if (cnt == kSegs) {
            over = true;
            break;
        }
        if (lane == 0) list[cnt] = mn;
        ++cnt;
        cur = mn;
    }
    __syncthreads();
    if (over) {
        if (lane == 0) cmode[s] = 0;
        return;
    }
    if (lane < kSegs) segbase[s * kSegs + lane] = (lane < cnt ? list[lane] : list[0]) << 12;
    if (lane == 0) cmode[s] = 1;
    const int len4 = (len + 3) & ~3;
    uint16_t *out = code + cptr[s];
    for (int k = 0; k < len4; ++k) {
        uint16_t c = 0;
        if (k < len) {
            const int32_t col = idx[ell_pos(1, base, k, lane)];
            const int b = col >> 12;
            int seg = 0;
            while (seg + 1 < cnt && list[seg] != b) ++seg;
            c = (uint16_t)((seg << 12) | (col & (kSegSpan - 1)));
        }
        const int64_t at = (int64_t)(k >> 2) * (4 * kSlice) + 4 * lane + (k & 3);
        out[at] = c;
        // FP32 weights in the same layout (rounded as the paired FP32 copy)
        if (w32q) w32q[cptr[s] + at] = k < len ? (float)w[ell_pos(1, base, k, lane)] : 0.0f;
    }
}

// Every coded slot decoded back to its column and compared with the 32-bit
// id it stands for; a slice with any difference loses its codes (cmode 0:
// the sweeps read its 32-bit ids) and is counted in *bad.  One wavefront per
// slice.
__global__ __launch_bounds__(256) void k_check_codes(const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ slice_len,
                                                     const int32_t *__restrict__ idx, int64_t nslices,
                                                     const int64_t *__restrict__ cptr,
                                                     const uint16_t *__restrict__ code,
                                                     const int32_t *__restrict__ segbase, int8_t *__restrict__ cmode,
                                                     unsigned long long *bad) {
    const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices || !cmode[s]) return;
    const int len = slice_len[s];
    const int64_t base = slice_ptr[s];
    const uint16_t *in = code + cptr[s];
    bool ok = true;
    for (int k = 0; k < len; ++k) {
        const uint32_t c = in[(int64_t)(k >> 2) * (4 * kSlice) + 4 * lane + (k & 3)];
        const int32_t col = segbase[s * kSegs + (c >> 12)] + (int32_t)(c & (kSegSpan - 1));
        ok = ok && col == idx[ell_pos(1, base, k, lane)];
    }
    if (__all(ok)) return;
    if (lane == 0) {
        cmode[s] = 0;
        atomicAdd(bad, 1ull);
    }
}

hipError_t launch_flag_near(hipStream_t s, int64_t N, int32_t n_max, const int32_t *sten, const int16_t *nrow,
                            const int8_t *type, int8_t *near) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flag_near, dim3(grid1d(N, 256)), dim3(256), 0, s, N, n_max, sten, nrow, type, near);
    return hipGetLastError();
}

hipError_t launch_encode_codes(hipStream_t s, const Ell &e) {
    if (!e.nslices || e.layout != 1 || !e.code) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_encode_codes, dim3((unsigned)e.nslices), dim3(kSlice), 0, s, e.slice_ptr, e.slice_len, e.idx,
                       e.nslices, e.cptr, e.code, e.segbase, e.cmode, e.w, e.w32q);
    return hipGetLastError();
}

hipError_t launch_check_codes(hipStream_t s, const Ell &e, unsigned long long *bad) {
    if (!e.nslices || e.layout != 1 || !e.code) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_check_codes, dim3(grid1d(e.nslices, 4)), dim3(256), 0, s, e.slice_ptr, e.slice_len, e.idx,
                       e.nslices, e.cptr, e.code, e.segbase, e.cmode, bad);
    return hipGetLastError();
}

// The Neumann update of one step (evaluate all new boundary values from the
// current iterate, then store them in both buffers).
hipError_t launch_neumann_update(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                 const double *g, double *u_cur, double *u_next, double *nb, bool direct) {
    if (!e.nslices) return hipSuccess;
    const dim3 grid((unsigned)e.nslices);
    double *uc = direct ? u_cur : nullptr, *un = direct ? u_next : nullptr;
    if (e.layout)
        hipLaunchKernelGGL(k_neumann_eval<1>, grid, dim3(kNeuWaves * 64), 0, s, e.slice_ptr, e.slice_len, e.idx, e.w, N_int,
                           N_neu, wself, g, u_cur, nb, uc, un, e.uniform_len);
    else
        hipLaunchKernelGGL(k_neumann_eval<0>, grid, dim3(kNeuWaves * 64), 0, s, e.slice_ptr, e.slice_len, e.idx, e.w, N_int,
                           N_neu, wself, g, u_cur, nb, uc, un, e.uniform_len);
    if (!direct)
        hipLaunchKernelGGL(k_neumann_store, dim3(grid1d(N_neu, 256)), dim3(256), 0, s, N_int, N_neu, nb, u_cur,
                           u_next);
    return hipGetLastError();
}

// out[N_int + j] = (D u) at Neumann row j (its normal-derivative stencil).
hipError_t launch_neumann_apply(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                const double *u, double *out) {
    if (!e.nslices) return hipSuccess;
    const dim3 grid((unsigned)e.nslices);
    if (e.layout)
        hipLaunchKernelGGL(k_neumann_eval<1>, grid, dim3(kNeuWaves * 64), 0, s, e.slice_ptr, e.slice_len, e.idx, e.w, N_int,
                           N_neu, wself, nullptr, u, out, nullptr, nullptr, e.uniform_len);
    else
        hipLaunchKernelGGL(k_neumann_eval<0>, grid, dim3(kNeuWaves * 64), 0, s, e.slice_ptr, e.slice_len, e.idx, e.w, N_int,
                           N_neu, wself, nullptr, u, out, nullptr, nullptr, e.uniform_len);
    return hipGetLastError();
}

hipError_t launch_add_correction(hipStream_t s, int64_t N_int, double *u, const float *e) {
    if (N_int <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_correction, dim3(grid1d(N_int, 256)), dim3(256), 0, s, N_int, u, e);
    return hipGetLastError();
}

hipError_t launch_err_norm(hipStream_t s, int64_t N, const double *u, const double *uref, double *partials, int nblk,
                           unsigned long long *max_slot) {
    hipLaunchKernelGGL(k_err_norm, dim3(nblk), dim3(256), 0, s, N, u, uref, partials, max_slot);
    return hipGetLastError();
}

hipError_t launch_sum_partials(hipStream_t s, const double *partials, int n, double *out) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_transpose_scatter(hipStream_t s, const Ell &e, int64_t N_int, const double *v, double *out) {
    if (!e.nslices) return hipSuccess;
    hipLaunchKernelGGL((k_transpose_scatter<4>), dim3(grid1d(e.nslices, 4)), dim3(256), 0, s, e.slice_ptr,
                       e.slice_len, e.idx, e.w, e.nslices, N_int, v, out, e.layout);
    return hipGetLastError();
}

hipError_t launch_adjoint_update(hipStream_t s, int64_t N_int, double dt, double *lam, double *acc, double *tmp) {
    if (N_int <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_update, dim3(grid1d(N_int, 256)), dim3(256), 0, s, N_int, dt, lam, acc, tmp);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid1d(n, 256)), dim3(256), 0, s, n, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(grid1d(n, 256)), dim3(256), 0, s, n, perm, src, dst);
    return hipGetLastError();
}

// *out = the double whose IEEE bits a max-reduction slot holds.
__global__ void k_slot_to_double(const unsigned long long *__restrict__ slot, double *__restrict__ out) {
    if (threadIdx.x == 0) *out = __longlong_as_double((long long)*slot);
}

hipError_t launch_slot_to_double(hipStream_t s, const unsigned long long *slot, double *out) {
    hipLaunchKernelGGL(k_slot_to_double, dim3(1), dim3(64), 0, s, slot, out);
    return hipGetLastError();
}

hipError_t launch_fill_f64(hipStream_t s, int64_t n, double v, double *p) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3(grid1d(n, 256)), dim3(256), 0, s, n, v, p);
    return hipGetLastError();
}
hipError_t launch_fill_f32(hipStream_t s, int64_t n, float v, float *p) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(grid1d(n, 256)), dim3(256), 0, s, n, v, p);
    return hipGetLastError();
}
hipError_t launch_fill_u64(hipStream_t s, int64_t n, unsigned long long v, unsigned long long *p) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid1d(n, 256)), dim3(256), 0, s, n, v, p);
    return hipGetLastError();
}
hipError_t launch_scale_interior(hipStream_t s, int64_t N, int64_t N_int, double a, const double *src, double *dst) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_interior, dim3(grid1d(N, 256)), dim3(256), 0, s, N, N_int, a, src, dst);
    return hipGetLastError();
}

}  // namespace rbf
