// Sweep kernels of the explicit RBF-FD iteration (Sec. II-C, the Jacobi step
// u <- u + dt (L_h u - f) with L_h u at a node a weighted sum over its support,
// Sec. II).  All of them read the packed operator (sliced ELL, 64 rows per
// slice, entries of a slice stored entry-major so that one wavefront reads
// contiguous 256 B index and 512 B weight lines per support entry).
//
// The sweep is bound by HBM bandwidth: per interior node-update it must move
// 4n bytes of indices, 8n of weights, and 24 of f, u and u_new.  Index and
// weight streams are read once per sweep and use non-temporal loads so that
// the gathered solution vector stays in L2 / Infinity Cache.  Rows of a slice
// are spatial neighbours and support entries are sorted by column id, so the
// k-th gathers of a wavefront fall on a few adjacent cache lines.
//
// Workgroups are dispatched round-robin over the 8 XCDs; with xcd_remap each
// XCD instead owns a contiguous range of slices, so its private L2 holds one
// contiguous window of the gathered vector instead of eight.
#include "rbf_internal.h"

namespace rbf {
namespace {

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblk, int remap) {
    if (!remap) return bid;
    const int64_t per = nblk >> 3, rem = nblk & 7;
    const int64_t x = bid & 7, i = bid >> 3;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Slice of the calling wavefront.  flags bit 0: XCD remap; bit 1: visit the
// slices in reverse order (the odd sweeps of a zig-zag sequence, which start
// where the previous sweep ended, on lines still held by the memory-side
// Infinity Cache).  The row order within a sweep does not change results.
template <int WAVES>
__device__ __forceinline__ int64_t slice_index(int64_t nslices, int flags) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x, flags & 1);
    int64_t s = blk * WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if ((flags & 2) && s < nslices) s = nslices - 1 - s;
    return s;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), off, 64);
        unsigned hi = __shfl_xor((unsigned)(v >> 32), off, 64);
        unsigned long long o = ((unsigned long long)hi << 32) | lo;
        v = o > v ? o : v;
    }
    return v;
}

// Max of |values| over the workgroup into *slot, comparing IEEE bit patterns
// of non-negative doubles (monotone; a NaN outranks every number).
template <int WAVES>
__device__ __forceinline__ void block_max_to_slot(unsigned long long bits, unsigned long long *slot) {
    __shared__ unsigned long long red[WAVES];
    bits = wave_max_u64(bits);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
#pragma unroll
        for (int q = 1; q < WAVES; ++q) m = red[q] > m ? red[q] : m;
        if (m) atomicMax(slot, m);
    }
}

// Element position of support entry k of `lane` in a slice starting at base.
//   layout 0: base + 64 k + lane (one dword / qword per lane per entry)
//   layout 1: slice length padded to even; entry pairs interleaved,
//             base + 128 (k / 2) + 2 lane + k % 2, for indices and weights
//             alike: per 2 entries one 8-byte index vector and one 16-byte
//             FP64 weight vector per lane (a wavefront load covers 512 B /
//             1 KB contiguous).
__host__ __device__ __forceinline__ int64_t ell_pos(int layout, int64_t base, int k, int lane) {
    if (layout == 0) return base + (int64_t)k * kSlice + lane;
    return base + (int64_t)(k >> 1) * (2 * kSlice) + 2 * lane + (k & 1);
}

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Vec2;
template <>
struct Vec2<double> { typedef f64x2 type; };
template <>
struct Vec2<float> { typedef f32x2 type; };

// sum_k w[k] * x[idx[k]] over one row's packed entries (k < len), layout 0.
template <typename T, int U, int LAYOUT>
struct RowDot {
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w,
                                            const T *__restrict__ x, int64_t base, int lane, int len) {
        T acc = T(0);
        int k = 0;
        base += lane;
        for (; k + U <= len; k += U) {
            int32_t j[U];
            T ww[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                j[q] = ld_stream(idx + base + (int64_t)(k + q) * kSlice);
                ww[q] = ld_stream(w + base + (int64_t)(k + q) * kSlice);
            }
            T xx[U];
#pragma unroll
            for (int q = 0; q < U; ++q) xx[q] = x[j[q]];
#pragma unroll
            for (int q = 0; q < U; ++q) acc = fma(ww[q], xx[q], acc);
        }
        for (; k < len; ++k) {
            const int32_t j = ld_stream(idx + base + (int64_t)k * kSlice);
            const T ww = ld_stream(w + base + (int64_t)k * kSlice);
            acc = fma(ww, x[j], acc);
        }
        return acc;
    }
};

// Layout 1: pairs of entries as vectors; len is even.
template <typename T, int U>
struct RowDot<T, U, 1> {
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w,
                                            const T *__restrict__ x, int64_t base, int lane, int len) {
        typedef typename Vec2<T>::type V;
        constexpr int P = U / 2;
        T acc = T(0);
        const i32x2 *ip = (const i32x2 *)(idx + base) + lane;
        const V *wp = (const V *)(w + base) + lane;
        int k = 0;
        for (; k + U <= len; k += U) {
            i32x2 j[P];
            V ww[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                j[q] = __builtin_nontemporal_load(ip + ((k >> 1) + q) * kSlice);
                ww[q] = __builtin_nontemporal_load(wp + ((k >> 1) + q) * kSlice);
            }
            T xx[U];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                xx[2 * q] = x[j[q].x];
                xx[2 * q + 1] = x[j[q].y];
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                acc = fma(ww[q].x, xx[2 * q], acc);
                acc = fma(ww[q].y, xx[2 * q + 1], acc);
            }
        }
        for (; k < len; k += 2) {
            const i32x2 j = __builtin_nontemporal_load(ip + (k >> 1) * kSlice);
            const V ww = __builtin_nontemporal_load(wp + (k >> 1) * kSlice);
            acc = fma(ww.x, x[j.x], acc);
            acc = fma(ww.y, x[j.y], acc);
        }
        return acc;
    }
};

// Layout 1, software-pipelined: the index and weight vectors of the next
// group of U entries are requested before the current group's gathers, so a
// wavefront keeps two groups of stream loads in flight.
template <typename T, int U>
struct RowDot<T, U, 2> {
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w,
                                            const T *__restrict__ x, int64_t base, int lane, int len) {
        typedef typename Vec2<T>::type V;
        constexpr int P = U / 2;
        T acc = T(0);
        const i32x2 *ip = (const i32x2 *)(idx + base) + lane;
        const V *wp = (const V *)(w + base) + lane;
        const int groups = len / U;
        i32x2 jn[P];
        V wn[P];
        if (groups > 0) {
#pragma unroll
            for (int q = 0; q < P; ++q) {
                jn[q] = __builtin_nontemporal_load(ip + q * kSlice);
                wn[q] = __builtin_nontemporal_load(wp + q * kSlice);
            }
        }
        for (int g = 0; g < groups; ++g) {
            i32x2 jc[P];
            V wc[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                jc[q] = jn[q];
                wc[q] = wn[q];
            }
            if (g + 1 < groups) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    jn[q] = __builtin_nontemporal_load(ip + ((g + 1) * P + q) * kSlice);
                    wn[q] = __builtin_nontemporal_load(wp + ((g + 1) * P + q) * kSlice);
                }
            }
            T xx[U];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                xx[2 * q] = x[jc[q].x];
                xx[2 * q + 1] = x[jc[q].y];
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                acc = fma(wc[q].x, xx[2 * q], acc);
                acc = fma(wc[q].y, xx[2 * q + 1], acc);
            }
        }
        for (int k = groups * U; k < len; k += 2) {
            const i32x2 j = __builtin_nontemporal_load(ip + (k >> 1) * kSlice);
            const V ww = __builtin_nontemporal_load(wp + (k >> 1) * kSlice);
            acc = fma(ww.x, x[j.x], acc);
            acc = fma(ww.y, x[j.y], acc);
        }
        return acc;
    }
};

typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// Column of a 16-bit code: the segment base is held by lane `segment` of the
// wavefront (segreg = segbase[16 s + lane % 16]) and fetched by a lane permute.
__device__ __forceinline__ int32_t code_col(uint32_t c, int32_t segreg) {
    return __builtin_amdgcn_ds_bpermute((int)((c >> 10) & 0x3cu), segreg) + (int32_t)(c & 0xfffu);
}

// Compressed rows (Ell::code): 4 codes per 8-byte vector, weights as pairs
// (layout 1); len is even, codes are padded to a multiple of 4.
template <typename T, int U>
struct RowDotC {
    static_assert(U % 4 == 0, "groups of whole code vectors");
    __device__ static __forceinline__ T run(const uint16_t *__restrict__ code, int32_t segreg,
                                            const T *__restrict__ w, const T *__restrict__ x, int lane, int len) {
        typedef typename Vec2<T>::type V;
        T acc = T(0);
        const u16x4 *cp = (const u16x4 *)code + lane;
        const V *wp = (const V *)w + lane;
        int k = 0;
        for (; k + U <= len; k += U) {
            u16x4 c[U / 4];
            V ww[U / 2];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) c[q] = __builtin_nontemporal_load(cp + ((k >> 2) + q) * kSlice);
#pragma unroll
            for (int q = 0; q < U / 2; ++q) ww[q] = __builtin_nontemporal_load(wp + ((k >> 1) + q) * kSlice);
            T xx[U];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) {
                xx[4 * q] = x[code_col(c[q].x, segreg)];
                xx[4 * q + 1] = x[code_col(c[q].y, segreg)];
                xx[4 * q + 2] = x[code_col(c[q].z, segreg)];
                xx[4 * q + 3] = x[code_col(c[q].w, segreg)];
            }
#pragma unroll
            for (int q = 0; q < U / 2; ++q) {
                acc = fma(ww[q].x, xx[2 * q], acc);
                acc = fma(ww[q].y, xx[2 * q + 1], acc);
            }
        }
        for (; k < len; k += 2) {
            const u16x4 c = __builtin_nontemporal_load(cp + (k >> 2) * kSlice);
            const V ww = __builtin_nontemporal_load(wp + (k >> 1) * kSlice);
            const uint32_t c0 = (k & 2) ? c.z : c.x, c1 = (k & 2) ? c.w : c.y;
            acc = fma(ww.x, x[code_col(c0, segreg)], acc);
            acc = fma(ww.y, x[code_col(c1, segreg)], acc);
        }
        return acc;
    }
};

// Compressed view of a packed operator handed to the sweep kernels (all null
// when the plain column ids are read).
struct Codes {
    const uint16_t *code;
    const int64_t *cptr;
    const int32_t *segbase;
    const int8_t *cmode;
};

// Row sum of the calling lane's row of `slice`, from codes where the slice
// has them, else from the 32-bit ids.
// LAYOUT 3 is layout 1 read through the codes (kernels compiled for it hold
// both loops; the others hold only their own, which keeps their registers).
template <typename T, int U, int LAYOUT>
__device__ __forceinline__ T row_dot(const Codes &cs, const int64_t *__restrict__ slice_ptr,
                                     const int32_t *__restrict__ idx, const T *__restrict__ w,
                                     const T *__restrict__ x, int64_t slice, int lane, int len) {
    if constexpr (LAYOUT == 3) {
        if (cs.cmode[slice]) {
            const int32_t segreg = cs.segbase[slice * kSegs + (lane & (kSegs - 1))];
            return RowDotC<T, U>::run(cs.code + cs.cptr[slice], segreg, w + slice_ptr[slice], x, lane, len);
        }
        return RowDot<T, U, 1>::run(idx, w, x, slice_ptr[slice], lane, len);
    } else {
        return RowDot<T, U, LAYOUT>::run(idx, w, x, slice_ptr[slice], lane, len);
    }
}

// One explicit step on every interior row; optionally max |rho| into slot.
template <int WAVES, int U, int LAYOUT, bool REDUCE>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_f64(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, Codes cs, int64_t nslices, int64_t N_int, const double *__restrict__ f,
    const double *__restrict__ u_old, double *__restrict__ u_new, double dt, unsigned long long *res_slot,
    int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (slice < nslices) {
        const int len = slice_len[slice];
        const double acc = row_dot<double, U, LAYOUT>(cs, slice_ptr, idx, w, u_old, slice, lane, len);
        const int64_t row = slice * kSlice + lane;
        if (row < N_int) {
            const double rho = acc - f[row];
            u_new[row] = u_old[row] + dt * rho;
            bits = (unsigned long long)__double_as_longlong(fabs(rho));
        }
    }
    if (REDUCE) block_max_to_slot<WAVES>(bits, res_slot);
}

// FP32 step on the correction: e_new = e + dt (L32 e - r).
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_f32(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const float *__restrict__ w, Codes cs, int64_t nslices, int64_t N_int, const float *__restrict__ r,
    const float *__restrict__ e_old, float *__restrict__ e_new, float dt, int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int len = slice_len[slice];
    const float acc = row_dot<float, U, LAYOUT>(cs, slice_ptr, idx, w, e_old, slice, lane, len);
    const int64_t row = slice * kSlice + lane;
    if (row < N_int) e_new[row] = e_old[row] + dt * (acc - r[row]);
}

// Lu (and, with f, max |Lu - f| into slot).
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_apply_f64(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t nslices, int64_t N_int, const double *__restrict__ u,
    double *__restrict__ Lu, const double *__restrict__ f, unsigned long long *res_slot, int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (slice < nslices) {
        const int len = slice_len[slice];
        const double acc = RowDot<double, U, LAYOUT>::run(idx, w, u, slice_ptr[slice], lane, len);
        const int64_t row = slice * kSlice + lane;
        if (row < N_int) {
            if (Lu) Lu[row] = acc;
            if (f) bits = (unsigned long long)__double_as_longlong(fabs(acc - f[row]));
        }
    }
    if (res_slot) block_max_to_slot<WAVES>(bits, res_slot);
}

// Outer residual of the refinement loop: r32 = (float)(f - L64 u); e0 = 0;
// max |f - L64 u| into slot (the residual of u) when slot is given.
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_outer_residual(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t nslices, int64_t N_int, const double *__restrict__ f,
    const double *__restrict__ u, float *__restrict__ r32, float *__restrict__ e0, unsigned long long *res_slot,
    int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (slice < nslices) {
        const int len = slice_len[slice];
        const double acc = RowDot<double, U, LAYOUT>::run(idx, w, u, slice_ptr[slice], lane, len);
        const int64_t row = slice * kSlice + lane;
        if (row < N_int) {
            const double r = f[row] - acc;
            r32[row] = (float)r;
            e0[row] = 0.0f;
            bits = (unsigned long long)__double_as_longlong(fabs(r));
        }
    }
    if (res_slot) block_max_to_slot<WAVES>(bits, res_slot);
}

// One adjoint step on the transposed operator (rows of L^T = interior columns
// of L): lam_new = lam + dt (L_II^T lam), acc += lam_new.
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_adjoint_gather(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t nslices, int64_t N_int, const double *__restrict__ lam_old,
    double *__restrict__ lam_new, double *__restrict__ acc, double dt, int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int len = slice_len[slice];
    const double s = RowDot<double, U, LAYOUT>::run(idx, w, lam_old, slice_ptr[slice], lane, len);
    const int64_t row = slice * kSlice + lane;
    if (row < N_int) {
        const double l = lam_old[row] + dt * s;
        lam_new[row] = l;
        acc[row] += l;
    }
}

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
__global__ void k_pack_ell(int64_t row0, int64_t nrows, int32_t n_max, int32_t kmax, int64_t nslices, int layout,
                           const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                           const int32_t *__restrict__ sten, const int16_t *__restrict__ nrow,
                           const double *__restrict__ w_can, const int64_t *__restrict__ slice_ptr,
                           const int32_t *__restrict__ slice_len, int32_t *__restrict__ idx, double *__restrict__ w,
                           float *__restrict__ w32, double *__restrict__ wself, int32_t *__restrict__ foreign) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / kmax;
    const int k = (int)(t - i * kmax);
    if (i >= nslices * kSlice) return;
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
            const int32_t *row = sten + r * (int64_t)n_max;
            col = iperm[row[k]];
            int rank = 0;
            for (int q = 0; q < n; ++q) rank += (iperm[row[q]] < col) ? 1 : 0;
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
// With u_store (supports of interior nodes and the row itself only, so no
// Neumann row reads another's value) the new value goes straight into both
// iterate buffers: u_store[0] = the current one, u_store[1] = the next.
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_neumann_eval(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, int64_t nslices, int64_t N_int, int64_t N_neu, const double *__restrict__ wself,
    const double *__restrict__ g, const double *u, double *__restrict__ nb, double *u_cur, double *u_next) {
    const int64_t slice = (int64_t)blockIdx.x * WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int len = slice_len[slice];
    const double acc = RowDot<double, U, LAYOUT>::run(idx, w, u, slice_ptr[slice], lane, len);
    const int64_t j = slice * kSlice + lane;
    if (j >= N_neu) return;
    if (g) {
        const double v = (g[N_int + j] - acc) / wself[j];
        if (u_cur) {
            u_cur[N_int + j] = v;
            u_next[N_int + j] = v;
        } else {
            nb[j] = v;
        }
    } else {
        nb[N_int + j] = acc + wself[j] * u[N_int + j];  // without data: the derivative itself
    }
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

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Dispatch over the tuned (waves per block, unroll, layout) triples.
template <template <int, int, int> class F, typename... A>
hipError_t dispatch_shape(const SweepCfg &c, int layout, A &&...a) {
#define RBF_CASE(WV, UN)                                                                            \
    if (c.waves_per_block == WV && c.unroll == UN) {                                                \
        if (!layout) return F<WV, UN, 0>::run(a...);                                                \
        return c.pipeline ? F<WV, UN, 2>::run(a...) : F<WV, UN, 1>::run(a...);                       \
    }
    RBF_CASE(2, 4) RBF_CASE(2, 8) RBF_CASE(2, 16)
    RBF_CASE(4, 4) RBF_CASE(4, 8) RBF_CASE(4, 16)
    RBF_CASE(8, 4) RBF_CASE(8, 8) RBF_CASE(8, 16)
#undef RBF_CASE
    return hipErrorInvalidValue;
}

// The same over the shapes of the sweeps that read codes (LAYOUT 3).
template <template <int, int, int> class F, typename... A>
hipError_t dispatch_codes(const SweepCfg &c, A &&...a) {
#define RBF_CASE(WV, UN) \
    if (c.waves_per_block == WV && c.unroll == UN) return F<WV, UN, 3>::run(a...);
    RBF_CASE(2, 4) RBF_CASE(2, 8) RBF_CASE(2, 16)
    RBF_CASE(4, 4) RBF_CASE(4, 8) RBF_CASE(4, 16)
    RBF_CASE(8, 4) RBF_CASE(8, 8) RBF_CASE(8, 16)
#undef RBF_CASE
    return hipErrorInvalidValue;
}

// Whether a sweep with shape c reads the codes of e.
inline bool use_codes(const SweepCfg &c, const Ell &e) { return c.codes && e.layout == 1 && e.cmode; }

inline Codes codes_of(const Ell &e) { return Codes{e.code, e.cptr, e.segbase, e.cmode}; }

template <int WV, int UN, int LY>
struct SweepF64 {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const double *f, const double *uo, double *un,
                          double dt, unsigned long long *slot, int remap) {
        if (!e.nslices) return hipSuccess;
        const unsigned g = grid1d(e.nslices, WV);
        const Codes cs = codes_of(e);
        if (slot)
            hipLaunchKernelGGL((k_sweep_f64<WV, UN, LY, true>), dim3(g), dim3(WV * 64), 0, s, e.slice_ptr,
                               e.slice_len, e.idx, e.w, cs, e.nslices, N_int, f, uo, un, dt, slot, remap);
        else
            hipLaunchKernelGGL((k_sweep_f64<WV, UN, LY, false>), dim3(g), dim3(WV * 64), 0, s, e.slice_ptr,
                               e.slice_len, e.idx, e.w, cs, e.nslices, N_int, f, uo, un, dt, slot, remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct SweepF32 {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const float *r, const float *eo, float *en,
                          float dt, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_sweep_f32<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w32, codes_of(e), e.nslices, N_int, r, eo, en, dt,
                           remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct ApplyF64 {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const double *u, double *Lu, const double *f,
                          unsigned long long *slot, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_apply_f64<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w, e.nslices, N_int, u, Lu, f, slot, remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct AdjGather {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const double *lo, double *ln, double *acc,
                          double dt, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_adjoint_gather<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w, e.nslices, N_int, lo, ln, acc, dt, remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct OuterRes {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const double *f, const double *u, float *r32,
                          float *e0, unsigned long long *slot, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_outer_residual<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w, e.nslices, N_int, f, u, r32, e0, slot, remap);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_pack_ell(hipStream_t s, int64_t row0, int64_t nrows, int32_t n_max, const int32_t *perm,
                           const int32_t *iperm, const int32_t *sten, const int16_t *nrow, const double *w_can,
                           const Ell &e, double *wself, int32_t *foreign) {
    const int32_t kmax = e.max_len;
    const int64_t total = e.nslices * kSlice * (int64_t)kmax;
    if (!total) return hipSuccess;
    hipLaunchKernelGGL(k_pack_ell, dim3(grid1d(total, 256)), dim3(256), 0, s, row0, nrows, n_max, kmax, e.nslices,
                       e.layout, perm, iperm, sten, nrow, w_can, e.slice_ptr, e.slice_len, e.idx, e.w, e.w32, wself,
                       foreign);
    return hipGetLastError();
}

// Segment codes of one slice per workgroup (one wavefront): the distinct
// aligned 4096-id blocks touched by any entry of the slice (padding entries
// included, so every stored column stays encodable) are found in ascending
// order by repeated wavefront minima; with at most kSegs of them the slice
// gets codes (cmode 1), else it keeps only its 32-bit ids (cmode 0).
__global__ __launch_bounds__(64) void k_encode_codes(const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ slice_len,
                                                     const int32_t *__restrict__ idx, int64_t nslices,
                                                     const int64_t *__restrict__ cptr, uint16_t *__restrict__ code,
                                                     int32_t *__restrict__ segbase, int8_t *__restrict__ cmode) {
    __shared__ uint16_t blk[kMaxSupport * kSlice];
    __shared__ int32_t list[kSegs];
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int len = slice_len[s];
    const int64_t base = slice_ptr[s];
    for (int k = 0; k < len; ++k) blk[k * kSlice + lane] = (uint16_t)(idx[ell_pos(1, base, k, lane)] >> 12);
    __syncthreads();
    int cnt = 0, cur = -1;
    bool over = false;
    for (int it = 0; it <= kSegs; ++it) {
        int mn = 0x7fffffff;
        for (int k = 0; k < len; ++k) {
            const int v = blk[k * kSlice + lane];
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
        out[(int64_t)(k >> 2) * (4 * kSlice) + 4 * lane + (k & 3)] = c;
    }
}

hipError_t launch_encode_codes(hipStream_t s, const Ell &e) {
    if (!e.nslices || e.layout != 1 || !e.code) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_encode_codes, dim3((unsigned)e.nslices), dim3(kSlice), 0, s, e.slice_ptr, e.slice_len, e.idx,
                       e.nslices, e.cptr, e.code, e.segbase, e.cmode);
    return hipGetLastError();
}

// The Neumann update of one step (evaluate all new boundary values from the
// current iterate, then store them in both buffers).
hipError_t launch_neumann_update(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                 const double *g, double *u_cur, double *u_next, double *nb, bool direct) {
    if (!e.nslices) return hipSuccess;
    const unsigned grid = grid1d(e.nslices, 4);
    double *uc = direct ? u_cur : nullptr, *un = direct ? u_next : nullptr;
    if (e.layout)
        hipLaunchKernelGGL((k_neumann_eval<4, 8, 1>), dim3(grid), dim3(256), 0, s, e.slice_ptr, e.slice_len, e.idx,
                           e.w, e.nslices, N_int, N_neu, wself, g, u_cur, nb, uc, un);
    else
        hipLaunchKernelGGL((k_neumann_eval<4, 8, 0>), dim3(grid), dim3(256), 0, s, e.slice_ptr, e.slice_len, e.idx,
                           e.w, e.nslices, N_int, N_neu, wself, g, u_cur, nb, uc, un);
    if (!direct)
        hipLaunchKernelGGL(k_neumann_store, dim3(grid1d(N_neu, 256)), dim3(256), 0, s, N_int, N_neu, nb, u_cur,
                           u_next);
    return hipGetLastError();
}

// out[N_int + j] = (D u) at Neumann row j (its normal-derivative stencil).
hipError_t launch_neumann_apply(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                const double *u, double *out) {
    if (!e.nslices) return hipSuccess;
    const unsigned grid = grid1d(e.nslices, 4);
    if (e.layout)
        hipLaunchKernelGGL((k_neumann_eval<4, 8, 1>), dim3(grid), dim3(256), 0, s, e.slice_ptr, e.slice_len, e.idx,
                           e.w, e.nslices, N_int, N_neu, wself, nullptr, u, out, nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_neumann_eval<4, 8, 0>), dim3(grid), dim3(256), 0, s, e.slice_ptr, e.slice_len, e.idx,
                           e.w, e.nslices, N_int, N_neu, wself, nullptr, u, out, nullptr, nullptr);
    return hipGetLastError();
}

inline int order_flags(const SweepCfg &c, int parity) { return c.xcd_remap | ((c.zigzag && (parity & 1)) ? 2 : 0); }

hipError_t launch_sweep_f64(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *f,
                            const double *u_old, double *u_new, double dt, unsigned long long *res_slot,
                            int parity) {
    if (use_codes(c, e))
        return dispatch_codes<SweepF64>(c, s, e, N_int, f, u_old, u_new, dt, res_slot, order_flags(c, parity));
    return dispatch_shape<SweepF64>(c, e.layout, s, e, N_int, f, u_old, u_new, dt, res_slot, order_flags(c, parity));
}

hipError_t launch_sweep_f32(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const float *r,
                            const float *e_old, float *e_new, float dt, int parity) {
    if (use_codes(c, e))
        return dispatch_codes<SweepF32>(c, s, e, N_int, r, e_old, e_new, dt, order_flags(c, parity));
    return dispatch_shape<SweepF32>(c, e.layout, s, e, N_int, r, e_old, e_new, dt, order_flags(c, parity));
}

hipError_t launch_apply_f64(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *u,
                            double *Lu, const double *f, unsigned long long *res_slot) {
    return dispatch_shape<ApplyF64>(c, e.layout, s, e, N_int, u, Lu, f, res_slot, c.xcd_remap);
}

hipError_t launch_outer_residual(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *f,
                                 const double *u, float *r32, float *e0, unsigned long long *res_slot) {
    return dispatch_shape<OuterRes>(c, e.layout, s, e, N_int, f, u, r32, e0, res_slot, c.xcd_remap);
}

hipError_t launch_adjoint_gather(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *lam_old,
                                 double *lam_new, double *acc, double dt, int parity) {
    return dispatch_shape<AdjGather>(c, e.layout, s, e, N_int, lam_old, lam_new, acc, dt, order_flags(c, parity));
}

hipError_t launch_add_correction(hipStream_t s, int64_t N_int, double *u, const float *e) {
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
    hipLaunchKernelGGL(k_adjoint_update, dim3(grid1d(N_int, 256)), dim3(256), 0, s, N_int, dt, lam, acc, tmp);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst) {
    hipLaunchKernelGGL(k_gather, dim3(grid1d(n, 256)), dim3(256), 0, s, n, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst) {
    hipLaunchKernelGGL(k_scatter, dim3(grid1d(n, 256)), dim3(256), 0, s, n, perm, src, dst);
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
    hipLaunchKernelGGL(k_scale_interior, dim3(grid1d(N, 256)), dim3(256), 0, s, N, N_int, a, src, dst);
    return hipGetLastError();
}

}  // namespace rbf
