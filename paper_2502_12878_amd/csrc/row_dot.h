// Device building blocks shared by the kernels that read the packed operator:
// slice scheduling (XCD-aware block order, zig-zag order), wavefront and
// workgroup max reductions, the positions of support entries in the packed
// layouts, and the row sums over a row's support entries (32-bit column ids
// in three layouts, or 16-bit segment codes).
#pragma once

#include "rbf_internal.h"

namespace rbf {
namespace {

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }

// Stream load of the packed operator: non-temporal (NT, kept out of the
// caches) or an ordinary load (may stay in the memory-side cache between
// sweeps).
template <bool NT, typename T>
__device__ __forceinline__ T ld_op(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

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

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Gathers of the iterate through a raw buffer resource: one 32-bit byte
// offset per lane (no 64-bit address arithmetic, half the address
// registers), and an offset past the n elements reads 0 instead of faulting.
template <typename T>
struct BufGather;
template <>
struct BufGather<double> {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufGather(const double *p, int64_t n) {
        const uint64_t bytes = (uint64_t)n * 8u;
        r = __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, (int)(bytes > 0xffffffffu ? 0xffffffffu : bytes),
                                              0x00020000);
    }
    __device__ __forceinline__ double operator[](int32_t j) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)j * 8u, 0, 0));
    }
};
template <>
struct BufGather<float> {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufGather(const float *p, int64_t n) {
        const uint64_t bytes = (uint64_t)n * 4u;
        r = __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, (int)(bytes > 0xffffffffu ? 0xffffffffu : bytes),
                                              0x00020000);
    }
    __device__ __forceinline__ float operator[](int32_t j) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)j * 4u, 0, 0));
    }
};

// sum_k w[k] * x[idx[k]] over one row's packed entries (k < len), layout 0.
template <typename T, int U, int LAYOUT>
struct RowDot {
    template <class X>
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w, const X &x,
                                            int64_t base, int lane, int len) {
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
    template <class X>
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w, const X &x,
                                            int64_t base, int lane, int len) {
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
    template <class X>
    __device__ static __forceinline__ T run(const int32_t *__restrict__ idx, const T *__restrict__ w, const X &x,
                                            int64_t base, int lane, int len) {
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

// The last len - kt < U entries of a coded row (kt a multiple of 4): all
// their code and weight vectors are requested at once, then the gathers,
// then the products in entry order (the order of the one-pair-at-a-time
// loop, so the result is the same bit for bit).
template <typename T, int U, bool NT, class X>
__device__ __forceinline__ T coded_tail(const u16x4 *cp, const typename Vec2<T>::type *wp, int32_t segreg,
                                        const X &x, int kt, int len, T acc) {
    typedef typename Vec2<T>::type V;
    if (kt >= len) return acc;
    u16x4 c[U / 4];
    V ww[U / 2];
#pragma unroll
    for (int q = 0; q < U / 4; ++q)
        if (kt + 4 * q < len) c[q] = ld_op<NT>(cp + ((kt >> 2) + q) * kSlice);
#pragma unroll
    for (int q = 0; q < U / 2; ++q)
        if (kt + 2 * q < len) ww[q] = ld_op<NT>(wp + ((kt >> 1) + q) * kSlice);
    T xx[U];
#pragma unroll
    for (int q = 0; q < U / 4; ++q)
        if (kt + 4 * q < len) {
            xx[4 * q] = x[code_col(c[q].x, segreg)];
            xx[4 * q + 1] = x[code_col(c[q].y, segreg)];
            if (kt + 4 * q + 2 < len) {
                xx[4 * q + 2] = x[code_col(c[q].z, segreg)];
                xx[4 * q + 3] = x[code_col(c[q].w, segreg)];
            }
        }
#pragma unroll
    for (int q = 0; q < U / 2; ++q)
        if (kt + 2 * q < len) {
            acc = fma(ww[q].x, xx[2 * q], acc);
            acc = fma(ww[q].y, xx[2 * q + 1], acc);
        }
    return acc;
}

// Compressed rows (Ell::code): 4 codes per 8-byte vector, weights as pairs
// (layout 1); len is even, codes are padded to a multiple of 4.
template <typename T, int U, bool NT = true>
struct RowDotC {
    static_assert(U % 4 == 0, "groups of whole code vectors");
    template <class X>
    __device__ static __forceinline__ T run(const uint16_t *__restrict__ code, int32_t segreg,
                                            const T *__restrict__ w, const X &x, int lane, int len) {
        typedef typename Vec2<T>::type V;
        T acc = T(0);
        const u16x4 *cp = (const u16x4 *)code + lane;
        const V *wp = (const V *)w + lane;
        int k = 0;
        for (; k + U <= len; k += U) {
            u16x4 c[U / 4];
            V ww[U / 2];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) c[q] = ld_op<NT>(cp + ((k >> 2) + q) * kSlice);
#pragma unroll
            for (int q = 0; q < U / 2; ++q) ww[q] = ld_op<NT>(wp + ((k >> 1) + q) * kSlice);
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
        return coded_tail<T, U, NT>(cp, wp, segreg, x, k, len, acc);
    }
};

// RowDotC, software-pipelined: the codes and weights of the next group of U
// entries are requested before the current group's gathers.
template <typename T, int U, bool NT = true>
struct RowDotCP {
    static_assert(U % 4 == 0, "groups of whole code vectors");
    template <class X>
    __device__ static __forceinline__ T run(const uint16_t *__restrict__ code, int32_t segreg,
                                            const T *__restrict__ w, const X &x, int lane, int len) {
        typedef typename Vec2<T>::type V;
        T acc = T(0);
        const u16x4 *cp = (const u16x4 *)code + lane;
        const V *wp = (const V *)w + lane;
        const int groups = len / U;
        u16x4 cn[U / 4];
        V wn[U / 2];
        if (groups > 0) {
#pragma unroll
            for (int q = 0; q < U / 4; ++q) cn[q] = ld_op<NT>(cp + q * kSlice);
#pragma unroll
            for (int q = 0; q < U / 2; ++q) wn[q] = ld_op<NT>(wp + q * kSlice);
        }
        for (int g = 0; g < groups; ++g) {
            u16x4 cc[U / 4];
            V wc[U / 2];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) cc[q] = cn[q];
#pragma unroll
            for (int q = 0; q < U / 2; ++q) wc[q] = wn[q];
            if (g + 1 < groups) {
#pragma unroll
                for (int q = 0; q < U / 4; ++q) cn[q] = ld_op<NT>(cp + ((g + 1) * (U / 4) + q) * kSlice);
#pragma unroll
                for (int q = 0; q < U / 2; ++q) wn[q] = ld_op<NT>(wp + ((g + 1) * (U / 2) + q) * kSlice);
            }
            T xx[U];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) {
                xx[4 * q] = x[code_col(cc[q].x, segreg)];
                xx[4 * q + 1] = x[code_col(cc[q].y, segreg)];
                xx[4 * q + 2] = x[code_col(cc[q].z, segreg)];
                xx[4 * q + 3] = x[code_col(cc[q].w, segreg)];
            }
#pragma unroll
            for (int q = 0; q < U / 2; ++q) {
                acc = fma(wc[q].x, xx[2 * q], acc);
                acc = fma(wc[q].y, xx[2 * q + 1], acc);
            }
        }
        return coded_tail<T, U, NT>(cp, wp, segreg, x, groups * U, len, acc);
    }
};

// RowDotCP with ordinary loads for a lane of rl <= len entries (a lane-ordered
// operator, Ell::lmeta): the code and weight vectors past the lane's own
// entries are read through raw buffer resources at an offset beyond their
// range, which returns 0 without a memory access, so the lines that hold only
// padding of the slice's shorter lanes are never fetched.  Masked entries add
// fma(0, x, acc) = acc; the lane's entries are summed in the order of
// RowDotCP, and the last, partial group gathers only up to the slice length.
template <int U>
struct RowDotCM {
    static_assert(U % 4 == 0, "groups of whole code vectors");
    template <class X>
    __device__ static __forceinline__ double run(const uint16_t *__restrict__ code, int32_t segreg,
                                                 const double *__restrict__ w, const X &x, int lane, int len, int rl) {
        constexpr uint32_t kOff = 0x80000000u;  // past both ranges: reads 0
        const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc((void *)code, 0, 0x7fffffff, 0x00020000);
        const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc((void *)w, 0, 0x7fffffff, 0x00020000);
        // code vector r (entries 4r .. 4r + 3) at byte 512 r + 8 lane; weight
        // pair p (entries 2p, 2p + 1) at byte 1024 p + 16 lane
        const uint32_t cl = 8u * lane, wl = 16u * lane;
        auto cload = [&](int r) {
            const uint32_t off = 4 * r < rl ? 512u * r + cl : kOff;
            return __builtin_bit_cast(u16x4, __builtin_amdgcn_raw_buffer_load_b64(rc, off, 0, 0));
        };
        auto wload = [&](int p) {
            const uint32_t off = 2 * p < rl ? 1024u * p + wl : kOff;
            return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rw, off, 0, 0));
        };
        double acc = 0.0;
        const int full = len / U, groups = (len + U - 1) / U;
        u16x4 cn[U / 4];
        f64x2 wn[U / 2];
        if (groups > 0) {
#pragma unroll
            for (int q = 0; q < U / 4; ++q) cn[q] = cload(q);
#pragma unroll
            for (int q = 0; q < U / 2; ++q) wn[q] = wload(q);
        }
        for (int g = 0; g < full; ++g) {
            u16x4 cc[U / 4];
            f64x2 wc[U / 2];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) cc[q] = cn[q];
#pragma unroll
            for (int q = 0; q < U / 2; ++q) wc[q] = wn[q];
            if (g + 1 < groups) {
#pragma unroll
                for (int q = 0; q < U / 4; ++q) cn[q] = cload((g + 1) * (U / 4) + q);
#pragma unroll
                for (int q = 0; q < U / 2; ++q) wn[q] = wload((g + 1) * (U / 2) + q);
            }
            double xx[U];
#pragma unroll
            for (int q = 0; q < U / 4; ++q) {
                xx[4 * q] = x[code_col(cc[q].x, segreg)];
                xx[4 * q + 1] = x[code_col(cc[q].y, segreg)];
                xx[4 * q + 2] = x[code_col(cc[q].z, segreg)];
                xx[4 * q + 3] = x[code_col(cc[q].w, segreg)];
            }
#pragma unroll
            for (int q = 0; q < U / 2; ++q) {
                acc = fma(wc[q].x, xx[2 * q], acc);
                acc = fma(wc[q].y, xx[2 * q + 1], acc);
            }
        }
        if (full < groups) {  // entries kt .. len - 1, already requested (len is even)
            const int kt = full * U;
            double xx[U];
#pragma unroll
            for (int q = 0; q < U / 4; ++q)
                if (kt + 4 * q < len) {
                    xx[4 * q] = x[code_col(cn[q].x, segreg)];
                    xx[4 * q + 1] = x[code_col(cn[q].y, segreg)];
                    if (kt + 4 * q + 2 < len) {
                        xx[4 * q + 2] = x[code_col(cn[q].z, segreg)];
                        xx[4 * q + 3] = x[code_col(cn[q].w, segreg)];
                    }
                }
#pragma unroll
            for (int q = 0; q < U / 2; ++q)
                if (kt + 2 * q < len) {
                    acc = fma(wn[q].x, xx[2 * q], acc);
                    acc = fma(wn[q].y, xx[2 * q + 1], acc);
                }
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
// LAYOUT 3 / 4 are layouts 1 / 2 read through the codes, 5 / 6 the same with
// ordinary instead of non-temporal stream loads, 7 is 6 with the loads past
// the lane's rl entries masked (RowDotCM, FP64 only) (kernels compiled for
// them hold both loops; the others hold only their own, which keeps their
// registers).
template <typename T, int U, int LAYOUT, class X>
__device__ __forceinline__ T row_dot(const Codes &cs, const int64_t *__restrict__ slice_ptr,
                                     const int32_t *__restrict__ idx, const T *__restrict__ w, const X &x,
                                     int64_t slice, int lane, int len, int rl = 0) {
    if constexpr (LAYOUT >= 3) {
        constexpr bool NT = LAYOUT <= 4;                    // 5 / 6 / 7: ordinary stream loads
        constexpr bool PIPE = LAYOUT == 4 || LAYOUT >= 6;
        // the slice's descriptors in one round trip (segbase and cptr exist,
        // unused, for slices without codes)
        const int8_t coded = cs.cmode[slice];
        const int32_t segreg = cs.segbase[slice * kSegs + (lane & (kSegs - 1))];
        const int64_t cbase = cs.cptr[slice];
        const int64_t sbase = slice_ptr[slice];
        if (coded) {
            if constexpr (LAYOUT == 7)
                return RowDotCM<U>::run(cs.code + cbase, segreg, w + sbase, x, lane, len, rl);
            else if constexpr (PIPE)
                return RowDotCP<T, U, NT>::run(cs.code + cbase, segreg, w + sbase, x, lane, len);
            else
                return RowDotC<T, U, NT>::run(cs.code + cbase, segreg, w + sbase, x, lane, len);
        }
        return RowDot<T, U, PIPE ? 2 : 1>::run(idx, w, x, sbase, lane, len);
    } else {
        return RowDot<T, U, LAYOUT>::run(idx, w, x, slice_ptr[slice], lane, len);
    }
}

}  // namespace

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace rbf
