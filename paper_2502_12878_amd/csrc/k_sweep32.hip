// FP32 inner sweep of the refinement loop, e <- e + dt (L32 e - r), reading
// the FP32 weights of coded slices in the layout of the 16-bit codes: entry k
// of lane l at cptr[s] + 256 (k / 4) + 4 l + k % 4 (Ell::w32q), so a lane
// loads four codes (8 B) and their four weights (16 B) with one vector load
// each.  Slices without codes read the paired layout.  Each row's entries are
// summed in the same order as in the other sweep layouts, so the iterates are
// bitwise those of k_sweep_f32.
#include "row_dot.h"

namespace rbf {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// sum_k w[k] e[col(k)] over one coded row: codes and weights as 4-vectors;
// len is even, both arrays are padded to a multiple of 4 (padding skipped).
// PIPE requests the next group's vectors before the current group's gathers.
template <int U, bool NT, bool PIPE>
struct RowDotCQ {
    static_assert(U % 4 == 0, "groups of whole vectors");
    template <class X>
    __device__ static __forceinline__ float run(const uint16_t *__restrict__ code, const float *__restrict__ wq,
                                                int32_t segreg, const X &x, int lane, int len) {
        constexpr int Q = U / 4;
        float acc = 0.0f;
        const u16x4 *cp = (const u16x4 *)code + lane;
        const f32x4 *wp = (const f32x4 *)wq + lane;
        const int groups = len / U;
        u16x4 cn[Q];
        f32x4 wn[Q];
        if (PIPE && groups > 0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                cn[q] = ld_op<NT>(cp + q * kSlice);
                wn[q] = ld_op<NT>(wp + q * kSlice);
            }
        }
        for (int g = 0; g < groups; ++g) {
            u16x4 c[Q];
            f32x4 ww[Q];
            if (PIPE) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    c[q] = cn[q];
                    ww[q] = wn[q];
                }
                if (g + 1 < groups) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        cn[q] = ld_op<NT>(cp + ((g + 1) * Q + q) * kSlice);
                        wn[q] = ld_op<NT>(wp + ((g + 1) * Q + q) * kSlice);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    c[q] = ld_op<NT>(cp + (g * Q + q) * kSlice);
                    ww[q] = ld_op<NT>(wp + (g * Q + q) * kSlice);
                }
            }
            float xx[U];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                xx[4 * q] = x[code_col(c[q].x, segreg)];
                xx[4 * q + 1] = x[code_col(c[q].y, segreg)];
                xx[4 * q + 2] = x[code_col(c[q].z, segreg)];
                xx[4 * q + 3] = x[code_col(c[q].w, segreg)];
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                acc = fmaf(ww[q].x, xx[4 * q], acc);
                acc = fmaf(ww[q].y, xx[4 * q + 1], acc);
                acc = fmaf(ww[q].z, xx[4 * q + 2], acc);
                acc = fmaf(ww[q].w, xx[4 * q + 3], acc);
            }
        }
        for (int k = groups * U; k < len; k += 4) {
            const u16x4 c = ld_op<NT>(cp + (k >> 2) * kSlice);
            const f32x4 ww = ld_op<NT>(wp + (k >> 2) * kSlice);
            acc = fmaf(ww.x, x[code_col(c.x, segreg)], acc);
            acc = fmaf(ww.y, x[code_col(c.y, segreg)], acc);
            if (k + 2 < len) {  // len is even: the last vector may hold 2 entries
                acc = fmaf(ww.z, x[code_col(c.z, segreg)], acc);
                acc = fmaf(ww.w, x[code_col(c.w, segreg)], acc);
            }
        }
        return acc;
    }
};

// LAYOUT 3..6 as in row_dot (codes; 5 / 6 with ordinary loads; 4 / 6
// pipelined).
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_f32q(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const float *__restrict__ w, const float *__restrict__ wq, Codes cs, int64_t nslices, int64_t N_int,
    int64_t ncols, const float *__restrict__ r, const float *__restrict__ e_old, float *__restrict__ e_new, float dt,
    int order) {
    constexpr bool NT = LAYOUT <= 4;
    constexpr bool PIPE = LAYOUT == 4 || LAYOUT == 6;
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    // the slice's descriptors and the row's r and e in one round trip
    const int len = slice_len[slice];
    const int8_t coded = cs.cmode[slice];
    const int32_t segreg = cs.segbase[slice * kSegs + (lane & (kSegs - 1))];
    const int64_t cbase = cs.cptr[slice];
    const int64_t sbase = slice_ptr[slice];
    const int64_t row = slice * kSlice + lane;
    const bool live = row < N_int;
    const float rr = live ? r[row] : 0.0f;
    const float er = live ? e_old[row] : 0.0f;
    const BufGather<float> x(e_old, ncols);
    float acc;
    if (coded) acc = RowDotCQ<U, NT, PIPE>::run(cs.code + cbase, wq + cbase, segreg, x, lane, len);
    else acc = RowDot<float, U, PIPE ? 2 : 1>::run(idx, w, x, sbase, lane, len);
    if (live) e_new[row] = er + dt * (acc - rr);
}

template <int WV, int UN, int LY>
hipError_t run_f32q(hipStream_t s, const Ell &e, int64_t N_int, const float *r, const float *eo, float *en, float dt,
                    int order) {
    hipLaunchKernelGGL((k_sweep_f32q<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s, e.slice_ptr,
                       e.slice_len, e.idx, e.w32, e.w32q, Codes{e.code, e.cptr, e.segbase, e.cmode}, e.nslices,
                       N_int, e.ncols, r, eo, en, dt, order);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_f32q(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const float *r,
                             const float *e_old, float *e_new, float dt, int parity) {
    if (!e.nslices) return hipSuccess;
    if (!e.w32q || !e.cmode || !e.w32) return hipErrorInvalidValue;
    const int order = c.xcd_remap | ((c.zigzag && (parity & 1)) ? 2 : 0);
    const int lay = c.temporal ? (c.pipeline ? 6 : 5) : (c.pipeline ? 4 : 3);
#define RBF_CASE(WV, UN)                                                                   \
    if (c.waves_per_block == WV && c.unroll == UN) {                                       \
        switch (lay) {                                                                     \
        case 3: return run_f32q<WV, UN, 3>(s, e, N_int, r, e_old, e_new, dt, order);       \
        case 4: return run_f32q<WV, UN, 4>(s, e, N_int, r, e_old, e_new, dt, order);       \
        case 5: return run_f32q<WV, UN, 5>(s, e, N_int, r, e_old, e_new, dt, order);       \
        default: return run_f32q<WV, UN, 6>(s, e, N_int, r, e_old, e_new, dt, order);      \
        }                                                                                  \
    }
    RBF_CASE(2, 4) RBF_CASE(2, 8) RBF_CASE(2, 16) RBF_CASE(2, 32)
    RBF_CASE(4, 4) RBF_CASE(4, 8) RBF_CASE(4, 16) RBF_CASE(4, 32)
    RBF_CASE(8, 4) RBF_CASE(8, 8) RBF_CASE(8, 16) RBF_CASE(8, 32)
#undef RBF_CASE
    return hipErrorInvalidValue;
}

}  // namespace rbf
