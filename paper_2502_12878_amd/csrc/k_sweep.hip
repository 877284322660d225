// Sweep kernels of the explicit RBF-FD iteration (Sec. II-C, the Jacobi step
// u <- u + dt (L_h u - f) with L_h u at a node a weighted sum over its support,
// Sec. II) and the single-operator kernels built from the same row sums.  All
// of them read a packed operator (sliced ELL, 64 rows per slice = one
// wavefront; layouts and row sums in row_dot.h).
//
// The sweep is bound by HBM bandwidth: per interior node-update it moves the
// row's column ids (4 B each, or 2 B as segment codes), its weights (8 B) and
// 24 B of f, u and u_new.  Operator streams are read once per sweep, with
// non-temporal loads or, in the "temporal" layouts, ordinary loads that let
// the memory-side Infinity Cache keep the end of one sweep for the start of
// the next (zig-zag order).  Rows of a slice are spatial neighbours and
// support entries are sorted by column id, so the k-th gathers of a
// wavefront fall on a few adjacent cache lines.
//
// Workgroups are dispatched round-robin over the 8 XCDs; with xcd_remap each
// XCD instead owns a contiguous range of slices, so its private L2 holds one
// contiguous window of the gathered vector instead of eight.  The shape
// (workgroup size, unroll, layout, order) is chosen per operator by the
// autotuner; every shape sums each row in the same order.
//
// The adjoint's transposed steps are this same sweep on the transposed
// operator L_II^T (Horner form of the gradient sum; rbf_api.cpp).
#include "row_dot.h"

namespace rbf {
namespace {

// Row of lane `lane` of `slice` and its entry count: lanes hold rows in
// order unless the operator has a lane order (Ell::lmeta).
struct LaneRow {
    int64_t row;
    int len;
};
template <bool ORDERED>
__device__ __forceinline__ LaneRow lane_row(const uint16_t *__restrict__ lmeta, int64_t slice, int lane, int len) {
    if (ORDERED || lmeta) {
        const int m = lmeta[slice * kSlice + lane];
        return LaneRow{slice * kSlice + (m & (kSlice - 1)), m >> 6};
    }
    return LaneRow{slice * kSlice + lane, len};
}

// One explicit step on every interior row; optionally max |rho| into slot.
template <int WAVES, int U, int LAYOUT, bool REDUCE>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_f64(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, Codes cs, const uint16_t *__restrict__ lmeta, int64_t s0, int64_t nslices,
    int64_t N_int, int64_t ncols, const double *__restrict__ f, const double *__restrict__ u_old,
    double *__restrict__ u_new, double dt, unsigned long long *res_slot, int order) {
    const int64_t local = slice_index<WAVES>(nslices, order);
    const int64_t slice = s0 + local;
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (local < nslices) {
        const int len = slice_len[slice];
        const LaneRow lr = lane_row<LAYOUT == 7>(lmeta, slice, lane, len);
        const int64_t row = lr.row;
        const bool live = row < N_int;
        const double fr = live ? f[row] : 0.0;  // requested with the slice's descriptors
        const double ur = live ? u_old[row] : 0.0;
        const double acc =
            row_dot<double, U, LAYOUT>(cs, slice_ptr, idx, w, BufGather<double>(u_old, ncols), slice, lane, len, lr.len);
        if (live) {
            const double rho = acc - fr;
            u_new[row] = ur + dt * rho;
            bits = (unsigned long long)__double_as_longlong(fabs(rho));
        }
    }
    if (REDUCE) block_max_to_slot<WAVES>(bits, res_slot);
}

// FP32 step on the correction: e_new = e + dt (L32 e - r).
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_sweep_f32(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const float *__restrict__ w, Codes cs, int64_t nslices, int64_t N_int, int64_t ncols, const float *__restrict__ r,
    const float *__restrict__ e_old, float *__restrict__ e_new, float dt, int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int len = slice_len[slice];
    const int64_t row = slice * kSlice + lane;
    const bool live = row < N_int;
    const float rr = live ? r[row] : 0.0f;
    const float er = live ? e_old[row] : 0.0f;
    const float acc = row_dot<float, U, LAYOUT>(cs, slice_ptr, idx, w, BufGather<float>(e_old, ncols), slice, lane, len);
    if (live) e_new[row] = er + dt * (acc - rr);
}

// Lu (and, with f, max |Lu - f| into slot).
template <int WAVES, int U, int LAYOUT>
__global__ __launch_bounds__(WAVES * 64) void k_apply_f64(
    const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ slice_len, const int32_t *__restrict__ idx,
    const double *__restrict__ w, const uint16_t *__restrict__ lmeta, int64_t nslices, int64_t N_int, int64_t ncols,
    const double *__restrict__ u, double *__restrict__ Lu, const double *__restrict__ f,
    unsigned long long *res_slot, int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (slice < nslices) {
        const int len = slice_len[slice];
        const double acc = RowDot<double, U, LAYOUT>::run(idx, w, BufGather<double>(u, ncols), slice_ptr[slice], lane, len);
        const int64_t row = lane_row<false>(lmeta, slice, lane, len).row;
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
    const double *__restrict__ w, int64_t nslices, int64_t N_int, int64_t ncols, const double *__restrict__ f,
    const double *__restrict__ u, float *__restrict__ r32, float *__restrict__ e0, unsigned long long *res_slot,
    int order) {
    const int64_t slice = slice_index<WAVES>(nslices, order);
    const int lane = threadIdx.x & 63;
    unsigned long long bits = 0;
    if (slice < nslices) {
        const int len = slice_len[slice];
        const double acc = RowDot<double, U, LAYOUT>::run(idx, w, BufGather<double>(u, ncols), slice_ptr[slice], lane, len);
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

// The same over the shapes of the sweeps that read codes (LAYOUT 3 to 6, and
// 7: layout 6 with each lane's loads masked past its row's length, for FP64
// sweeps of an operator with a lane order).
template <template <int, int, int> class F, bool MASKABLE, typename... A>
hipError_t dispatch_codes(const SweepCfg &c, bool masked, A &&...a) {
#define RBF_CASE(WV, UN) \
    if (c.waves_per_block == WV && c.unroll == UN) {                                                \
        if constexpr (MASKABLE)                                                                     \
            if (masked && c.temporal && c.pipeline) return F<WV, UN, 7>::run(a...);                 \
        if (c.temporal) return c.pipeline ? F<WV, UN, 6>::run(a...) : F<WV, UN, 5>::run(a...);      \
        return c.pipeline ? F<WV, UN, 4>::run(a...) : F<WV, UN, 3>::run(a...);                       \
    }
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
                          double dt, unsigned long long *slot, int remap, int64_t s0, int64_t ns) {
        if (ns <= 0) return hipSuccess;
        const unsigned g = grid1d(ns, WV);
        const Codes cs = codes_of(e);
        if (slot)
            hipLaunchKernelGGL((k_sweep_f64<WV, UN, LY, true>), dim3(g), dim3(WV * 64), 0, s, e.slice_ptr,
                               e.slice_len, e.idx, e.w, cs, e.lmeta, s0, ns, N_int, e.ncols, f, uo, un, dt, slot,
                               remap);
        else
            hipLaunchKernelGGL((k_sweep_f64<WV, UN, LY, false>), dim3(g), dim3(WV * 64), 0, s, e.slice_ptr,
                               e.slice_len, e.idx, e.w, cs, e.lmeta, s0, ns, N_int, e.ncols, f, uo, un, dt, slot,
                               remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct SweepF32 {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const float *r, const float *eo, float *en,
                          float dt, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_sweep_f32<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w32, codes_of(e), e.nslices, N_int, e.ncols, r, eo, en, dt,
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
                           e.slice_ptr, e.slice_len, e.idx, e.w, e.lmeta, e.nslices, N_int, e.ncols, u, Lu, f, slot,
                           remap);
        return hipGetLastError();
    }
};

template <int WV, int UN, int LY>
struct OuterRes {
    static hipError_t run(hipStream_t s, const Ell &e, int64_t N_int, const double *f, const double *u, float *r32,
                          float *e0, unsigned long long *slot, int remap) {
        if (!e.nslices) return hipSuccess;
        hipLaunchKernelGGL((k_outer_residual<WV, UN, LY>), dim3(grid1d(e.nslices, WV)), dim3(WV * 64), 0, s,
                           e.slice_ptr, e.slice_len, e.idx, e.w, e.nslices, N_int, e.ncols, f, u, r32, e0, slot, remap);
        return hipGetLastError();
    }
};

}  // namespace

inline int order_flags(const SweepCfg &c, int parity) { return c.xcd_remap | ((c.zigzag && (parity & 1)) ? 2 : 0); }

hipError_t launch_sweep_f64(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *f,
                            const double *u_old, double *u_new, double dt, unsigned long long *res_slot,
                            int parity, int64_t s0, int64_t ns) {
    if (s0 < 0 || s0 > e.nslices) return hipErrorInvalidValue;
    if (ns < 0 || s0 + ns > e.nslices) ns = e.nslices - s0;
    if (use_codes(c, e))
        return dispatch_codes<SweepF64, true>(c, e.lmeta != nullptr, s, e, N_int, f, u_old, u_new, dt, res_slot,
                                              order_flags(c, parity), s0, ns);
    return dispatch_shape<SweepF64>(c, e.layout, s, e, N_int, f, u_old, u_new, dt, res_slot, order_flags(c, parity),
                                    s0, ns);
}

hipError_t launch_sweep_f32(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const float *r,
                            const float *e_old, float *e_new, float dt, int parity) {
    if (use_codes(c, e))
        return dispatch_codes<SweepF32, false>(c, false, s, e, N_int, r, e_old, e_new, dt, order_flags(c, parity));
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

}  // namespace rbf
