// Null-space weight kernel templates (included by the per-size instance
// files k_weights_ns_*.hip, compiled in parallel; the host side is in
// k_weights_ns.hip).
// Null-space solver for the larger RBF-FD weight systems (Sec. II: the
// augmented system [A P; P^T 0][w; lambda] = [L Phi; L p] with phi = r^3 and
// the M monomials of degree <= m, n support nodes, K = n - M).
//
// Fundamental null-space basis from an LU factorisation of P with partial
// pivoting: with the rows of P reordered pivots first, P = [L1; L2] U, every
// w with P^T w = Lp is w = v + G z, where (in that row order)
//     G = [X; I_K],  X = -L1^{-T} L2^T,   v = [v1; 0],  v1 = L1^{-T} U^{-T} Lp,
// and z solves the reduced system
//     C z = G^T (L Phi - A v),   C = G^T A G.
// r^3 is conditionally positive definite of order 2, so for m >= 1 (all
// linear monomials in P) C is symmetric positive definite: Cholesky applies.
// Partial pivoting keeps |L| <= 1, and X stays small on RBF-FD supports
// (|X| ~ 3, cond C ~ 1e3 for n = 2M).  The result is the system's unique
// solution computed in another order than Gaussian elimination: it agrees
// with the elimination to ~1e-12 relative, not bitwise.
//
// One 256-thread workgroup per system, two per CU (LDS under half a CU):
//   1. local coordinates y, the right-hand sides;
//   2. LU of P, one row per lane (its M entries in registers), with L p as an
//      extra row that is eliminated but never chosen as pivot: its
//      multipliers are U^{-T} Lp.  Per column one barrier: each wavefront
//      posts its best candidate row (largest |entry|, lowest row on ties) to
//      LDS, every lane takes the winner and eliminates within the column's
//      panel of kPW columns; at a panel's end the columns past it take the
//      panel's kPW updates at once (U12 = L11^{-1} A12 by one lane per
//      column, then every free row subtracts l_k U12[k] in pivot order: the
//      products and their order of the column-by-column elimination);
//   3. every non-pivot row (and the extra row) solves L1^T xi = its
//      multipliers with the rows of L1 from LDS: -xi is its column of X
//      (the extra row's xi is v1); [X v1] goes to LDS;
//   4. by row blocks of 16 of the reordered A (pivot rows, then the others):
//      T = A[block, pivots] [X v1] + A[block, non-pivots] [I 0] on FP64
//      matrix cores (v_mfma_f64_16x16x4f64; [X v1] in registers, the block of
//      A generated in LDS), then C_aug += [X v1]^T[., block] T for pivot
//      blocks, or C_aug[block, .] += T for the others.  C_aug = [G v]^T A
//      [G v] (lower tiles, in registers) holds C and, in its last row,
//      (G^T A v)^T;
//   5. Cholesky of C on those tiles, with the reduced right-hand side as an
//      extra row (its multipliers are L^{-1} r): per column block its owning
//      wavefront factors the block in registers (DPP and lane permutes, no
//      barrier), then every wavefront updates its later blocks by L_ap L_bp^T
//      on the matrix cores; backward substitution by blocks from the same
//      tiles; w = v + G z back in support order.
// Singular systems: an LU pivot at most 2^-45 max|P| (the supports cannot fix
// the monomials: too few or degenerate nodes) or a Cholesky pivot at most
// 2^-45 max C_ii (e.g. duplicate nodes) report ESINGULAR.
#pragma once

#include "weights_common.h"

namespace rbf {
namespace {

constexpr int kLT = 256;        // threads per workgroup
constexpr int kPW = 8;          // LU panel width (columns updated per pivot step)
constexpr int kLW = kLT / 64;   // wavefronts

// v_mfma_f64_16x16x4f64 (D = A B + C; A 16x4, B 4x16): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; element r of its result is
// D[l / 16 + 4 r][l % 16].
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Start of row i of L1 (rows of even length, so paired reads stay aligned).
__host__ __device__ inline int l1_off(int i) { return i * (i - 1) / 2 + i / 2; }

// LDS layout of one system, offsets in doubles.
struct LuLayout {
    int n, M, K, M4, nJ, ldx, lda, ldst;
    int y, b1, b2, ints, vec, misc, xreg, treg, total;
};

__host__ __device__ inline LuLayout lu_layout(int n, int M, int MB, int KB) {
    LuLayout L{};
    L.n = n;
    L.M = M;
    L.K = n - M;
    L.M4 = (M + 3) & ~3;
    L.nJ = (L.K + 1 + 15) / 16;
    L.ldx = L.K + 1;          // [X v1], row-major (M rows)
    L.lda = L.M4 + 1;         // block of A: odd stride, the 16 rows of a fragment in distinct banks
    L.ldst = 16 * L.nJ;       // 16 ldst: one column block's L tiles
    int o = 0;
    L.y = o;
    o += 3 * n + (n & 1);
    L.b1 = o;
    o += n + (n & 1);
    L.b2 = o;
    o += M + (M & 1);
    L.ints = o;                // int32 pivot rows [M], non-pivot rows [K]
    o += (n + 1) / 2 + 1;
    o += o & 1;
    L.vec = o;                 // rhs [KB], L^{-1} r [KB], z [KB], 1 / diag L [KB]
    o += 4 * KB;
    L.misc = o;
    o += 64;
    L.xreg = o;                // LU candidate rows, then L1, then [X v1]
    int xr = 8 * kLW + 2 * kLW * MB;
    if (MB > kPW) xr += kPW * kPW + kPW * (MB - kPW + 2);  // a panel's L11 and U12 (LU in kPW-column panels)
    if (l1_off(M) + 2 > xr) xr = l1_off(M) + 2;
    if (M * L.ldx > xr) xr = M * L.ldx;
    o += xr + (xr & 1);
    L.treg = o;                // block of A, then a column block's L tiles
    int tr = 16 * L.lda;
    if (16 * L.ldst > tr) tr = 16 * L.ldst;
    if (2 * (KB + 2) > tr) tr = 2 * (KB + 2);
    o += tr + (tr & 1);
    L.total = o;
    return L;
}

// Lane exchange inside rows of 16 lanes by DPP (quad permutations and row
// mirrors): ALU latency, no LDS round trip.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16

__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Value of lane src (any lane of the wavefront) by the LDS crossbar (no LDS
// memory).  Every lane must be active.
__device__ __forceinline__ double lane_perm(double v, int src) {
    const int a = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Value of lane N of the calling lane's row of 16 (DPP row_newbcast, one
// 64-bit move).  Every lane of the row must be active.
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + N, 0xF, 0xF, false);
}
__device__ __forceinline__ double row_bcast(double v, int n) {  // n a constant once unrolled
    switch (n) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
    }
}

// Maximum over the wavefront, the same value on every lane: within each row
// of 16 (pairs, quads, halves, rows), then the four rows.
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppMirror>(v));
    return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// A_ik = |y_i - y_k|^3 (the cubic polyharmonic spline between two support nodes).
template <int DIM>
__device__ __forceinline__ double phs3(const double *y, int i, int k) {
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double t = y[3 * i + a] - y[3 * k + a];
        d2 = fma(t, t, d2);
    }
    const double r = sqrt(d2);
    return (r * r) * r;
}

// A double in LDS (address space 3): volatile stores through it stay single
// ds_write_b64 (not paired, so no register copies for the pair's operands).
typedef __attribute__((address_space(3))) double lds_f64;

// An offset the compiler cannot fold into later address arithmetic: the LDS
// base of a row is computed once, and the static offsets of its elements fit
// the instructions' offset fields.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// x[j] -= f * src[j] for j0 <= j < j1 (compile-time bounds once unrolled;
// src 16-byte aligned and readable up to the even index past j1 - 1).  The
// reads are 16-byte pairs in chunks of two pairs, D chunks ahead of the
// products, into D + 1 rotating slots, with scheduling fences between chunks
// so the compiler neither hoists every read of the row (registers) nor sinks
// them next to their use (LDS latency).
template <int B, int D>
__device__ __forceinline__ void row_axpy(double (&x)[B], const double *src, double f, int j0, int j1) {
    constexpr int CP = 2, NS = D + 1, NC = (B / 2 + CP - 1) / CP + 1;
    const double2 *s2 = reinterpret_cast<const double2 *>(src);
    const int p0 = j0 / 2, p1 = (j1 + 1) / 2;
    double2 buf[NS][CP];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int q = 0; q < CP; ++q) {
            const int pp = p0 + c * CP + q;
            buf[c][q] = pp < p1 ? s2[pp] : double2{0.0, 0.0};
        }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int cp = p0 + c * CP;
        if (cp < p1) {
#pragma unroll
            for (int q = 0; q < CP; ++q) {
                const int pp = cp + D * CP + q;
                if (pp < p1) buf[(c + D) % NS][q] = s2[pp];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < CP; ++q) {
                const int j = 2 * (cp + q);
                const double2 v = buf[c % NS][q];
                if (j >= j0 && j < j1 && j < B) x[j] = fma(-f, v.x, x[j]);
                if (j + 1 >= j0 && j + 1 < j1 && j + 1 < B) x[j + 1] = fma(-f, v.y, x[j + 1]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Exponents of the first 96 monomials in the graded order of make_exponents
// (degree, then the x exponent descending, then the y exponent descending),
// as a compile-time table: indexed from fully unrolled loops, every lookup
// folds to a constant.
struct MonoExp {
    signed char e[96][3];
};

template <int DIM>
constexpr MonoExp make_mono_exp() {
    MonoExp t{};
    int c = 0;
    for (int deg = 0; c < 96; ++deg) {
        if (DIM == 1) {
            t.e[c][0] = (signed char)deg;
            ++c;
        } else if (DIM == 2) {
            for (int e0 = deg; e0 >= 0 && c < 96; --e0, ++c) {
                t.e[c][0] = (signed char)e0;
                t.e[c][1] = (signed char)(deg - e0);
            }
        } else {
            for (int e0 = deg; e0 >= 0; --e0)
                for (int e1 = deg - e0; e1 >= 0 && c < 96; --e1, ++c) {
                    t.e[c][0] = (signed char)e0;
                    t.e[c][1] = (signed char)e1;
                    t.e[c][2] = (signed char)(deg - e0 - e1);
                }
        }
    }
    return t;
}

template <int DIM>
constexpr MonoExp kMonoExp = make_mono_exp<DIM>();

template <int DIM, int MB, int KB>
__device__ __forceinline__ void solve_lu_item(const WCtx &cx, const Item &it, double *lds) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: scalar branches on it
    const int64_t li = it.first;
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(DIM, m);
    const int K = n - M;
    const int S = n + M;
    const LuLayout L = lu_layout(n, M, MB, KB);
    double *y = lds + L.y, *b1 = lds + L.b1, *b2 = lds + L.b2, *vec = lds + L.vec, *misc = lds + L.misc;
    int *ipiv = (int *)(lds + L.ints), *inp = ipiv + M;
    double *rhs = vec, *yv = vec + KB, *zv = vec + 2 * KB, *ldiag = vec + 3 * KB;  // ldiag: 1 / L[k][k]
    double *red = misc;                       // reductions (kLW doubles)
    double *sc = misc + 8;                    // s
    int *wcnt = (int *)(misc + 12);           // non-pivot rows per wavefront
    int8_t *ex = (int8_t *)(misc + 32);       // monomial exponents (84 x 3 bytes)
    double *xreg = lds + L.xreg, *treg = lds + L.treg;

    // ---- 1. local coordinates and right-hand sides
    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < DIM; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) make_exponents(DIM, m, ex);
    local_coords(cx, c, n, y, sc, t, kLT, red);
    __syncthreads();
    const double s = sc[0];
    for (int k = t; k < n; k += kLT) b1[k] = entry(k, S, n, M, S, DIM, y, ex, op, nv);
    for (int j = t; j < M; j += kLT) b2[j] = entry(n + j, S, n, M, S, DIM, y, ex, op, nv);
    __syncthreads();

    // ---- 2. LU of P with partial pivoting, one row per lane; row n = Lp
    const int row = t;
    const int ldx = L.ldx;
    double *Xs = xreg;
    int rank = -1;
    bool bad = false;
    {
    double x[MB];
    double pmax = 0.0;
    {
        // powers of the row's coordinates, then products in the graded order
        const int rr = row < n ? row : 0;
        constexpr int E = 6;  // m <= 6; entries past M are discarded
        double pw[DIM][E + 1];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double ya = y[3 * rr + a];
            pw[a][0] = 1.0;
#pragma unroll
            for (int e = 1; e <= E; ++e) pw[a][e] = pw[a][e - 1] * ya;
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            double mj = pw[0][min((int)kMonoExp<DIM>.e[j][0], E)];
#pragma unroll
            for (int a = 1; a < DIM; ++a) mj *= pw[a][min((int)kMonoExp<DIM>.e[j][a], E)];
            const double v = j < M ? (row < n ? mj : (row == n ? b2[j] : 0.0)) : 0.0;
            x[j] = v;
            pmax = fmax(pmax, row < n ? fabs(v) : 0.0);
        }
    }
    const double tinyP = group_max(pmax, t, kLT, red) * 0x1p-45;
    bad = !(s > 0.0);
    bool isfree = row < n;
    int mystep = -1;
    // candidates, double-buffered: per wavefront a header (|pivot|, row, -,
    // 1 / pivot) and the row's entries past the pivot column; the
    // posting lane divides while its row stores drain, off the step's path
    double *hdr = xreg;                    // [2][kLW][4]
    double *slots = xreg + 8 * kLW;        // [2][kLW][MB]
    auto post = [&](int k1, double v) __attribute__((always_inline)) {  // candidate for column k1: |x[k1]| or -1
        const double wm = wave_max(v);
        const unsigned long long bl = __ballot(v == wm);
        if (wm < 0.0) {
            // no candidate row on this wavefront: only the header, which never wins
            if (lane == 0) hdr[((k1 & 1) * kLW + wave) * 4] = wm;
        } else if (lane == __ffsll((unsigned long long)bl) - 1) {
            // one lane writes: single stores straight from the row registers
            volatile lds_f64 *h = (volatile lds_f64 *)(hdr + ((k1 & 1) * kLW + wave) * 4);
            h[0] = wm;
            h[1] = (double)row;
            volatile lds_f64 *sl = (volatile lds_f64 *)(slots + opaque(((k1 & 1) * kLW + wave) * MB));
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j > k1 && j < (k1 / kPW) * kPW + kPW) sl[j] = x[j];  // the rest of its panel
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j == k1) h[3] = 1.0 / x[j];
        }
    };
    post(0, isfree ? fabs(x[0]) : -1.0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        if (k < M && !bad) {
            const double *hb = hdr + (k & 1) * kLW * 4;
            double best = hb[0], rpv = hb[3];
            int bw = 0, prow = (int)hb[1];
#pragma unroll
            for (int w = 1; w < kLW; ++w) {
                const double v = hb[4 * w];
                if (v > best) {
                    best = v;
                    bw = w;
                    rpv = hb[4 * w + 3];
                    prow = (int)hb[4 * w + 1];
                }
            }
            if (!(best > tinyP)) {
                bad = true;  // uniform: every thread read the same candidates
            } else {
                const double *u = slots + opaque(((k & 1) * kLW + bw) * MB);
                if (row == prow) {
                    isfree = false;
                    mystep = k;
                }
                const int pe = (k / kPW) * kPW + kPW < MB ? (k / kPW) * kPW + kPW : MB;  // end of k's panel
                if (isfree || row == n) {
                    const double l = x[k] * rpv;
                    x[k] = l;
                    row_axpy<MB, 4>(x, u, l, k + 1, pe);
                }
                if (k + 1 < M && k + 1 < pe) post(k + 1, isfree ? fabs(x[k + 1]) : -1.0);
                __syncthreads();
            }
        }
        if (k % kPW == kPW - 1 && k + 1 < MB && k + 1 < M && !bad) {
            // end of panel p: the columns past it get the panel's kPW updates
            // at once.  The panel's pivot rows post their entries there (A12)
            // and their multipliers of the panel's earlier pivots (L11); one
            // lane per column takes U12 = L11^{-1} A12 in pivot order (the
            // values those rows had when chosen); every free row then
            // subtracts l_k U12[k] for k in pivot order: per element the
            // products and their order of the column-by-column elimination.
            const int p = k / kPW, c0 = kPW * (p + 1), TP = (MB - c0 + 1) & ~1;
            double *L11 = slots + 2 * kLW * MB, *U12 = L11 + kPW * kPW;
            if (mystep >= kPW * p && mystep < c0) {
                const int kk = mystep - kPW * p;
#pragma unroll
                for (int j = 0; j < kPW; ++j)
                    if (j < kk) L11[kk * kPW + j] = x[kPW * p + j];
#pragma unroll
                for (int j = c0; j < MB; ++j) U12[kk * TP + (j - c0)] = x[j];
            }
            __syncthreads();
            for (int j = t; j < TP; j += kLT) {
                double uu[kPW];
#pragma unroll
                for (int q = 0; q < kPW; ++q) uu[q] = U12[q * TP + j];
#pragma unroll
                for (int q = 1; q < kPW; ++q)
#pragma unroll
                    for (int r = 0; r < q; ++r) uu[q] = fma(-L11[q * kPW + r], uu[r], uu[q]);
#pragma unroll
                for (int q = 0; q < kPW; ++q) U12[q * TP + j] = uu[q];
            }
            __syncthreads();
            if (isfree || row == n) {
#pragma unroll
                for (int q = 0; q < kPW; ++q) row_axpy<MB, 4>(x, U12 + q * TP - c0, x[kPW * p + q], c0, MB);
            }
            post(c0, isfree ? fabs(x[c0]) : -1.0);
            __syncthreads();
        }
    }

    if (!bad) {
        // rows of L1 (multipliers of the pivot rows), pivot and non-pivot row lists
        if (mystep >= 0) {
            ipiv[mystep] = row;
            double *lr = xreg + l1_off(mystep);
#pragma unroll
            for (int j = 0; j + 1 < MB; ++j)
                if (j < mystep) lr[j] = x[j];
        }
        const unsigned long long bl = __ballot(isfree);
        if (lane == 0) wcnt[wave] = (int)__popcll(bl);
        __syncthreads();
        int base = 0;
        for (int w = 0; w < wave; ++w) base += wcnt[w];
        if (isfree) {
            rank = base + (int)__popcll(bl & ((1ull << lane) - 1ull));
            inp[rank] = row;
        }
        // ---- 3. L1^T xi = multipliers (rows of L1 from LDS, right-looking)
        if (wave * 64 <= n) {
#pragma unroll
            for (int i = MB - 1; i >= 1; --i) {
                if (i < M) row_axpy<MB, 4>(x, xreg + opaque(l1_off(i)), x[i], 0, i);
            }
        }
        __syncthreads();  // L1 read before [X v1] overwrites it
        if (isfree) {
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < M) Xs[j * ldx + rank] = -x[j];
        } else if (row == n) {
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if (j < M) Xs[j * ldx + K] = x[j];
        }
        __syncthreads();
    }
    }  // LU rows

    // ---- 4. C_aug = [G v]^T A [G v] by row blocks on matrix cores
    const int nJ = L.nJ, M4 = L.M4, lda = L.lda;
    const int l16 = lane & 15, lq = lane >> 4;
    // column blocks of this wavefront: block w, and for nJ > 4 one of the
    // blocks 4, 5 (paired with the blocks of fewest lower tiles)
    const int cb0 = wave < nJ ? wave : -1;
    const int cb1 = (nJ == 6 && wave == 2) ? 5 : ((nJ >= 5 && wave == 3) ? 4 : -1);
    f64x4 acc0[6], acc1[2];
#pragma unroll
    for (int d = 0; d < 6; ++d) acc0[d] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 2; ++d) acc1[d] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (!bad) {
        double xr0[MB / 4], xr1[MB / 4];
#pragma unroll
        for (int q = 0; q < MB / 4; ++q) {
            const int j = 4 * q + lq;
            const int c0 = 16 * cb0 + l16, c1 = 16 * cb1 + l16;
            xr0[q] = (cb0 >= 0 && j < M && c0 <= K) ? Xs[j * ldx + c0] : 0.0;
            xr1[q] = (cb1 >= 0 && j < M && c1 <= K) ? Xs[j * ldx + c1] : 0.0;
        }
        const int nPB = (M + 15) / 16, nNB = (K + 15) / 16;
        double *at = treg;
        for (int blk = 0; blk < nPB + nNB; ++blk) {
            const bool pivb = blk < nPB;
            const int r0 = pivb ? 16 * blk : 16 * (blk - nPB);
            const int rlim = pivb ? M : K;
            const int *rowpos = pivb ? ipiv : inp;
            {
                const int i = t & 15;
                const bool rv = r0 + i < rlim;
                const int ri = rv ? rowpos[r0 + i] : 0;
                for (int j = t >> 4; j < M4; j += kLT / 16)
                    at[i * lda + j] = (rv && j < M) ? phs3<DIM>(y, ri, ipiv[j]) : 0.0;
            }
            __syncthreads();
            // T = A[block, pivots] [X v1] + A[block, non-pivots] [I 0] for both
            // column blocks, the identity part as the initial value; the two
            // accumulation chains interleaved, one A-block read for both
            const int cc0 = 16 * cb0 + l16, cc1 = 16 * cb1 + l16;
            f64x4 T0 = {0.0, 0.0, 0.0, 0.0}, T1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = lq + 4 * r;
                const bool rv = r0 + i < rlim;
                const int ri = rv ? rowpos[r0 + i] : 0;
                if (cb0 >= 0) T0[r] = (rv && cc0 < K) ? phs3<DIM>(y, ri, inp[cc0]) : 0.0;
                if (cb1 >= 0) T1[r] = (rv && cc1 < K) ? phs3<DIM>(y, ri, inp[cc1]) : 0.0;
            }
            const double *ar = at + l16 * lda + lq;
            if (cb1 >= 0) {
#pragma unroll
                for (int q = 0; q < MB / 4; ++q)
                    if (4 * q < M4) {
                        const double av = ar[4 * q];
                        T0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xr0[q], T0, 0, 0, 0);
                        T1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xr1[q], T1, 0, 0, 0);
                    }
            } else if (cb0 >= 0) {
#pragma unroll
                for (int q = 0; q < MB / 4; ++q)
                    if (4 * q < M4) T0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[4 * q], xr0[q], T0, 0, 0, 0);
            }
            if (pivb) {
                // C_aug[a, cb] += [X v1]^T[a-block, block rows] T, the tiles'
                // chains interleaved
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const int j = r0 + 4 * s4 + lq;
                    const bool jv = j < M;
#pragma unroll
                    for (int d = 0; d < 6; ++d) {
                        const int a = cb0 + d;
                        if (cb0 >= 0 && a < nJ) {
                            const int ca = 16 * a + l16;
                            const double xa = (jv && ca <= K) ? Xs[j * ldx + ca] : 0.0;
                            acc0[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, T0[s4], acc0[d], 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const int a = cb1 + d;
                        if (cb1 >= 0 && a < nJ) {
                            const int ca = 16 * a + l16;
                            const double xa = (jv && ca <= K) ? Xs[j * ldx + ca] : 0.0;
                            acc1[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, T1[s4], acc1[d], 0, 0, 0);
                        }
                    }
                }
            } else {
                // rows M + r0 .. : C_aug[r0 / 16, cb] += T (same fragment layout)
                const int a = r0 / 16;
#pragma unroll
                for (int d = 0; d < 6; ++d)
                    if (cb0 >= 0 && a == cb0 + d) acc0[d] += T0;
#pragma unroll
                for (int d = 0; d < 2; ++d)
                    if (cb1 >= 0 && a == cb1 + d) acc1[d] += T1;
            }
            __syncthreads();
        }
    }

    // ---- 5. Cholesky of C_aug's leading K x K block with the reduced
    // right-hand side r = G^T b1 - G^T A v as row K (its multipliers are
    // L^{-1} r), on the tiles the matrix cores left in registers: tile (a, b)
    // belongs to the wavefront of column block b, lane l element e holding
    // row 16 a + l / 16 + 4 e, column 16 b + l % 16.  Per column block p the
    // owner factors the block's 16 columns inside the wavefront (column k
    // reaches each row of 16 lanes by DPP, row k of the diagonal tile by a
    // lane permute: no barrier), stages the block's L tiles in LDS, and after
    // one barrier every wavefront subtracts L_ap L_bp^T from its tiles (a, b),
    // b > p, on the matrix cores.  Then L^T z = L^{-1} r by blocks, from p =
    // nJ - 1 down, each owner with its own tiles.
    int *cflag = (int *)(misc + 16);  // a pivot failed in some owner's block
    if (!bad && t < K) {
        double a0 = 0.0, a1 = 0.0;
        int j = 0;
        for (; j + 1 < M; j += 2) {
            a0 = fma(Xs[j * ldx + t], b1[ipiv[j]], a0);
            a1 = fma(Xs[(j + 1) * ldx + t], b1[ipiv[j + 1]], a1);
        }
        if (j < M) a0 = fma(Xs[j * ldx + t], b1[ipiv[j]], a0);
        rhs[t] = (a0 + a1) + b1[inp[t]];
    }
    if (t == 0) *cflag = 0;
    __syncthreads();
    double *stg = treg;  // L tiles (a, p), a > p, of the current block: column-major 16 x 16 at 256 (a - p)
    // row K := r_j - C_aug[K][j] for j < K, 0 past it; the largest diagonal
    double dmax = 0.0;
    auto prep = [&](auto &T, int cb) __attribute__((always_inline)) {
        constexpr int NT = sizeof(T) / sizeof(T[0]);
        if (cb < 0) return;
#pragma unroll
        for (int d = 0; d < NT; ++d)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = 16 * (cb + d) + lq + 4 * r, gj = 16 * cb + l16;
                if (gi == K) T[d][r] = gj < K ? rhs[gj] - T[d][r] : 0.0;
                if (d == 0 && gi == gj && gi < K) dmax = fmax(dmax, T[d][r]);
            }
    };
    if (!bad) {
        prep(acc0, cb0);
        prep(acc1, cb1);
    }
    const double tinyC = group_max(dmax, t, kLT, red) * 0x1p-45;
    // in-wavefront factorization of column block cb (diagonal tile T[0]);
    // L's row K multipliers go to yv, 1 / L[k][k] to ldiag
    // Step k subtracts C[i][k] C[k][j] / d from every element of the block's
    // columns j > k (lanes of other columns take a zero factor; the upper
    // half of the diagonal tile is updated too, and never read again), and
    // the division of column k by sqrt(d) waits to the block's end: no later
    // step of the block reads column k.
    auto factor = [&](auto &T, int cb) __attribute__((always_inline)) {
        constexpr int NT = sizeof(T) / sizeof(T[0]);
        double myrd = 1.0;  // 1 / d of this lane's column
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int gk = 16 * cb + k;
            if (gk < K && !bad) {
                const double d = lane_value(T[0][k / 4], (k % 4) * 16 + k);
                if (!(d > tinyC)) {
                    bad = true;  // uniform in the wavefront
                } else {
                    const double rd = 1.0 / d;
                    const double cj = lane_perm(T[0][k / 4], (k % 4) * 16 + l16);  // C[k][j]
                    const double cjr = l16 > k ? cj * rd : 0.0;
                    myrd = l16 == k ? rd : myrd;
#pragma unroll
                    for (int dd = 0; dd < NT; ++dd)
                        if (cb + dd < nJ) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) T[dd][r] = fma(-row_bcast(T[dd][r], k), cjr, T[dd][r]);
                        }
                }
            }
        }
        if (bad) {
            if (lane == 0) *cflag = 1;
            return;
        }
        const double myrl = sqrt(myrd);  // 1 / L[j][j]
        if (lq == 0 && 16 * cb + l16 < K) ldiag[16 * cb + l16] = myrl;
#pragma unroll
        for (int dd = 0; dd < NT; ++dd)
            if (cb + dd < nJ) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T[dd][r] *= myrl;
                    const int gi = 16 * (cb + dd) + lq + 4 * r, gj = 16 * cb + l16;
                    if (gi == K && gj < K) yv[gj] = T[dd][r];
                    if (dd > 0) stg[(dd * 16 + l16) * 16 + lq + 4 * r] = T[dd][r];
                }
            }
    };
    // tiles (a, cb), a >= cb > p: T -= L_ap L_cb,p^T (A and B fragments read
    // alike: lane l takes L[l % 16][4 s + l / 16] of its tile)
    auto trail = [&](auto &T, int cb, int p) __attribute__((always_inline)) {
        constexpr int NT = sizeof(T) / sizeof(T[0]);
        if (cb <= p) return;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const double bv = stg[((cb - p) * 16 + 4 * s4 + lq) * 16 + l16];
#pragma unroll
            for (int dd = 0; dd < NT; ++dd)
                if (cb + dd < nJ) {
                    const double av = -stg[((cb + dd - p) * 16 + 4 * s4 + lq) * 16 + l16];
                    T[dd] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, T[dd], 0, 0, 0);
                }
        }
    };
    for (int p = 0; p < nJ && 16 * p < K; ++p) {
        if (!bad) {
            if (cb0 == p) factor(acc0, cb0);
            else if (cb1 == p) factor(acc1, cb1);
        }
        __syncthreads();
        bad = bad || *cflag != 0;
        if (!bad) {
            trail(acc0, cb0, p);
            trail(acc1, cb1, p);
        }
        __syncthreads();  // staging rewritten by the next block's owner
    }
    // L^T z = L^{-1} r: block p's owner takes s = y_p - sum_{a > p} L_ap^T z_a
    // from its tiles, then solves with its diagonal tile from k = 15 down
    auto bsub = [&](auto &T, int cb) __attribute__((always_inline)) {
        constexpr int NT = sizeof(T) / sizeof(T[0]);
        double part = 0.0;
#pragma unroll
        for (int dd = 1; dd < NT; ++dd)
            if (cb + dd < nJ) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gi = 16 * (cb + dd) + lq + 4 * r;
                    part = fma(T[dd][r], gi < K ? zv[gi] : 0.0, part);
                }
            }
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        const int gj = 16 * cb + l16;
        double sj = (gj < K ? yv[gj] : 0.0) - part;
#pragma unroll
        for (int k = 15; k >= 0; --k) {
            const int gk = 16 * cb + k;
            if (gk < K) {
                const double zk = lane_value(sj, k) * ldiag[gk];
                const double lkj = lane_perm(T[0][k / 4], (k % 4) * 16 + l16);  // L[k][j], j < k
                sj = l16 < k ? fma(-lkj, zk, sj) : sj;
                if (lane == 0) zv[gk] = zk;
            }
        }
    };
    if (!bad) {
        for (int p = nJ - 1; p >= 0; --p) {
            if (16 * p < K) {
                if (cb0 == p) bsub(acc0, cb0);
                else if (cb1 == p) bsub(acc1, cb1);
                __syncthreads();
            }
        }
    }

    // ---- 6. w = v + G z in support order
    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (bad) {
        for (int k = t; k < n; k += kLT) w[k] = 0.0;
        if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
    } else {
        const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
        for (int q = t; q < K; q += kLT) w[inp[q]] = zv[q] / s2;
        // pivot rows: v1_j + (X z)_j from the rows of [X v1]
        if (t < M) {
            const double *xr = Xs + t * ldx;
            double a0 = 0.0, a1 = 0.0;
            int j = 0;
            for (; j + 1 < K; j += 2) {
                a0 = fma(xr[j], zv[j], a0);
                a1 = fma(xr[j + 1], zv[j + 1], a1);
            }
            if (j < K) a0 = fma(xr[j], zv[j], a0);
            w[ipiv[t]] = (xr[K] + (a0 + a1)) / s2;
        }
    }
    __syncthreads();
}

template <int DIM, int MB, int KB>
__global__ __launch_bounds__(kLT) __attribute__((amdgpu_waves_per_eu(2))) void k_weights_ns(
    WCtx cx, const Item *__restrict__ items, int64_t nitems, int32_t *counter) {
    extern __shared__ __align__(16) double lds_ns[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t q = s_item;
        __syncthreads();
        if (q >= nitems) return;
        solve_lu_item<DIM, MB, KB>(cx, items[q], lds_ns);
    }
}

}  // namespace

// One compiled size (row arrays of MB entries for the LU, KB for the
// Cholesky): kernel handle and launch, defined by RBF_NS_INSTANCE in the
// instance files.
#define RBF_NS_DECL(D, MBB, KBB)                                                                                \
    const void *ns_kernel_##D##_##MBB##_##KBB();                                                                \
    hipError_t ns_launch_##D##_##MBB##_##KBB(hipStream_t s, int grid, size_t lds_bytes, int64_t N,                \
                                             const double *xyz, const int32_t *sten, const int16_t *nrow,        \
                                             int32_t n_max, const int32_t *rows, const int8_t *mrow,             \
                                             const int8_t *type, const double *normals, double *w_out,          \
                                             DevStatus *status, const void *items, int64_t nitems,              \
                                             int32_t *counter);
#define RBF_NS_INSTANCE(D, MBB, KBB)                                                                            \
    const void *ns_kernel_##D##_##MBB##_##KBB() { return (const void *)k_weights_ns<D, MBB, KBB>; }             \
    hipError_t ns_launch_##D##_##MBB##_##KBB(hipStream_t s, int grid, size_t lds_bytes, int64_t N,                \
                                             const double *xyz, const int32_t *sten, const int16_t *nrow,        \
                                             int32_t n_max, const int32_t *rows, const int8_t *mrow,             \
                                             const int8_t *type, const double *normals, double *w_out,          \
                                             DevStatus *status, const void *items, int64_t nitems,              \
                                             int32_t *counter) {                                                \
        WCtx cx{D, N, xyz, sten, nrow, n_max, rows, mrow, w_out, type, normals, nullptr, 0, 0, status};           \
        hipLaunchKernelGGL((k_weights_ns<D, MBB, KBB>), dim3(grid), dim3(kLT), lds_bytes, s, cx,                  \
                           (const Item *)items, nitems, counter);                                               \
        return hipGetLastError();                                                                                \
    }
// (dimension, MB, KB) of the compiled sizes
#define RBF_NS_SIZES(X) X(2, 16, 16) X(2, 24, 24) X(2, 40, 40) X(2, 64, 64) X(3, 20, 32) X(3, 36, 40) X(3, 56, 64) X(3, 84, 86)

}  // namespace rbf
