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
//      LDS, every lane takes the winner and eliminates;
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
//   5. Cholesky of C, one row per lane, with the reduced right-hand side as
//      an extra row (its multipliers are L^{-1} r); backward substitution by
//      per-step reductions; w = v + G z back in support order.
// Singular systems: an LU pivot at most 2^-45 max|P| (the supports cannot fix
// the monomials: too few or degenerate nodes) or a Cholesky pivot at most
// 2^-45 max C_ii (e.g. duplicate nodes) report ESINGULAR.
#pragma once

#include "weights_common.h"

namespace rbf {
namespace {

constexpr int kLT = 256;        // threads per workgroup
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

__host__ __device__ inline LuLayout lu_layout(int n, int M, int B) {
    LuLayout L{};
    L.n = n;
    L.M = M;
    L.K = n - M;
    L.M4 = (M + 3) & ~3;
    L.nJ = (L.K + 1 + 15) / 16;
    L.ldx = L.K + 1;          // [X v1], row-major (M rows)
    L.lda = L.M4 + 1;         // block of A: odd stride, the 16 rows of a fragment in distinct banks
    L.ldst = 16 * L.nJ;       // staging rows of C_aug
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
    L.vec = o;                 // rhs [B], L^{-1} r [B], z [B], diag L [B]
    o += 4 * B;
    L.misc = o;
    o += 64;
    L.xreg = o;                // LU candidate rows, then L1, then [X v1]
    int xr = 2 * kLW * (B + 2);
    if (l1_off(M) + 2 > xr) xr = l1_off(M) + 2;
    if (M * L.ldx > xr) xr = M * L.ldx;
    o += xr + (xr & 1);
    L.treg = o;                // block of A, then C_aug staging, then Cholesky columns
    int tr = 16 * L.lda;
    if (16 * L.ldst > tr) tr = 16 * L.ldst;
    if (2 * (B + 2) > tr) tr = 2 * (B + 2);
    o += tr + (tr & 1);
    L.total = o;
    return L;
}

// Lane exchange within each half-wave by ds_swizzle (bit mode: lane ^ X),
// which needs no address registers.
template <int X>
__device__ __forceinline__ double swz_xor(double v) {
    constexpr int pat = 0x1F | (X << 10);
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), pat);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), pat);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Maximum over the wavefront, the same value on every lane.
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, swz_xor<1>(v));
    v = fmax(v, swz_xor<2>(v));
    v = fmax(v, swz_xor<4>(v));
    v = fmax(v, swz_xor<8>(v));
    v = fmax(v, swz_xor<16>(v));
    return fmax(lane_value(v, 0), lane_value(v, 32));
}

// Sum over the wavefront (butterfly within the halves, then the two halves),
// the same value on every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v += swz_xor<1>(v);
    v += swz_xor<2>(v);
    v += swz_xor<4>(v);
    v += swz_xor<8>(v);
    v += swz_xor<16>(v);
    return lane_value(v, 0) + lane_value(v, 32);
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

// P_ij = monomial j at support node i.
template <int DIM>
__device__ __forceinline__ double monomial(const double *y, const int8_t *ex, int i, int j) {
    double p = 1.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        for (int e = 0; e < ex[3 * j + a]; ++e) p *= y[3 * i + a];
    return p;
}

// x[j] -= f * src[j] for j0 <= j < j1 (compile-time bounds once unrolled):
// the reads in chunks of 4, each chunk's reads issued before the previous
// chunk's products, and scheduling fences between chunks, so that only two
// chunks of operands are in registers next to the row.
template <int B>
__device__ __forceinline__ void row_axpy(double (&x)[B], const double *src, double f, int j0, int j1) {
    constexpr int CH = 4;
    double cur[CH], nxt[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) cur[q] = j0 + q < j1 ? src[j0 + q] : 0.0;
#pragma unroll
    for (int c = 0; c < B; c += CH) {
        const int cj = j0 + c;
        if (cj < j1) {
#pragma unroll
            for (int q = 0; q < CH; ++q) nxt[q] = cj + CH + q < j1 ? src[cj + CH + q] : 0.0;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < CH; ++q)
                if (cj + q < j1) x[cj + q] = fma(-f, cur[q], x[cj + q]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < CH; ++q) cur[q] = nxt[q];
        }
    }
}

template <int DIM, int B>
__device__ __forceinline__ void solve_lu_item(const WCtx &cx, const Item &it, double *lds) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t li = it.first;
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(DIM, m);
    const int K = n - M;
    const int S = n + M;
    const LuLayout L = lu_layout(n, M, B);
    double *y = lds + L.y, *b1 = lds + L.b1, *b2 = lds + L.b2, *vec = lds + L.vec, *misc = lds + L.misc;
    int *ipiv = (int *)(lds + L.ints), *inp = ipiv + M;
    double *rhs = vec, *yv = vec + B, *zv = vec + 2 * B, *ldiag = vec + 3 * B;
    double *red = misc;                       // reductions (kLW doubles)
    double *sc = misc + 8;                    // s
    int *wcnt = (int *)(misc + 12);           // non-pivot rows per wavefront
    double *part = misc + 16;                 // backward-solve partial sums [2][2]
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
    double x[B];
    double pmax = 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
        double v = 0.0;
        if (j < M) {
            if (row < n) v = monomial<DIM>(y, ex, row, j);
            else if (row == n) v = b2[j];
        }
        x[j] = v;
        if (row < n) pmax = fmax(pmax, fabs(v));
        if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    const double tinyP = group_max(pmax, t, kLT, red) * 0x1p-45;
    bad = !(s > 0.0);
    bool isfree = row < n;
    int mystep = -1;
    constexpr int SL = B + 2;  // candidate slot: |pivot|, row, row entries 0..B-1
    {
        const double v = isfree ? fabs(x[0]) : -1.0;
        const double wm = wave_max(v);
        const unsigned long long bl = __ballot(v == wm);
        if (lane == __ffsll((unsigned long long)bl) - 1) {
            double *sl = xreg + wave * SL;
            sl[0] = wm;
            sl[1] = (double)row;
#pragma unroll
            for (int j = 0; j < B; ++j) sl[2 + j] = x[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if (k < M && !bad) {
            const double *sb = xreg + (k & 1) * kLW * SL;
            double best = sb[0];
            int bw = 0;
#pragma unroll
            for (int w = 1; w < kLW; ++w) {
                const double v = sb[w * SL];
                if (v > best) {
                    best = v;
                    bw = w;
                }
            }
            if (!(best > tinyP)) {
                bad = true;  // uniform: every thread read the same candidates
            } else {
                const double *u = sb + bw * SL;
                const int prow = (int)u[1];
                const double pv = u[2 + k];
                if (row == prow) {
                    isfree = false;
                    mystep = k;
                }
                if (isfree || row == n) {
                    const double l = x[k] / pv;
                    x[k] = l;
                    row_axpy<B>(x, u + 2, l, k + 1, B);
                }
                if (k + 1 < M) {
                    const double v = isfree ? fabs(x[k + 1]) : -1.0;
                    const double wm = wave_max(v);
                    const unsigned long long bl = __ballot(v == wm);
                    if (lane == __ffsll((unsigned long long)bl) - 1) {
                        double *sl = xreg + (((k + 1) & 1) * kLW + wave) * SL;
                        sl[0] = wm;
                        sl[1] = (double)row;
#pragma unroll
                        for (int j = k + 1; j < B; ++j) sl[2 + j] = x[j];
                    }
                }
                __syncthreads();
            }
        }
    }

    if (!bad) {
        // rows of L1 (multipliers of the pivot rows), pivot and non-pivot row lists
        if (mystep >= 0) {
            ipiv[mystep] = row;
            double *lr = xreg + l1_off(mystep);
#pragma unroll
            for (int j = 0; j + 1 < B; ++j)
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
            for (int i = B - 1; i >= 1; --i) {
                if (i < M) row_axpy<B>(x, xreg + l1_off(i), x[i], 0, i);
            }
        }
        __syncthreads();  // L1 read before [X v1] overwrites it
        if (isfree) {
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (j < M) Xs[j * ldx + rank] = -x[j];
        } else if (row == n) {
#pragma unroll
            for (int j = 0; j < B; ++j)
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
        double xr0[B / 4], xr1[B / 4];
#pragma unroll
        for (int q = 0; q < B / 4; ++q) {
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
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cb = h == 0 ? cb0 : cb1;
                if (cb >= 0) {
                    // identity part A[block, non-pivots] [I 0] as the initial value
                    f64x4 T;
                    const int cc = 16 * cb + l16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = lq + 4 * r;
                        T[r] = (r0 + i < rlim && cc < K) ? phs3<DIM>(y, rowpos[r0 + i], inp[cc]) : 0.0;
                    }
                    const double *ar = at + l16 * lda + lq;
#pragma unroll
                    for (int q = 0; q < B / 4; ++q)
                        if (4 * q < M4)
                            T = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[4 * q], h == 0 ? xr0[q] : xr1[q], T, 0, 0, 0);
                    if (pivb) {
                        // C_aug[a, cb] += [X v1]^T[a-block, block rows] T
#pragma unroll
                        for (int d = 0; d < 6; ++d) {
                            const int a = cb + d;
                            if (a < nJ && (h == 0 || d < 2)) {
                                f64x4 acc = h == 0 ? acc0[d] : acc1[d < 2 ? d : 0];
                                const int ca = 16 * a + l16;
#pragma unroll
                                for (int s4 = 0; s4 < 4; ++s4) {
                                    const int j = r0 + 4 * s4 + lq;
                                    const double xa = (j < M && ca <= K) ? Xs[j * ldx + ca] : 0.0;
                                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, T[s4], acc, 0, 0, 0);
                                }
                                if (h == 0) acc0[d] = acc;
                                else acc1[d < 2 ? d : 0] = acc;
                            }
                        }
                    } else {
                        // rows M + r0 .. : C_aug[r0 / 16, cb] += T (same fragment layout)
                        const int a = r0 / 16;
#pragma unroll
                        for (int d = 0; d < 6; ++d) {
                            if (a == cb + d && (h == 0 || d < 2)) {
                                if (h == 0) acc0[d] += T;
                                else acc1[d < 2 ? d : 0] += T;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- 5. Cholesky of C with the reduced right-hand side as row K
    // r = G^T b1 - G^T A v: X^T b1[pivots] + b1[non-pivots] - C_aug[K, 0..K-1]
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
    // lower tiles of C_aug to one row per lane (rows 0..K), by row blocks
    double x[B];
#pragma unroll
    for (int j = 0; j < B; ++j) x[j] = 0.0;
    double dmax = 0.0;
    if (!bad) {
        double *st = treg;
        const int ldst = L.ldst;
        for (int a = 0; a < nJ; ++a) {
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (cb0 >= 0 && cb0 + d == a) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) st[(lq + 4 * r) * ldst + 16 * cb0 + l16] = acc0[d][r];
                }
            }
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (cb1 >= 0 && cb1 + d == a) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) st[(lq + 4 * r) * ldst + 16 * cb1 + l16] = acc1[d][r];
                }
            }
            __syncthreads();
            if (t >= 16 * a && t < 16 * a + 16 && t <= K) {
                const double *sr = st + (t - 16 * a) * ldst;
#pragma unroll
                for (int j = 0; j < B; ++j) x[j] = j <= t ? sr[j] : 0.0;
                if (t < K) dmax = sr[t];
            }
            __syncthreads();
        }
    }
    const double tinyC = group_max(dmax, t, kLT, red) * 0x1p-45;
    const int ci = t;
    const bool crow = ci <= K;
    if (!bad && ci == K) {
#pragma unroll
        for (int j = 0; j < B; ++j) x[j] = j < K ? rhs[j] - x[j] : 0.0;
    }
    double *colb = treg;  // column k of the updated matrix, double-buffered [2][B + 2]
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if (k < K && !bad) {
            double *cbk = colb + (k & 1) * (B + 2);
            if (crow && ci >= k) cbk[ci] = x[k];
            __syncthreads();
            const double d = cbk[k];
            if (!(d > tinyC)) {
                bad = true;  // uniform
            } else {
                const double lkk = sqrt(d);
                if (t == 0) ldiag[k] = lkk;
                if (crow && ci > k) {
                    const double f = x[k] / d;
                    // columns up to B - 1: those past K hold no row entries
                    // (never read by rows 0..K), so the update stays static
                    row_axpy<B>(x, cbk, f, k + 1, B);
                    x[k] = x[k] / lkk;  // L[ci][k] (row K: (L^{-1} r)_k)
                }
            }
        }
    }
    if (!bad) {
        if (ci == K) {
#pragma unroll
            for (int j = 0; j < B; ++j)
                if (j < K) yv[j] = x[j];
        }
        __syncthreads();
        // L^T z = L^{-1} r: z_k from the column-k products of the rows below
        double zi = 0.0;
#pragma unroll
        for (int k = B - 1; k >= 0; --k) {
            if (k < K) {
                double p = (ci > k && ci < K) ? x[k] * zi : 0.0;
                p = wave_sum(p);
                if (lane == 0 && wave < 2) part[(k & 1) * 2 + wave] = p;
                __syncthreads();
                if (ci == k) zi = (yv[k] - (part[(k & 1) * 2] + part[(k & 1) * 2 + 1])) / ldiag[k];
            }
        }
        if (ci < K) zv[ci] = zi;
        __syncthreads();
    }

    // ---- 6. w = v + G z in support order
    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (bad) {
        for (int k = t; k < n; k += kLT) w[k] = 0.0;
        if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
    } else {
        const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
        for (int q = t; q < K; q += kLT) w[inp[q]] = zv[q] / s2;
        for (int j = t; j < M; j += kLT) {
            const double *xr = Xs + j * ldx;
            double a0 = xr[K], a1 = 0.0;
            int q = 0;
            for (; q + 1 < K; q += 2) {
                a0 = fma(xr[q], zv[q], a0);
                a1 = fma(xr[q + 1], zv[q + 1], a1);
            }
            if (q < K) a0 = fma(xr[q], zv[q], a0);
            w[ipiv[j]] = (a0 + a1) / s2;
        }
    }
    __syncthreads();
}

template <int DIM, int B>
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
        solve_lu_item<DIM, B>(cx, items[q], lds_ns);
    }
}

}  // namespace

// One compiled size: kernel handle and launch (defined by RBF_NS_INSTANCE in
// the instance files).
#define RBF_NS_DECL(D, BB)                                                                                    \
    const void *ns_kernel_##D##_##BB();                                                                       \
    hipError_t ns_launch_##D##_##BB(hipStream_t s, int grid, size_t lds_bytes, int64_t N, const double *xyz,     \
                                    const int32_t *sten, const int16_t *nrow, int32_t n_max, const int32_t *rows, \
                                    const int8_t *mrow, const int8_t *type, const double *normals, double *w_out,  \
                                    DevStatus *status, const void *items, int64_t nitems, int32_t *counter);
#define RBF_NS_INSTANCE(D, BB)                                                                                \
    const void *ns_kernel_##D##_##BB() { return (const void *)k_weights_ns<D, BB>; }                          \
    hipError_t ns_launch_##D##_##BB(hipStream_t s, int grid, size_t lds_bytes, int64_t N, const double *xyz,     \
                                    const int32_t *sten, const int16_t *nrow, int32_t n_max, const int32_t *rows, \
                                    const int8_t *mrow, const int8_t *type, const double *normals, double *w_out,  \
                                    DevStatus *status, const void *items, int64_t nitems, int32_t *counter) {      \
        WCtx cx{D, N, xyz, sten, nrow, n_max, rows, mrow, w_out, type, normals, nullptr, 0, 0, status};          \
        hipLaunchKernelGGL((k_weights_ns<D, BB>), dim3(grid), dim3(kLT), lds_bytes, s, cx, (const Item *)items, \
                           nitems, counter);                                                                     \
        return hipGetLastError();                                                                                \
    }
#define RBF_NS_SIZES(X) X(2, 16) X(2, 24) X(2, 40) X(2, 64) X(3, 24) X(3, 40) X(3, 64) X(3, 88)

}  // namespace rbf
