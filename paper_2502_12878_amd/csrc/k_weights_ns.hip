// Null-space solver for the larger RBF-FD weight systems (Sec. II: the
// augmented system [A P; P^T 0][w; lambda] = [L Phi; L p] with phi = r^3 and
// the M monomials of degree <= m, n support nodes).
//
// With the Householder QR P = Q [R; 0], Q = H_0 H_1 ... H_{M-1}, the
// constraint P^T w = Lp fixes the part of w in the range of P:
// w = Q [y1; z] with R^T y1 = Lp.  The other K = n - M unknowns solve the
// projected system
//     C z = Z^T (L Phi - A v),   C = Z^T A Z,
// where Z = Q [0; I_K] is an orthonormal basis of null(P^T) and
// v = Q [y1; 0]; then w = v + Z z (lambda is not needed).  r^3 is
// conditionally positive definite of order 2, so for m >= 1 (all linear
// monomials in P) C is positive definite: Cholesky applies.  The result is
// the system's unique solution, computed in another order than Gaussian
// elimination (agreement with the elimination is a tolerance, ~1e-12
// relative on these systems, not bit equality).
//
// One 512-thread workgroup per system; all intermediates on chip:
//   1. local coordinates y, the columns of P and the right-hand side;
//   2. QR: each of the first six wavefronts holds 16 columns of P in
//      registers (lanes: 16 columns x 4 chunks of RC rows); per reflector the
//      owner column's four lanes form it and put it in LDS, one barrier, every
//      other column applies it (dot over its chunks, two shuffles);
//   3. y1 by forward substitution with R^T (one wavefront);
//   4. [Z v] = Q [[0; I_K] | [y1; 0]]: the reflectors applied in reverse to
//      K + 1 columns held in registers, the reflectors read from LDS;
//   5. by row blocks of 16: the block of A generated in LDS, T = A[block, :]
//      [Z v] and C += Z[block, :]^T T on FP64 matrix cores
//      (v_mfma_f64_16x16x4f64), C's tiles accumulated in registers;
//   6. Cholesky of C (trailing updates spread over the workgroup), the two
//      triangular solves, w = v + Z z.
// The register-resident loops run over whole chunks with no per-row branch
// (rows past n are kept at zero), so their LDS reads issue back to back.
// Singular systems: a diagonal entry of R at most 2^-45 max|P| (the supports
// cannot fix the monomials: too few or degenerate nodes) or a Cholesky pivot
// at most 2^-45 max C_ii (e.g. duplicate nodes) report ESINGULAR.
#include <algorithm>

#include "weights_common.h"

namespace rbf {
namespace {

constexpr int kNT = 512;          // threads per workgroup
constexpr int kNW = kNT / 64;     // wavefronts
constexpr int kNsColW = 6;        // wavefronts holding columns (16 each)
constexpr int kNsMaxCTiles = 4;   // C tiles per wavefront

// v_mfma_f64_16x16x4f64 (D = A B + C; A 16x4, B 4x16): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; element r of its result is
// D[l / 16 + 4 r][l % 16] (layout checked on the device).
typedef double f64x4 __attribute__((ext_vector_type(4)));

}  // namespace

// Rows per chunk (each column of P or [Z v] is split over four lanes): the
// register arrays are sized by it at compile time (even, for paired LDS reads).
int ns_rows_per_chunk(int n) {
    const int r = (n + 3) / 4;
    return r <= 12 ? 12 : (r <= 18 ? 18 : (r <= 24 ? 24 : (r <= 42 ? 42 : (r <= 44 ? 44 : 0))));
}

// LDS layout of one system (offsets in doubles), from n, M and the chunk size.
__host__ __device__ NsLayout ns_layout_rc(int n, int M, int RC) {
    NsLayout L{};
    L.n = n;
    L.M = M;
    L.K = n - M;
    L.R = RC;
    int ldz = L.K + 1;
    ldz += ((24 - ldz % 32) + 32) % 32;  // row stride = 24 mod 32 doubles: MFMA fragment reads spread over all banks
    L.ldz = ldz;
    L.nJ = (L.K + 1 + 15) / 16;
    L.nA = (L.K + 15) / 16;
    // factored columns of P: column-major with stride 4 RC + 2 (a double
    // stride of 2 mod 4 puts the 16 columns a chunk reads in distinct banks)
    const int n4 = (n + 3) & ~3, nRp = 4 * RC + 2;
    int o = 0;
    L.big = o;
    o += M * nRp > n4 * ldz ? M * nRp : n4 * ldz;  // factored P (column-major), then [Z v] (row-major, stride ldz)
    L.ablk = o;
    o += 16 * n4;                      // block of A; C (packed lower) in step 6
    L.tblk = o;
    o += 16 * ldz > 8 * RC ? 16 * ldz : 8 * RC;  // block of T; reflector buffers in step 2
    L.y = o;
    o += 3 * n + (n & 1);
    L.b1 = o;
    o += n + (n & 1);
    L.b2 = o;
    o += M + (M & 1);
    L.y1 = o;
    o += M + (M & 1);
    L.rhs = o;
    o += L.K + (L.K & 1);
    L.tau = o;
    o += M + (M & 1);
    L.misc = o;
    o += 64;                           // reductions, scalars, monomial exponents
    L.total = o;
    return L;
}

NsLayout ns_layout_host(int n, int M, int rc) { return ns_layout_rc(n, M, rc); }

bool ns_fits(int n, int M, size_t lds_limit) {
    const int RC = ns_rows_per_chunk(n);
    if (RC == 0 || M < 4 || n - M < 1 || M > 16 * kNsColW || n - M + 1 > 16 * kNsColW) return false;
    const NsLayout L = ns_layout_rc(n, M, RC);
    const int area = L.y - L.ablk;  // A-block and T-block areas
    if (L.K * (L.K + 1) / 2 + L.K > area) return false;
    if (L.nA * (L.nA + 1) / 2 + L.nA > kNsMaxCTiles * kNW) return false;
    return (size_t)L.total * sizeof(double) <= lds_limit;
}

namespace {

// Sum over the four row chunks of a column (lanes l, l ^ 16, l ^ 32, l ^ 48):
// (c0 + c1) + (c2 + c3) on every one of them (addition commutes bitwise).
__device__ __forceinline__ double chunk_sum(double v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// C tile q of the accumulation: the lower tiles (a >= b) by rows, then the
// tiles (a, bK) above the diagonal that hold column K of T (A v).
__device__ __forceinline__ void c_tile(int q, int nA, int bK, int &a, int &b) {
    const int nlow = nA * (nA + 1) / 2;
    if (q < nlow) {
        int r = 0;
        while ((r + 1) * (r + 2) / 2 <= q) ++r;
        a = r;
        b = q - r * (r + 1) / 2;
    } else {
        a = q - nlow;
        b = bK;
    }
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

// Element of the (lower) trailing triangle of a step: q -> (row ii >= col jj).
__device__ __forceinline__ void tri_index(int q, int &ii, int &jj) {
    int r = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    if ((r + 1) * (r + 2) / 2 <= q) ++r;
    if (r * (r + 1) / 2 > q) --r;
    ii = r;
    jj = q - r * (r + 1) / 2;
}

template <int DIM, int RC>
__device__ __forceinline__ void solve_ns_item(const WCtx &cx, const Item &it, double *lds) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t li = it.first;
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(DIM, m);
    const int S = n + M;
    const NsLayout L = ns_layout_rc(n, M, RC);
    const int K = L.K, ldz = L.ldz;
    const int n4 = (n + 3) & ~3, nR = 4 * RC, nRp = nR + 2;
    double *big = lds + L.big, *ablk = lds + L.ablk, *tblk = lds + L.tblk;
    double *y = lds + L.y, *b1 = lds + L.b1, *b2 = lds + L.b2, *y1 = lds + L.y1, *rhs = lds + L.rhs;
    double *tau = lds + L.tau, *misc = lds + L.misc;
    double *red = misc;                            // 8 doubles
    double *sc = misc + 8;                         // scalars: s, tiny_C
    int *flag = (int *)(misc + 12);                // singular flag
    int8_t *ex = (int8_t *)(misc + 16);            // monomial exponents (84 x 3 bytes)

    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < DIM; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) {
        make_exponents(DIM, m, ex);
        *flag = 0;
    }
    local_coords(cx, c, n, y, sc, t, kNT, red);
    __syncthreads();
    const double s = sc[0];
    for (int k = t; k < n; k += kNT) b1[k] = entry(k, S, n, M, S, DIM, y, ex, op, nv);
    for (int j = t; j < M; j += kNT) b2[j] = entry(n + j, S, n, M, S, DIM, y, ex, op, nv);

    // ---- 2. Householder QR of P, columns in registers
    const int ch = lane >> 4;
    const int row0 = ch * RC;
    const int pcol = 16 * wave + (lane & 15);
    const bool hasp = wave < kNsColW && pcol < M;
    double pc[RC];
    double pmax = 0.0;
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int row = row0 + r;
        const double v = (hasp && row < n) ? monomial<DIM>(y, ex, row, pcol) : 0.0;
        pc[r] = v;
        pmax = fmax(pmax, fabs(v));
    }
    const double tinyP = group_max(pmax, t, kNT, red) * 0x1p-45;
    for (int k = 0; k < M; ++k) {
        double *vb = tblk + (k & 1) * nR;
        if (wave == (k >> 4)) {
            double sg = 0.0, al = 0.0;
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                const int row = row0 + r;
                const double xs = row > k ? pc[r] : 0.0;
                sg = fma(xs, xs, sg);
                al = row == k ? pc[r] : al;
            }
            sg = chunk_sum(sg);
            al = chunk_sum(al);
            double beta = al, tk = 0.0, scal = 0.0;
            if (sg != 0.0) {
                const double mu = sqrt(fma(al, al, sg));
                beta = al >= 0.0 ? -mu : mu;
                tk = (beta - al) / beta;
                scal = 1.0 / (al - beta);
            }
            if ((lane & 15) == (k & 15)) {
#pragma unroll
                for (int r = 0; r < RC; r += 2) {
                    const int row = row0 + r;
                    const double v0 = row > k ? pc[r] * scal : (row == k ? 1.0 : 0.0);
                    const double v1 = row + 1 > k ? pc[r + 1] * scal : (row + 1 == k ? 1.0 : 0.0);
                    pc[r] = row > k ? v0 : (row == k ? beta : pc[r]);
                    pc[r + 1] = row + 1 > k ? v1 : (row + 1 == k ? beta : pc[r + 1]);
                    *(double2 *)(vb + row) = double2{v0, v1};
                }
                if (ch == 0) {
                    tau[k] = tk;
                    if (!(fabs(beta) > tinyP)) *flag = 1;
                }
            }
        }
        __syncthreads();
        if (hasp && pcol > k) {
            // the reflector is read twice (dot, then update): reads of one
            // address by the 16 lanes of a chunk are served as one
            const double2 *v2 = (const double2 *)(vb + row0);
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int r = 0; r < RC; r += 2) {
                const double2 q2 = v2[r / 2];
                d0 = fma(q2.x, pc[r], d0);
                d1 = fma(q2.y, pc[r + 1], d1);
            }
            const double f = tau[k] * chunk_sum(d0 + d1);
#pragma unroll
            for (int r = 0; r < RC; r += 2) {
                const double2 q2 = v2[r / 2];
                pc[r] = fma(-f, q2.x, pc[r]);
                pc[r + 1] = fma(-f, q2.y, pc[r + 1]);
            }
        }
    }
    __syncthreads();
    bool bad = *flag != 0 || !(s > 0.0);
    // the factored columns, column-major with stride nRp into big: R on and
    // above the diagonal, the reflectors' entries below it (their unit
    // diagonal and zeros above are implied)
    if (!bad && hasp) {
#pragma unroll
        for (int r = 0; r < RC; r += 2) *(double2 *)(big + pcol * nRp + row0 + r) = double2{pc[r], pc[r + 1]};
    }
    __syncthreads();
    // ---- 3. R^T y1 = b2 (forward substitution, one wavefront)
    if (!bad && wave == 0) {
        double r0 = lane < M ? b2[lane] : 0.0, r1 = lane + 64 < M ? b2[lane + 64] : 0.0;
        for (int i = 0; i < M; ++i) {
            const double ri = i < 64 ? __shfl(r0, i, 64) : __shfl(r1, i - 64, 64);
            const double yi = ri / big[i * nRp + i];
            if (lane == 0) y1[i] = yi;
            if (lane > i && lane < M) r0 = fma(-big[lane * nRp + i], yi, r0);
            if (lane + 64 > i && lane + 64 < M) r1 = fma(-big[(lane + 64) * nRp + i], yi, r1);
        }
    }
    __syncthreads();
    // ---- 4. [Z v] = Q [[0; I_K] | [y1; 0]], columns in registers
    const bool hasz = !bad && wave < kNsColW && pcol <= K;
    double zc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int row = row0 + r;
        double v = 0.0;
        if (hasz && row < n) v = pcol < K ? (row == M + pcol ? 1.0 : 0.0) : (row < M ? y1[row] : 0.0);
        zc[r] = v;
    }
    if (hasz) {
        for (int k = M - 1; k >= 0; --k) {
            // reflector k: stored entries below row k, 1 at row k, 0 above
            const double2 *v2 = (const double2 *)(big + k * nRp + row0);
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int r = 0; r < RC; r += 2) {
                const double2 q2 = v2[r / 2];
                const int row = row0 + r;
                const double a0 = row > k ? q2.x : (row == k ? 1.0 : 0.0);
                const double a1 = row + 1 > k ? q2.y : (row + 1 == k ? 1.0 : 0.0);
                d0 = fma(a0, zc[r], d0);
                d1 = fma(a1, zc[r + 1], d1);
            }
            const double f = tau[k] * chunk_sum(d0 + d1);
#pragma unroll
            for (int r = 0; r < RC; r += 2) {
                const double2 q2 = v2[r / 2];
                const int row = row0 + r;
                const double a0 = row > k ? q2.x : (row == k ? 1.0 : 0.0);
                const double a1 = row + 1 > k ? q2.y : (row + 1 == k ? 1.0 : 0.0);
                zc[r] = fma(-f, a0, zc[r]);
                zc[r + 1] = fma(-f, a1, zc[r + 1]);
            }
        }
    }
    __syncthreads();  // every reflector read before big is overwritten
    if (!bad && wave < kNsColW && pcol < ldz) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int row = row0 + r;
            if (row < n4) big[row * ldz + pcol] = (pcol <= K && row < n) ? zc[r] : 0.0;
        }
    }
    __syncthreads();
    // ---- 5. C = Z^T A Z and Z^T A v on matrix cores, by row blocks of 16
    const int nA = L.nA, bK = K >> 4;
    const int nlow = nA * (nA + 1) / 2;
    const int ntiles = nlow + min(bK, nA);
    f64x4 acc[kNsMaxCTiles];
#pragma unroll
    for (int q = 0; q < kNsMaxCTiles; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int li16 = lane & 15, lk = lane >> 4;
    if (!bad) {
        for (int i0 = 0; i0 < n; i0 += 16) {
            for (int q = t; q < 16 * n4; q += kNT) {
                const int i = q / n4, k = q - i * n4;
                ablk[q] = (i0 + i < n && k < n) ? phs3<DIM>(y, i0 + i, k) : 0.0;
            }
            __syncthreads();
            if (wave < L.nJ) {  // T[block, 16 J .. 16 J + 15], J = wave
                const int col = 16 * wave + li16;
                const int colc = min(col, ldz - 1);
                f64x4 tacc = {0.0, 0.0, 0.0, 0.0};
                const double *ar = ablk + li16 * n4 + lk;
                const double *bc = big + lk * ldz + colc;
                for (int k0 = 0; k0 < n4; k0 += 4) {
                    const double a = ar[k0];
                    const double bb = bc[k0 * ldz];
                    tacc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, col < ldz ? bb : 0.0, tacc, 0, 0, 0);
                }
                if (col < ldz) {  // result element r of lane l: row l / 16 + 4 r, column l % 16
#pragma unroll
                    for (int r = 0; r < 4; ++r) tblk[(lk + 4 * r) * ldz + col] = tacc[r];
                }
            }
            __syncthreads();
#pragma unroll
            for (int qq = 0; qq < kNsMaxCTiles; ++qq) {
                const int q = wave + kNW * qq;
                if (q < ntiles) {
                    int a, b;
                    c_tile(q, nA, bK, a, b);
                    const int ca = 16 * a + li16, cb = 16 * b + li16;
                    const int cac = min(ca, K - 1), cbc = min(cb, K);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int row = i0 + 4 * kk + lk;
                        const double za = big[min(row, n4 - 1) * ldz + cac];
                        const double tb = tblk[(4 * kk + lk) * ldz + cbc];
                        const bool ok = row < n;
                        acc[qq] = __builtin_amdgcn_mfma_f64_16x16x4f64(ok && ca < K ? za : 0.0, ok && cb <= K ? tb : 0.0,
                                                                      acc[qq], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
    }
    // C (packed lower, row i from i(i+1)/2) and column K (Z^T A v) into the
    // A-block area
    double *Cp = ablk, *ck = ablk + K * (K + 1) / 2;
    if (!bad) {
#pragma unroll
        for (int qq = 0; qq < kNsMaxCTiles; ++qq) {
            const int q = wave + kNW * qq;
            if (q < ntiles) {
                int a, b;
                c_tile(q, nA, bK, a, b);
                const int col = 16 * b + li16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * a + lk + 4 * r;
                    if (row < K) {
                        if (col < K && col <= row) Cp[row * (row + 1) / 2 + col] = acc[qq][r];
                        else if (col == K) ck[row] = acc[qq][r];
                    }
                }
            }
        }
    }
    __syncthreads();
    // ---- 6. right-hand side Z^T b1 - Z^T A v; Cholesky; solves; w = v + Z z
    if (!bad && t < K) {
        double a0 = 0.0, a1 = 0.0;
        int row = 0;
        for (; row + 1 < n; row += 2) {
            a0 = fma(big[row * ldz + t], b1[row], a0);
            a1 = fma(big[(row + 1) * ldz + t], b1[row + 1], a1);
        }
        if (row < n) a0 = fma(big[row * ldz + t], b1[row], a0);
        rhs[t] = (a0 + a1) - ck[t];
    }
    if (!bad && wave == 0) {
        double dm = 0.0;
        for (int i = lane; i < K; i += 64) dm = fmax(dm, Cp[i * (i + 1) / 2 + i]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, 64));
        if (lane == 0) sc[1] = dm * 0x1p-45;
    }
    __syncthreads();
    const double tinyC = sc[1];
    // right-looking Cholesky: column k by the threads of its rows, the
    // trailing triangle spread over the whole workgroup
    for (int k = 0; k < K && !bad; ++k) {
        const double d = Cp[k * (k + 1) / 2 + k];
        if (!(d > tinyC)) {
            bad = true;  // uniform: every thread read the same pivot
            break;
        }
        const double lkk = sqrt(d);
        if (t > k && t < K) Cp[t * (t + 1) / 2 + k] /= lkk;
        __syncthreads();
        if (t == 0) Cp[k * (k + 1) / 2 + k] = lkk;
        const int tk = K - 1 - k;
        for (int q = t; q < tk * (tk + 1) / 2; q += kNT) {
            int ii, jj;
            tri_index(q, ii, jj);
            const int i = k + 1 + ii, j = k + 1 + jj;
            double *ri = Cp + i * (i + 1) / 2;
            ri[j] = fma(-ri[k], Cp[j * (j + 1) / 2 + k], ri[j]);
        }
        __syncthreads();
    }
    // forward then backward substitution with L (one wavefront, rows l and l + 64)
    if (!bad && wave == 0) {
        double r0 = lane < K ? rhs[lane] : 0.0, r1 = lane + 64 < K ? rhs[lane + 64] : 0.0;
        for (int k = 0; k < K; ++k) {
            const double rk = k < 64 ? __shfl(r0, k, 64) : __shfl(r1, k - 64, 64);
            const double yk = rk / Cp[k * (k + 1) / 2 + k];
            if (lane == k) r0 = yk;
            if (lane + 64 == k) r1 = yk;
            if (lane > k && lane < K) r0 = fma(-Cp[lane * (lane + 1) / 2 + k], yk, r0);
            if (lane + 64 > k && lane + 64 < K) r1 = fma(-Cp[(lane + 64) * (lane + 65) / 2 + k], yk, r1);
        }
        for (int k = K - 1; k >= 0; --k) {
            const double rk = k < 64 ? __shfl(r0, k, 64) : __shfl(r1, k - 64, 64);
            const double zk = rk / Cp[k * (k + 1) / 2 + k];
            if (lane == k) r0 = zk;
            if (lane + 64 == k) r1 = zk;
            const double *rowk = Cp + k * (k + 1) / 2;
            if (lane < k) r0 = fma(-rowk[lane], zk, r0);
            if (lane + 64 < k) r1 = fma(-rowk[lane + 64], zk, r1);
        }
        if (lane < K) rhs[lane] = r0;
        if (lane + 64 < K) rhs[lane + 64] = r1;
    }
    __syncthreads();
    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (bad) {
        for (int k = t; k < n; k += kNT) w[k] = 0.0;
        if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
    } else {
        const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
        for (int i = t; i < n; i += kNT) {
            const double *zi = big + i * ldz;
            double a0 = zi[K], a1 = 0.0;
            int a = 0;
            for (; a + 1 < K; a += 2) {
                a0 = fma(zi[a], rhs[a], a0);
                a1 = fma(zi[a + 1], rhs[a + 1], a1);
            }
            if (a < K) a0 = fma(zi[a], rhs[a], a0);
            w[i] = (a0 + a1) / s2;
        }
    }
    __syncthreads();
}

template <int DIM, int RC>
__global__ __launch_bounds__(kNT) void k_weights_ns(WCtx cx, const Item *__restrict__ items, int64_t nitems,
                                                    int32_t *counter) {
    extern __shared__ __align__(16) double lds_ns[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t q = s_item;
        __syncthreads();
        if (q >= nitems) return;
        solve_ns_item<DIM, RC>(cx, items[q], lds_ns);
    }
}

const void *ns_kernel(int dim, int rc) {
#define RBF_NS(D, R) \
    if (dim == D && rc == R) return (const void *)k_weights_ns<D, R>;
    RBF_NS(1, 12) RBF_NS(1, 18) RBF_NS(1, 24) RBF_NS(1, 42) RBF_NS(1, 44)
    RBF_NS(2, 12) RBF_NS(2, 18) RBF_NS(2, 24) RBF_NS(2, 42) RBF_NS(2, 44)
    RBF_NS(3, 12) RBF_NS(3, 18) RBF_NS(3, 24) RBF_NS(3, 42) RBF_NS(3, 44)
#undef RBF_NS
    return nullptr;
}

}  // namespace

// Workgroups of the null-space launch (one per CU at this LDS size), or 0.
int weights_ns_grid(int dim, int rc, size_t lds_bytes) {
    const void *kern = ns_kernel(dim, rc);
    if (!kern) return 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, lds_bytes) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_weights_ns(hipStream_t s, int dim, int rc, int64_t N, const double *xyz, const int32_t *sten,
                             const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                             const int8_t *type, const double *normals, double *w_out, DevStatus *status,
                             const void *items, int64_t nitems, int32_t *counter, size_t lds_bytes, int grid) {
    WCtx cx{dim, N, xyz, sten, nrow, n_max, rows, mrow, w_out, type, normals, nullptr, 0, 0, status};
    const void *kern = ns_kernel(dim, rc);
    if (grid <= 0 || !kern) return hipErrorInvalidConfiguration;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
#define RBF_NS(D, R)                                                                                              \
    if (dim == D && rc == R) {                                                                                   \
        hipLaunchKernelGGL((k_weights_ns<D, R>), dim3(grid), dim3(kNT), lds_bytes, s, cx, (const Item *)items,   \
                           nitems, counter);                                                                     \
        return hipGetLastError();                                                                                \
    }
    RBF_NS(1, 12) RBF_NS(1, 18) RBF_NS(1, 24) RBF_NS(1, 42) RBF_NS(1, 44)
    RBF_NS(2, 12) RBF_NS(2, 18) RBF_NS(2, 24) RBF_NS(2, 42) RBF_NS(2, 44)
    RBF_NS(3, 12) RBF_NS(3, 18) RBF_NS(3, 24) RBF_NS(3, 42) RBF_NS(3, 44)
#undef RBF_NS
    return hipErrorInvalidConfiguration;
}

}  // namespace rbf
