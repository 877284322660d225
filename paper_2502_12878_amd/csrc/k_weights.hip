// Batched RBF-FD weight solves (Sec. II: the augmented system
// [A P; P^T 0][w; lambda] = [L Phi; L p] with phi(r) = r^3 and monomials of
// degree <= m, L = Laplacian).
//
// One persistent launch walks a queue of work items of three kinds:
//   SMALL  4 systems with S = n + M <= 40, one wavefront each, matrix in LDS;
//   MID    1 system with S <= 112 on the whole workgroup, matrix in LDS;
//   LARGE  1 system with larger S on the whole workgroup: the matrix lives in
//          a per-workgroup scratch slab (L2 / Infinity Cache resident) and is
//          factored by panels of `panel` columns staged in LDS together with
//          the matching block of pivot rows.
// Items are queued largest first so the tail of the launch is short.
//
// Every path performs, element by element, the same floating-point
// operations in the same order as plain Gaussian elimination with partial
// pivoting: pivot = first row of largest |a_ik|; after the swap,
// l_i = a_ik / a_kk and a_ij <- a_ij - l_i*a_kj (product and difference
// rounded separately; this file is built with -ffp-contract=off); back
// substitution by columns from the last unknown.  The blocked path defers the
// row swaps of a panel for the trailing columns; a swap only exchanges two
// rows below the pivot row, so it commutes with the earlier updates of the
// same panel and the per-element sequence is unchanged.  Results are
// therefore independent of the panel width and of the work split.
#include "rbf_internal.h"

namespace rbf {
namespace {

constexpr int kBS = 256;  // threads per workgroup
constexpr int kSmallS = 40;
constexpr int kMidS = 112;

enum ItemKind : int32_t { kSmall = 0, kMid = 1, kLarge = 2 };

struct Item {
    int32_t kind;
    int32_t count;   // systems in the item (SMALL: up to 4)
    int64_t first;   // index into the row list
};

struct WCtx {
    int dim;
    int64_t N;
    const double *xyz;
    const int32_t *sten;
    const int16_t *nrow;
    int32_t n_max;
    const int32_t *rows;    // centre ids, grouped by (n, m)
    const int8_t *mrow;     // m per listed centre
    double *w_out;          // [N][n_max] canonical
    const int8_t *type;     // node types (2 = Neumann: normal-derivative row)
    const double *normals;  // [dim][N] unit normals of Neumann nodes (or null)
    double *scratch;        // LARGE slabs
    int64_t slab;           // doubles per slab
    int panel;
    DevStatus *status;
};

// Monomial exponents of degree <= m: graded by degree, then the x exponent
// descending, then the y exponent descending.
__device__ int make_exponents(int dim, int m, int8_t *ex /* [84][3] */) {
    int c = 0;
    for (int deg = 0; deg <= m; ++deg) {
        if (dim == 1) {
            ex[3 * c] = deg; ex[3 * c + 1] = 0; ex[3 * c + 2] = 0; ++c;
        } else if (dim == 2) {
            for (int a = deg; a >= 0; --a) { ex[3 * c] = a; ex[3 * c + 1] = deg - a; ex[3 * c + 2] = 0; ++c; }
        } else {
            for (int a = deg; a >= 0; --a)
                for (int b = deg - a; b >= 0; --b) {
                    ex[3 * c] = a; ex[3 * c + 1] = b; ex[3 * c + 2] = deg - a - b; ++c;
                }
        }
    }
    return c;
}

__device__ __forceinline__ int num_monomials(int dim, int m) {
    // C(m + d, d)
    if (dim == 1) return m + 1;
    if (dim == 2) return (m + 1) * (m + 2) / 2;
    return (m + 1) * (m + 2) * (m + 3) / 6;
}

__device__ __forceinline__ double d2_exact(int dim, const double *xyz, int64_t N, int64_t j, int64_t c) {
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
        const double t = xyz[a * N + j] - xyz[a * N + c];
        const double t2 = t * t;
        s = (a == 0) ? t2 : s + t2;
    }
    return s;
}

__device__ void report_status(DevStatus *st, int code, int64_t node) {
    atomicCAS(&st->code, 0, code);
    atomicMin((unsigned long long *)&st->info, (unsigned long long)node);
}

// Element (k, l) of the augmented matrix, 0 <= l <= S (column S = rhs).
// op 0: Laplacian rows; op 1: derivative along the unit normal nv (Neumann
// rows), whose right-hand side is 3|y_k| ((0 - y_k) . nv) for the r^3 block
// and nv_a for the linear monomial y_a.
__device__ __forceinline__ double entry(int k, int l, int n, int M, int S, int dim, const double *y,
                                        const int8_t *ex, int op, const double *nv) {
    const double c3 = 3.0 * (double)(dim + 1);
    if (l == S) {
        if (k < n) {
            double r2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                const double t2 = y[3 * k + a] * y[3 * k + a];
                r2 = (a == 0) ? t2 : r2 + t2;
            }
            if (op == 0) return c3 * sqrt(r2);
            double dn = 0.0;
            for (int a = 0; a < dim; ++a) {
                const double t = (0.0 - y[3 * k + a]) * nv[a];
                dn = (a == 0) ? t : dn + t;
            }
            return (3.0 * sqrt(r2)) * dn;
        }
        const int j = k - n;
        const int deg = ex[3 * j] + ex[3 * j + 1] + ex[3 * j + 2];
        if (op == 0) {
            const bool pure = ex[3 * j] == 2 || ex[3 * j + 1] == 2 || ex[3 * j + 2] == 2;
            return (deg == 2 && pure) ? 2.0 : 0.0;
        }
        double v = 0.0;
        if (deg == 1)
            for (int a = 0; a < dim; ++a)
                if (ex[3 * j + a] == 1) v = nv[a];
        return v;
    }
    if (k < n && l < n) {
        double r2 = 0.0;
        for (int a = 0; a < dim; ++a) {
            const double t = y[3 * k + a] - y[3 * l + a];
            const double t2 = t * t;
            r2 = (a == 0) ? t2 : r2 + t2;
        }
        const double r = sqrt(r2);
        return (r * r) * r;
    }
    if (k >= n && l >= n) return 0.0;
    const int row = k < n ? k : l;          // support node
    const int j = k < n ? l - n : k - n;    // monomial
    double p = 1.0;
    for (int a = 0; a < dim; ++a)
        for (int e = 0; e < ex[3 * j + a]; ++e) p = p * y[3 * row + a];
    return p;
}

// Per-system preamble: scale s and local coordinates y (LDS), run by the
// threads [t0, t0 + T) of the system's group.  Returns s (read after a
// workgroup barrier by the caller).
__device__ void local_coords(const WCtx &cx, int64_t c, int n, double *y, double *s_out, int t, int T,
                             double *red /* [T] */) {
    const int32_t *st = cx.sten + c * (int64_t)cx.n_max;
    double mx = 0.0;
    for (int k = t; k < n; k += T) mx = fmax(mx, d2_exact(cx.dim, cx.xyz, cx.N, st[k], c));
    red[t] = mx;
    __syncthreads();
    if (t == 0) {
        double m2 = 0.0;
        for (int q = 0; q < T; ++q) m2 = red[q] > m2 ? red[q] : m2;
        *s_out = sqrt(m2);
    }
    __syncthreads();
    const double s = *s_out;
    for (int q = t; q < 3 * n; q += T) {
        const int k = q / 3, a = q % 3;
        y[q] = a < cx.dim ? (cx.xyz[a * cx.N + st[k]] - cx.xyz[a * cx.N + c]) / s : 0.0;
    }
}

// GEPP + back substitution on an LDS-resident matrix A (S x (S+1), row stride
// ld) by a group of T threads; `grp` scalars live in LDS.  All groups of the
// workgroup call this together with the same S (barriers are uniform).
struct GroupScratch {
    int p;
    int bad;
    double piv;
    double s;
    double tiny;
};

template <int T>
__device__ bool gepp_lds(double *A, int S, int ld, double *lv, double *xs, GroupScratch *g, int t) {
    const int C = S + 1;
    const int lane = t & 63;
    bool dead = false;  // uniform within the group; barriers stay uniform
    for (int k = 0; k < S; ++k) {
        if (t < 64 && !dead) {  // pivot search by the group's first wavefront
            double best = -1.0;
            int p = S;
            for (int i = k + lane; i < S; i += 64) {
                const double v = fabs(A[i * ld + k]);
                if (v > best) { best = v; p = i; }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int op = __shfl_xor(p, off, 64);
                if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
            }
            if (lane == 0) {
                g->p = p;
                g->bad = !(best > g->tiny);
                g->piv = p < S ? A[p * ld + k] : 0.0;
            }
        }
        __syncthreads();
        dead = dead || g->bad;
        const int p = g->p;
        const double piv = g->piv;
        if (!dead) {
            // swap rows k and p beyond column k; multipliers from pre-swap rows
            if (p != k)
                for (int j = k + 1 + t; j < C; j += T) {
                    const double a = A[k * ld + j];
                    A[k * ld + j] = A[p * ld + j];
                    A[p * ld + j] = a;
                }
            for (int i = k + 1 + t; i < S; i += T) {
                const int src = (i == p) ? k : i;
                lv[i] = A[src * ld + k] / piv;
            }
        }
        __syncthreads();
        if (!dead) {
            if (t == 0) A[k * ld + k] = piv;
            const int rows = S - k - 1, cols = C - k - 1;
            for (int q = t; q < rows * cols; q += T) {
                const int i = k + 1 + q / cols, j = k + 1 + q % cols;
                const double prod = lv[i] * A[k * ld + j];
                A[i * ld + j] = A[i * ld + j] - prod;
            }
        }
        __syncthreads();
    }
    // back substitution by columns
    for (int j = S - 1; j >= 0; --j) {
        if (t == 0 && !dead) xs[j] = A[j * ld + S] / A[j * ld + j];
        __syncthreads();
        if (!dead) {
            const double xj = xs[j];
            for (int i = t; i < j; i += T) {
                const double prod = A[i * ld + j] * xj;
                A[i * ld + S] = A[i * ld + S] - prod;
            }
        }
        __syncthreads();
    }
    return !dead;
}

// SMALL and MID items: T threads per system, 256 / T systems per item.
template <int T>
__device__ void solve_lds_item(const WCtx &cx, const Item &it, char *lds, int S_lds) {
    const int grp = threadIdx.x / T, t = threadIdx.x % T;
    const int ld = S_lds + 1;
    // per-group LDS carve-up: A | y | lv | xs | red | ex | scalars
    const size_t a_bytes = (size_t)S_lds * ld * sizeof(double);
    const size_t per = a_bytes + (size_t)(5 * S_lds + T) * sizeof(double) + 84 * 3 + 64;
    const size_t per_al = (per + 15) & ~(size_t)15;
    char *base = lds + grp * per_al;
    double *A = (double *)base;
    double *y = (double *)(base + a_bytes);
    double *lv = y + 3 * S_lds;
    double *xs = lv + S_lds;
    double *red = xs + S_lds;
    int8_t *ex = (int8_t *)(red + T);
    GroupScratch *gs = (GroupScratch *)(((uintptr_t)(ex + 84 * 3) + 15) & ~(uintptr_t)15);

    const bool active = grp < it.count;
    const int64_t li = it.first + (active ? grp : 0);
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(cx.dim, m);
    const int S = n + M;  // uniform over the item
    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < cx.dim; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) make_exponents(cx.dim, m, ex);
    local_coords(cx, c, n, y, &gs->s, t, T, red);
    __syncthreads();
    const int C = S + 1;
    double amax = 0.0;
    for (int q = t; q < S * C; q += T) {
        const int k = q / C, l = q % C;
        const double v = entry(k, l, n, M, S, cx.dim, y, ex, op, nv);
        A[k * ld + l] = v;
        if (l < S) amax = fmax(amax, fabs(v));
    }
    red[t] = amax;
    __syncthreads();
    if (t == 0) {
        double mm = 0.0;
        for (int q = 0; q < T; ++q) mm = red[q] > mm ? red[q] : mm;
        gs->tiny = mm * 0x1p-45;
        gs->bad = 0;
    }
    __syncthreads();
    const double s = gs->s;
    const bool solved = gepp_lds<T>(A, S, ld, lv, xs, gs, t);
    const bool ok = solved && (s > 0.0);
    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (active) {
        if (ok) {
            const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
            for (int k = t; k < n; k += T) w[k] = xs[k] / s2;
        } else {
            for (int k = t; k < n; k += T) w[k] = 0.0;
            if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
        }
    }
    __syncthreads();
}

// LARGE item: whole workgroup, matrix in a global slab, panels in LDS.
__device__ void solve_blocked_item(const WCtx &cx, const Item &it, char *lds) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int64_t li = it.first;
    const int64_t c = cx.rows[li];
    const int n = cx.nrow[c];
    const int m = cx.mrow[li];
    const int M = num_monomials(cx.dim, m);
    const int S = n + M;
    const int C = S + 1;
    const int ld = C;
    const int PB = cx.panel;
    double *A = cx.scratch + (int64_t)blockIdx.x * cx.slab;

    // LDS: y | red | Lp [S][PB] | Ub [PB][C] | lv | piv idx | ex | scalars
    double *y = (double *)lds;
    double *red = y + 3 * kMaxSupport;
    double *Lp = red + kBS;
    double *Ub = Lp + (size_t)S * PB;
    double *bx = Ub + (size_t)PB * C;          // rhs / solution vector [S]
    int *pivs = (int *)(bx + S);
    int8_t *ex = (int8_t *)(pivs + 64);
    GroupScratch *gs = (GroupScratch *)(((uintptr_t)(ex + 84 * 3) + 15) & ~(uintptr_t)15);

    const int op = cx.type[c] == 2 ? 1 : 0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (op)
        for (int a = 0; a < cx.dim; ++a) nv[a] = cx.normals[a * cx.N + c];
    if (t == 0) make_exponents(cx.dim, m, ex);
    local_coords(cx, c, n, y, &gs->s, t, kBS, red);
    __syncthreads();
    const double s = gs->s;
    double amax = 0.0;
    for (int64_t q = t; q < (int64_t)S * C; q += kBS) {
        const int k = (int)(q / C), l = (int)(q % C);
        const double v = entry(k, l, n, M, S, cx.dim, y, ex, op, nv);
        A[(int64_t)k * ld + l] = v;
        if (l < S) amax = fmax(amax, fabs(v));
    }
    red[t] = amax;
    __syncthreads();
    if (t == 0) {
        double mm = 0.0;
        for (int q = 0; q < kBS; ++q) mm = red[q] > mm ? red[q] : mm;
        gs->tiny = mm * 0x1p-45;
        gs->bad = !(s > 0.0);
    }
    __syncthreads();
    bool ok = !gs->bad;

    for (int k0 = 0; ok && k0 < S; k0 += PB) {
        const int kb = min(PB, S - k0);
        const int prow = S - k0;
        // stage the panel: rows k0.., columns k0..k0+kb-1
        for (int q = t; q < prow * kb; q += kBS) {
            const int i = q / kb, j = q % kb;
            Lp[i * PB + j] = A[(int64_t)(k0 + i) * ld + k0 + j];
        }
        __syncthreads();
        // factor the panel; multipliers overwrite the eliminated entries
        for (int kk = 0; kk < kb; ++kk) {
            const int k = k0 + kk;
            if (t < 64) {
                double best = -1.0;
                int p = S;
                for (int i = kk + lane; i < prow; i += 64) {
                    const double v = fabs(Lp[i * PB + kk]);
                    if (v > best) { best = v; p = i; }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
                    const int op = __shfl_xor(p, off, 64);
                    if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
                }
                if (lane == 0) {
                    gs->p = p;
                    gs->bad = !(best > gs->tiny);
                    pivs[kk] = k0 + p;
                }
            }
            __syncthreads();
            if (gs->bad) { ok = false; break; }
            const int p = gs->p;
            if (p != kk)
                for (int j = t; j < kb; j += kBS) {
                    const double a = Lp[kk * PB + j];
                    Lp[kk * PB + j] = Lp[p * PB + j];
                    Lp[p * PB + j] = a;
                }
            __syncthreads();
            const double piv = Lp[kk * PB + kk];
            for (int i = kk + 1 + t; i < prow; i += kBS) Lp[i * PB + kk] = Lp[i * PB + kk] / piv;
            __syncthreads();
            const int cols = kb - kk - 1, rows = prow - kk - 1;
            for (int q = t; q < rows * cols; q += kBS) {
                const int i = kk + 1 + q / cols, j = kk + 1 + q % cols;
                const double prod = Lp[i * PB + kk] * Lp[kk * PB + j];
                Lp[i * PB + j] = Lp[i * PB + j] - prod;
            }
            __syncthreads();
            (void)k;
        }
        if (!ok) break;
        // write back the panel's pivot rows (upper part incl. diagonal)
        for (int q = t; q < kb * kb; q += kBS) {
            const int i = q / kb, j = q % kb;
            if (j >= i) A[(int64_t)(k0 + i) * ld + k0 + j] = Lp[i * PB + j];
        }
        // deferred row swaps on the trailing columns, in pivot order
        const int j0 = k0 + kb;
        const int tc = C - j0;
        for (int j = j0 + t; j < C; j += kBS)
            for (int kk = 0; kk < kb; ++kk) {
                const int p = pivs[kk];
                if (p != k0 + kk) {
                    const double a = A[(int64_t)(k0 + kk) * ld + j];
                    A[(int64_t)(k0 + kk) * ld + j] = A[(int64_t)p * ld + j];
                    A[(int64_t)p * ld + j] = a;
                }
            }
        __syncthreads();
        // U12: the panel's pivot rows over the trailing columns
        for (int j = j0 + t; j < C; j += kBS)
            for (int kk = 0; kk < kb; ++kk) {
                double v = A[(int64_t)(k0 + kk) * ld + j];
                for (int q = 0; q < kk; ++q) {
                    const double prod = Lp[kk * PB + q] * Ub[q * C + (j - j0)];
                    v = v - prod;
                }
                Ub[kk * C + (j - j0)] = v;
                A[(int64_t)(k0 + kk) * ld + j] = v;
            }
        __syncthreads();
        // trailing update with 4x4 register tiles
        const int tr = S - j0;
        const int ti = (tr + 3) / 4, tj = (tc + 3) / 4;
        for (int q = t; q < ti * tj; q += kBS) {
            const int i0 = j0 + (q / tj) * 4, c0 = (q % tj) * 4;
            double acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = (i0 + a < S && c0 + b < tc) ? A[(int64_t)(i0 + a) * ld + j0 + c0 + b] : 0.0;
            for (int kk = 0; kk < kb; ++kk) {
                double l[4], u[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) l[a] = (i0 + a < S) ? Lp[(i0 + a - k0) * PB + kk] : 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) u[b] = (c0 + b < tc) ? Ub[kk * C + c0 + b] : 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double prod = l[a] * u[b];
                        acc[a][b] = acc[a][b] - prod;
                    }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (i0 + a < S && c0 + b < tc) A[(int64_t)(i0 + a) * ld + j0 + c0 + b] = acc[a][b];
        }
        __syncthreads();
    }

    double *w = cx.w_out + c * (int64_t)cx.n_max;
    if (!ok) {
        for (int k = t; k < n; k += kBS) w[k] = 0.0;
        if (t == 0) report_status(cx.status, (int)RBF_ESINGULAR, c);
        __syncthreads();
        return;
    }
    // back substitution by columns, 64 columns at a time: wavefront 0 solves
    // the block's unknowns with shuffles, then every thread applies them to
    // the rows above in descending column order.
    for (int i = t; i < S; i += kBS) bx[i] = A[(int64_t)i * ld + S];
    __syncthreads();
    for (int j1 = S; j1 > 0; j1 -= 64) {
        const int jb0 = j1 > 64 ? j1 - 64 : 0;
        if (t < 64) {
            const int i = jb0 + lane;
            double b = i < j1 ? bx[i] : 0.0;
            for (int j = j1 - 1; j >= jb0; --j) {
                const double bj = __shfl(b, j - jb0, 64);
                const double xj = bj / A[(int64_t)j * ld + j];
                if (i == j) b = xj;
                if (i < j) {
                    const double prod = A[(int64_t)i * ld + j] * xj;
                    b = b - prod;
                }
            }
            if (i < j1) bx[i] = b;
        }
        __syncthreads();
        for (int i = t; i < jb0; i += kBS) {
            double b = bx[i];
            for (int j = j1 - 1; j >= jb0; --j) {
                const double prod = A[(int64_t)i * ld + j] * bx[j];
                b = b - prod;
            }
            bx[i] = b;
        }
        __syncthreads();
    }
    const double s2 = op ? s : s * s;  // degree -2 (Laplacian) or -1 (derivative)
    for (int k = t; k < n; k += kBS) w[k] = bx[k] / s2;
    __syncthreads();
}

__global__ __launch_bounds__(kBS) void k_weights(WCtx cx, const Item *__restrict__ items, int64_t nitems,
                                                 int32_t *counter, int S_small, int S_mid) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t q = s_item;
        __syncthreads();
        if (q >= nitems) return;
        const Item it = items[q];
        if (it.kind == kSmall) solve_lds_item<64>(cx, it, lds, S_small);
        else if (it.kind == kMid) solve_lds_item<kBS>(cx, it, lds, S_mid);
        else solve_blocked_item(cx, it, lds);
    }
}

size_t lds_small_bytes(int S_lds, int T) {
    const size_t a_bytes = (size_t)S_lds * (S_lds + 1) * sizeof(double);
    const size_t per = a_bytes + (size_t)(5 * S_lds + T) * sizeof(double) + 84 * 3 + 64;
    return ((per + 15) & ~(size_t)15) * (kBS / T);
}

size_t lds_blocked_bytes(int S, int PB) {
    return (size_t)(3 * kMaxSupport + kBS) * sizeof(double) + (size_t)S * PB * sizeof(double) +
           (size_t)PB * (S + 1) * sizeof(double) + (size_t)S * sizeof(double) + 64 * sizeof(int) + 84 * 3 + 64;
}

}  // namespace

int weights_small_limit() { return kSmallS; }
int weights_mid_limit() { return kMidS; }

size_t lds_total(int S_small, int S_mid, int S_large, int panel) {
    size_t lds = 0;
    if (S_small > 0) lds = std::max(lds, lds_small_bytes(S_small, 64));
    if (S_mid > 0) lds = std::max(lds, lds_small_bytes(S_mid, kBS));
    if (S_large > 0) lds = std::max(lds, lds_blocked_bytes(S_large, panel));
    return (lds + 255) & ~(size_t)255;
}

// Resident workgroups of the persistent launch on this device (0: does not fit).
int weights_grid(int S_small, int S_mid, int S_large, int panel) {
    const size_t lds = lds_total(S_small, S_mid, S_large, panel);
    if (hipFuncSetAttribute((const void *)k_weights, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_weights, kBS, lds) != hipSuccess) return 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

// Items: caller passes rows grouped into consecutive runs of equal (n, m).
// The host builds the queue (largest first) and sizes LDS for what is present.
hipError_t launch_weights_items(hipStream_t s, int dim, int64_t N, const double *xyz, const int32_t *sten,
                                const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                                const int8_t *type, const double *normals, double *w_out, double *scratch,
                                int64_t slab, int panel, DevStatus *status, const void *items, int64_t nitems,
                                int32_t *counter, int S_small, int S_mid, int S_large, int grid, int nslabs,
                                size_t *lds_used) {
    WCtx cx{dim, N, xyz, sten, nrow, n_max, rows, mrow, w_out, type, normals, scratch, slab, panel, status};
    const size_t lds = lds_total(S_small, S_mid, S_large, panel);
    if (lds_used) *lds_used = lds;
    if (grid <= 0) return hipErrorInvalidConfiguration;
    // a LARGE item uses scratch slab blockIdx.x: never launch more groups than slabs
    if (S_large > 0 && (scratch == nullptr || grid > nslabs)) return hipErrorInvalidConfiguration;
    hipError_t e = hipFuncSetAttribute((const void *)k_weights, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_weights, dim3(grid), dim3(kBS), lds, s, cx, (const Item *)items, nitems, counter, S_small,
                       S_mid);
    return hipGetLastError();
}

size_t weights_item_bytes() { return sizeof(Item); }

void weights_make_item(void *dst, int kind, int count, int64_t first) {
    Item it{kind, count, first};
    *(Item *)dst = it;
}

}  // namespace rbf
