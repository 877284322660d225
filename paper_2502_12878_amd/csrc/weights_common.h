// Device helpers shared by the weight solvers (k_weights.hip: Gaussian
// elimination in the oracle's operation order; k_weights_ns.hip: the
// null-space solver): the work-item queue, the per-launch context, the
// monomial exponents, the local coordinates and the entries of the augmented
// system [A P; P^T 0][w; lambda] = [L Phi; L p] (Sec. II).
#pragma once

#include "rbf_internal.h"

namespace rbf {
namespace {

enum ItemKind : int32_t { kSmall = 0, kLarge = 1 };

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

// Maximum over the T threads of a group (T = 64 or a multiple of 64): a
// wavefront reduction, then the wavefronts' results through red[].  The
// maximum of a set does not depend on the order it is taken in.
__device__ double group_max(double v, int t, int T, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if (T == 64) return v;
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double m = red[0];
    for (int q = 1; q < T / 64; ++q) m = fmax(m, red[q]);
    __syncthreads();
    return m;
}

// Per-system preamble: scale s and local coordinates y (LDS), run by the
// threads [t0, t0 + T) of the system's group.  Returns s (read after a
// workgroup barrier by the caller).
__device__ void local_coords(const WCtx &cx, int64_t c, int n, double *y, double *s_out, int t, int T,
                             double *red /* [T] */) {
    const int32_t *st = cx.sten + c * (int64_t)cx.n_max;
    double mx = 0.0;
    for (int k = t; k < n; k += T) mx = fmax(mx, d2_exact(cx.dim, cx.xyz, cx.N, st[k], c));
    const double s = sqrt(group_max(mx, t, T, red));
    if (t == 0) *s_out = s;
    for (int q = t; q < 3 * n; q += T) {
        const int k = q / 3, a = q % 3;
        y[q] = a < cx.dim ? (cx.xyz[a * cx.N + st[k]] - cx.xyz[a * cx.N + c]) / s : 0.0;
    }
}

}  // namespace
}  // namespace rbf
