/*
 * CPU oracle for the RBF-FD Poisson sweep of Vehovar, Rot and Kosec,
 * "Performance Trade-offs of High Order Meshless Approximation on Distributed
 * Memory Systems" (arXiv 2502.12878).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Nothing in the product
 * path may link or call it; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or table with
 * the HIP library.
 *
 * Arithmetic: IEEE-754 binary64, round to nearest, compiled with
 * -ffp-contract=off so that every a*b+c is a separate product and sum.  Every
 * loop runs in the order written here; nothing is blocked, fused or
 * reordered.  OpenMP appears only in orc_sweep_omp, the timed CPU baseline,
 * which is the sequential sweep with a parallel-for over rows (the paper's
 * intra-node parallelisation, Sec. II-B "Implementation").
 *
 * Status codes: 0 ok, 1 invalid argument, 3 singular local system,
 * 4 diverged, 5 not converged.
 *
 * Pins (see tests/test_oracle_*.py): closed-form stencils (5-point and
 * 7-point Laplacians, the natural cubic spline, the 4th-order 1D stencil),
 * monomial reproduction, invariances, LAPACK solves, scipy kNN and sparse
 * solves, the decay rate of the lowest mode, finite differences of the
 * adjoint.  No function here is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ESINGULAR 3
#define ORC_EDIVERGED 4
#define ORC_ENOTCONVERGED 5

/* ------------------------------------------------------------------------ */
/* Monomials of total degree <= m (Sec. II, augmentation; M = C(m+d, d)).    */
/* Order: graded by degree 0..m; within a degree the x exponent descends,    */
/* then the y exponent descends.                                             */
/* ------------------------------------------------------------------------ */
int orc_monomials(int dim, int m, int *exps /* [M][3], may be NULL */)
{
    int count = 0;
    for (int deg = 0; deg <= m; ++deg) {
        if (dim == 1) {
            if (exps) { exps[3 * count] = deg; exps[3 * count + 1] = 0; exps[3 * count + 2] = 0; }
            ++count;
        } else if (dim == 2) {
            for (int a = deg; a >= 0; --a) {
                if (exps) { exps[3 * count] = a; exps[3 * count + 1] = deg - a; exps[3 * count + 2] = 0; }
                ++count;
            }
        } else {
            for (int a = deg; a >= 0; --a)
                for (int b = deg - a; b >= 0; --b) {
                    if (exps) { exps[3 * count] = a; exps[3 * count + 1] = b; exps[3 * count + 2] = deg - a - b; }
                    ++count;
                }
        }
    }
    return count;
}

/* Squared distance between node j and node c: d2 = (dx*dx + dy*dy) + dz*dz
 * with dx = x_j - x_c, summed in axis order.  This exact expression defines
 * "nearest" and ties (Sec. II: supports are the n nearest nodes). */
static double sqdist(int dim, int64_t N, const double *xyz, int64_t j, int64_t c)
{
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
        double t = xyz[a * N + j] - xyz[a * N + c];
        double t2 = t * t;
        s = (a == 0) ? t2 : s + t2;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Supports by brute force (Sec. II): for each requested centre, the n nodes */
/* with the smallest keys (d2, id) in lexicographic order, listed in         */
/* ascending key order.  The centre itself has d2 = 0 and comes first.       */
/* ------------------------------------------------------------------------ */
/* With `type` given, a Neumann centre (type 2) draws its support from itself
 * and the interior nodes only (Sec. II-C: boundary values are computed from
 * the interior values of the last step in the boundary node's support). */
int orc_knn_typed(int dim, int64_t N, const double *xyz, int n, const int64_t *rows, int64_t nrows,
                  const int8_t *type, int32_t *out)
{
    if (dim < 1 || dim > 3 || n < 1 || n > N) return ORC_EINVAL;
    double *bd = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *bi = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t c = rows[q];
        int restrict_interior = type && type[c] == 2;
        int cnt = 0;
        for (int64_t j = 0; j < N; ++j) {
            if (restrict_interior && j != c && type[j] != 0) continue;
            double d2 = sqdist(dim, N, xyz, j, c);
            /* keep the n smallest (d2, j); j ascends, so a new key never
             * beats an equal-distance key already held */
            if (cnt == n && !(d2 < bd[n - 1])) continue;
            int pos = (cnt < n) ? cnt : n - 1;
            while (pos > 0 && d2 < bd[pos - 1]) {
                bd[pos] = bd[pos - 1];
                bi[pos] = bi[pos - 1];
                --pos;
            }
            bd[pos] = d2;
            bi[pos] = j;
            if (cnt < n) ++cnt;
        }
        if (cnt < n) { free(bd); free(bi); return ORC_EINVAL; }
        for (int k = 0; k < n; ++k) out[q * n + k] = (int32_t)bi[k];
    }
    free(bd);
    free(bi);
    return ORC_OK;
}

int orc_knn(int dim, int64_t N, const double *xyz, int n,
            const int64_t *rows, int64_t nrows, int32_t *out /* [nrows][n] */)
{
    return orc_knn_typed(dim, N, xyz, n, rows, nrows, NULL, out);
}

/* ------------------------------------------------------------------------ */
/* RBF-FD weights of the Laplacian for one centre (Sec. II, the augmented    */
/* system [A P; P^T 0][w; lambda] = [L Phi; L p]).                           */
/*                                                                          */
/* Local coordinates: s = sqrt(max_k d2(x_k, x_c)), y_k = (x_k - x_c)/s.      */
/* A_kl = r^3 with r = |y_k - y_l| (cubic polyharmonic spline),              */
/* P_kj = y_k^alpha_j, (L Phi)_k = 3(d+1)|y_k| (the Laplacian of r^3 in d    */
/* dimensions evaluated at the centre), (L p)_j = 2 for alpha_j = 2e_i, else */
/* 0.  The system is solved by Gaussian elimination with partial pivoting;   */
/* the weights in x are w_k = x_k/(s*s) because the Laplacian is homogeneous */
/* of degree -2.                                                             */
/*                                                                          */
/* Returns 0, or 3 when a pivot is exactly zero or smaller than 2^-45 times  */
/* the largest entry of the assembled matrix.  *pivot_ratio receives        */
/* min|pivot| / max|a| (a conditioning diagnostic).                          */
/* ------------------------------------------------------------------------ */
/* The same system for the derivative along a unit normal nv at the centre
 * (the Neumann rows of the mixed-boundary variant, Sec. II-C): the right-hand
 * side becomes (dPhi/dn)_k = 3|y_k| ((0 - y_k) . nv), the derivative of
 * |y - y_k|^3 at y = 0, and (dp/dn)_j = nv_a for the linear monomial y_a, 0
 * otherwise; the weights in x are w_k = x_k / s (degree -1).             */
/* ------------------------------------------------------------------------ */
/* Assemble the augmented matrix [A P b1; P^T 0 b2] (S rows, S+1 columns,
 * row-major, S = n + M) for centre c; op 0 = Laplacian, op 1 = derivative
 * along nv.  Returns the scale s (0 if all support nodes coincide with the
 * centre). */
static double assemble(int dim, int64_t N, const double *xyz, int64_t c,
                       const int32_t *sten, int n, int m, int op, const double *nv,
                       double *a, double *y)
{
    int exps[84 * 3];
    int M = orc_monomials(dim, m, exps);
    int S = n + M;
    int C = S + 1; /* augmented with the right-hand side as column S */

    /* scale: the largest support distance */
    double d2max = 0.0;
    for (int k = 0; k < n; ++k) {
        double d2 = sqdist(dim, N, xyz, sten[k], c);
        if (d2 > d2max) d2max = d2;
    }
    double s = sqrt(d2max);
    if (!(s > 0.0)) return 0.0;
    for (int k = 0; k < n; ++k)
        for (int ax = 0; ax < 3; ++ax)
            y[3 * k + ax] = (ax < dim) ? (xyz[ax * N + sten[k]] - xyz[ax * N + c]) / s : 0.0;

    /* assemble */
    for (int i = 0; i < S * C; ++i) a[i] = 0.0;
    const double c3 = 3.0 * (double)(dim + 1);
    for (int k = 0; k < n; ++k) {
        for (int l = 0; l < n; ++l) {
            double r2 = 0.0;
            for (int ax = 0; ax < dim; ++ax) {
                double t = y[3 * k + ax] - y[3 * l + ax];
                double t2 = t * t;
                r2 = (ax == 0) ? t2 : r2 + t2;
            }
            double r = sqrt(r2);
            a[k * C + l] = (r * r) * r;
        }
        for (int j = 0; j < M; ++j) {
            double p = 1.0;
            for (int ax = 0; ax < dim; ++ax)
                for (int e = 0; e < exps[3 * j + ax]; ++e) p = p * y[3 * k + ax];
            a[k * C + n + j] = p;  /* P   */
            a[(n + j) * C + k] = p; /* P^T */
        }
        double r2 = 0.0;
        for (int ax = 0; ax < dim; ++ax) {
            double t2 = y[3 * k + ax] * y[3 * k + ax];
            r2 = (ax == 0) ? t2 : r2 + t2;
        }
        if (op == 0) {
            a[k * C + S] = c3 * sqrt(r2);
        } else {
            double dn = 0.0; /* (0 - y_k) . nv */
            for (int ax = 0; ax < dim; ++ax) {
                double t = (0.0 - y[3 * k + ax]) * nv[ax];
                dn = (ax == 0) ? t : dn + t;
            }
            a[k * C + S] = (3.0 * sqrt(r2)) * dn;
        }
    }
    for (int j = 0; j < M; ++j) {
        int deg = exps[3 * j] + exps[3 * j + 1] + exps[3 * j + 2];
        if (op == 0) {
            int pure = (exps[3 * j] == 2 || exps[3 * j + 1] == 2 || exps[3 * j + 2] == 2);
            a[(n + j) * C + S] = (deg == 2 && pure) ? 2.0 : 0.0;
        } else {
            double v = 0.0;
            if (deg == 1)
                for (int ax = 0; ax < dim; ++ax)
                    if (exps[3 * j + ax] == 1) v = nv[ax];
            a[(n + j) * C + S] = v;
        }
    }
    return s;
}

/* Exported for tests: the assembled system of one centre. */
int orc_assemble(int dim, int64_t N, const double *xyz, int64_t c, const int32_t *sten,
                 int n, int m, double *a_out /* [S][S+1] */, double *s_out)
{
    double y[3 * 512];
    if (dim < 1 || dim > 3 || n < 1 || n > 512 || m < 0 || m > 6) return ORC_EINVAL;
    *s_out = assemble(dim, N, xyz, c, sten, n, m, 0, NULL, a_out, y);
    return ORC_OK;
}

static int weights_one(int dim, int64_t N, const double *xyz, int64_t c,
                       const int32_t *sten, int n, int m, int op, const double *nv,
                       double *w_out, double *pivot_ratio, double *work)
{
    int M = orc_monomials(dim, m, NULL);
    int S = n + M;
    int C = S + 1;
    double *a = work;             /* [S][C] */
    double *y = work + S * C;     /* [n][3] */
    double *x = y + 3 * n;        /* [S]    */
    double s = assemble(dim, N, xyz, c, sten, n, m, op, nv, a, y);
    if (!(s > 0.0)) { *pivot_ratio = 0.0; return ORC_ESINGULAR; }

    double amax = 0.0;
    for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j)
            if (fabs(a[i * C + j]) > amax) amax = fabs(a[i * C + j]);
    const double tiny = amax * 0x1p-45;

    /* Gaussian elimination with partial pivoting: for column k the pivot is
     * the first row i >= k with the largest |a_ik|; rows are swapped; each
     * lower row i gets a_ij - l_ik * a_kj with l_ik = a_ik / a_kk, for all
     * columns j > k including the right-hand side. */
    double pmin = INFINITY;
    for (int k = 0; k < S; ++k) {
        int p = k;
        double best = fabs(a[k * C + k]);
        for (int i = k + 1; i < S; ++i) {
            double v = fabs(a[i * C + k]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > tiny)) { *pivot_ratio = 0.0; return ORC_ESINGULAR; }
        if (best < pmin) pmin = best;
        if (p != k)
            for (int j = 0; j < C; ++j) {
                double t = a[k * C + j];
                a[k * C + j] = a[p * C + j];
                a[p * C + j] = t;
            }
        for (int i = k + 1; i < S; ++i) {
            double l = a[i * C + k] / a[k * C + k];
            for (int j = k + 1; j < C; ++j) {
                double prod = l * a[k * C + j];
                a[i * C + j] = a[i * C + j] - prod;
            }
        }
    }
    /* Back substitution by columns: x_j = b_j / a_jj, then every row above
     * subtracts a_ij * x_j, for j from the last unknown down to the first. */
    for (int j = S - 1; j >= 0; --j) {
        x[j] = a[j * C + S] / a[j * C + j];
        for (int i = 0; i < j; ++i) {
            double prod = a[i * C + j] * x[j];
            a[i * C + S] = a[i * C + S] - prod;
        }
    }
    double s2 = (op == 0) ? s * s : s;
    for (int k = 0; k < n; ++k) w_out[k] = x[k] / s2;
    *pivot_ratio = (amax > 0.0) ? pmin / amax : 0.0;
    return ORC_OK;
}

/* Weights for a list of centres.  stencils: [nrows][n_stride], row q holding
 * n_row[q] entries (n_row NULL -> all n_stride); m_row likewise (NULL -> m).
 * op_row[q] (NULL -> all 0) selects the operator: 0 Laplacian, 1 derivative
 * along normals[:, rows[q]] (normals: [dim][N]).
 * w_out: [nrows][n_stride], entries beyond n_row[q] set to 0.
 * On a singular system returns 3 and writes the centre id to *bad_row. */
int orc_weights_op(int dim, int64_t N, const double *xyz,
                   const int64_t *rows, int64_t nrows,
                   const int32_t *stencils, int n_stride, const int32_t *n_row,
                   int m, const int8_t *m_row, const int8_t *op_row, const double *normals,
                   double *w_out, double *pivot_ratio_out, int64_t *bad_row)
{
    if (dim < 1 || dim > 3 || n_stride < 1) return ORC_EINVAL;
    int S_max = n_stride + 84;
    double *work = (double *)malloc(sizeof(double) * ((size_t)S_max * (S_max + 1) + 4 * (size_t)S_max));
    int status = ORC_OK;
    for (int64_t q = 0; q < nrows; ++q) {
        int n = n_row ? n_row[q] : n_stride;
        int mm = m_row ? m_row[q] : m;
        double pr = 0.0;
        for (int k = 0; k < n_stride; ++k) w_out[q * n_stride + k] = 0.0;
        if (n < 1 || n > n_stride || mm < 0 || mm > 6) { status = ORC_EINVAL; if (bad_row) *bad_row = rows[q]; break; }
        int op = op_row ? op_row[q] : 0;
        double nv[3] = {0.0, 0.0, 0.0};
        if (op == 1) {
            if (!normals) { status = ORC_EINVAL; if (bad_row) *bad_row = rows[q]; break; }
            for (int ax = 0; ax < dim; ++ax) nv[ax] = normals[ax * N + rows[q]];
        }
        int st = weights_one(dim, N, xyz, rows[q], stencils + q * n_stride, n, mm, op, nv,
                             w_out + q * n_stride, &pr, work);
        if (pivot_ratio_out) pivot_ratio_out[q] = pr;
        if (st != ORC_OK) { status = st; if (bad_row) *bad_row = rows[q]; break; }
    }
    free(work);
    return status;
}

int orc_weights(int dim, int64_t N, const double *xyz,
                const int64_t *rows, int64_t nrows,
                const int32_t *stencils, int n_stride, const int32_t *n_row,
                int m, const int8_t *m_row,
                double *w_out, double *pivot_ratio_out, int64_t *bad_row)
{
    return orc_weights_op(dim, N, xyz, rows, nrows, stencils, n_stride, n_row, m, m_row, NULL, NULL,
                          w_out, pivot_ratio_out, bad_row);
}

/* ------------------------------------------------------------------------ */
/* The operator and the explicit step (Sec. II-C, the Jacobi step).          */
/* Stencils and weights are row-major [N][n_stride]; row r uses its first    */
/* n_row[r] entries (NULL -> n_stride).  Only interior rows (type 0) carry   */
/* an operator.                                                              */
/* ------------------------------------------------------------------------ */

/* Largest |v| where a NaN counts as larger than every number. */
static double nanmax_abs(double acc, double v)
{
    double a = fabs(v);
    if (isnan(acc) || isnan(a)) return NAN;
    return (a > acc) ? a : acc;
}

/* (L u)_r = sum_k w_rk u_{idx_rk} in stencil order: the Laplacian on
 * interior rows, the normal derivative on Neumann rows (their weights, own
 * entry included); 0 on Dirichlet rows. */
void orc_apply(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
               int n_stride, const int32_t *n_row, const double *u, double *Lu)
{
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] == 1) { Lu[r] = 0.0; continue; }
        int n = n_row ? n_row[r] : n_stride;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            double prod = w[r * n_stride + k] * u[idx[r * n_stride + k]];
            acc = acc + prod;
        }
        Lu[r] = acc;
    }
}

/* Neumann boundary update (Sec. II-C, the paragraph on enforcing the Neumann
 * condition): before a step, every Neumann node b (type 2) takes the value for
 * which its normal-derivative stencil returns the prescribed data f_b, with
 * the other nodes of its support at their previous-step values:
 *   u_b = (f_b - sum_{k: idx_bk != b} w_bk u_{idx_bk}) / w_bb.
 * All new values are computed from the old ones before any is stored. */
void orc_neumann_update(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                        int n_stride, const int32_t *n_row, const double *f, double *u)
{
    int64_t nn = 0;
    for (int64_t r = 0; r < N; ++r) nn += type[r] == 2;
    if (!nn) return;
    double *nb = (double *)malloc(sizeof(double) * (size_t)nn);
    int64_t q = 0;
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] != 2) continue;
        int n = n_row ? n_row[r] : n_stride;
        double acc = 0.0, self = 0.0;
        for (int k = 0; k < n; ++k) {
            int32_t j = idx[r * n_stride + k];
            if (j == r) { self = w[r * n_stride + k]; continue; }
            double prod = w[r * n_stride + k] * u[j];
            acc = acc + prod;
        }
        nb[q++] = (f[r] - acc) / self;
    }
    q = 0;
    for (int64_t r = 0; r < N; ++r)
        if (type[r] == 2) u[r] = nb[q++];
    free(nb);
}

/* One explicit step u_new = u_old + dt (L u_old - f) on interior rows, after
 * the Neumann update of u_old; Dirichlet and Neumann rows copy u_old.  Returns
 * max |L u_old - f| over interior rows (the residual of u_old). */
double orc_sweep(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                 int n_stride, const int32_t *n_row, const double *f, double dt,
                 double *u_old, double *u_new)
{
    orc_neumann_update(N, type, idx, w, n_stride, n_row, f, u_old);
    double res = 0.0;
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] != 0) { u_new[r] = u_old[r]; continue; }
        int n = n_row ? n_row[r] : n_stride;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            double prod = w[r * n_stride + k] * u_old[idx[r * n_stride + k]];
            acc = acc + prod;
        }
        double rho = acc - f[r];
        double step = dt * rho;
        u_new[r] = u_old[r] + step;
        res = nanmax_abs(res, rho);
    }
    return res;
}

/* The same step with the row loop split over OpenMP threads (the paper's
 * "#pragma omp parallel for", Sec. II-B).  Used only to time the CPU
 * baseline; per-row arithmetic is identical to orc_sweep. */
double orc_sweep_omp(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                     int n_stride, const int32_t *n_row, const double *f, double dt,
                     const double *u_old, double *u_new, int nthreads)
{
    double res = 0.0;
    int any_nan = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(max : res) reduction(| : any_nan)
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] != 0) { u_new[r] = u_old[r]; continue; }
        int n = n_row ? n_row[r] : n_stride;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            double prod = w[r * n_stride + k] * u_old[idx[r * n_stride + k]];
            acc = acc + prod;
        }
        double rho = acc - f[r];
        double step = dt * rho;
        u_new[r] = u_old[r] + step;
        double a = fabs(rho);
        if (isnan(a)) any_nan = 1;
        else if (a > res) res = a;
    }
    return any_nan ? NAN : res;
}

/* max |L u - f| over interior rows */
double orc_residual(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                    int n_stride, const int32_t *n_row, const double *f, const double *u)
{
    double res = 0.0;
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] != 0) continue;
        int n = n_row ? n_row[r] : n_stride;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            double prod = w[r * n_stride + k] * u[idx[r * n_stride + k]];
            acc = acc + prod;
        }
        res = nanmax_abs(res, acc - f[r]);
    }
    return res;
}

/* ------------------------------------------------------------------------ */
/* Iteration to tolerance (Sec. II-C; the periodic residual report of        */
/* Sec. III-A).  Steps run in chunks of `chunk`; the residual known after a  */
/* chunk is that of the iterate entering the chunk's last step.  After each  */
/* chunk:                                                                    */
/*   diverged  if that residual is not finite or exceeds 1e6 * res(u0);     */
/*   converged if it is <= tol_rel * max|f| over interior rows (tol_rel>0); */
/*   stalled   if it has not improved on the best seen for `stall` chunks;  */
/*   stop      at max_steps.                                                */
/* A NaN/Inf residual of u0 is divergence at step 0.  At the end the final   */
/* iterate's residual is evaluated once more.                                */
/* Result codes: 0 converged (or fixed-step run with tol_rel <= 0 that did   */
/* not diverge), 4 diverged, 5 not converged.                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t steps;
    double res0, res_last, res_final, fnorm;
    int64_t diverged_step;
    int converged, diverged;
} orc_iter_report;

int orc_iterate(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                int n_stride, const int32_t *n_row, const double *f, double dt,
                double *u /* in: u0 (Dirichlet rows hold g); out: final */,
                double *work /* [N] */, int64_t max_steps, double tol_rel,
                int64_t chunk, int64_t stall, orc_iter_report *rep)
{
    memset(rep, 0, sizeof(*rep));
    rep->diverged_step = -1;
    if (chunk < 1 || max_steps < 0) return ORC_EINVAL;
    double fnorm = 0.0;
    for (int64_t r = 0; r < N; ++r)
        if (type[r] == 0) fnorm = nanmax_abs(fnorm, f[r]);
    rep->fnorm = fnorm;
    double res0 = orc_residual(N, type, idx, w, n_stride, n_row, f, u);
    rep->res0 = res0;
    rep->res_last = res0;
    if (!isfinite(res0)) {
        rep->diverged = 1;
        rep->diverged_step = 0;
        rep->res_final = res0;
        return ORC_EDIVERGED;
    }
    double best = INFINITY;
    int64_t since_best = 0;
    int64_t steps = 0;
    double *a = u, *b = work;
    int status = (tol_rel > 0.0) ? ORC_ENOTCONVERGED : ORC_OK;
    while (steps < max_steps) {
        int64_t s = chunk;
        if (s > max_steps - steps) s = max_steps - steps;
        double res = 0.0;
        for (int64_t t = 0; t < s; ++t) {
            res = orc_sweep(N, type, idx, w, n_stride, n_row, f, dt, a, b);
            double *tmp = a; a = b; b = tmp;
        }
        steps += s;
        rep->res_last = res;
        if (!isfinite(res) || res > 1e6 * res0) {
            rep->diverged = 1;
            rep->diverged_step = steps;
            status = ORC_EDIVERGED;
            break;
        }
        if (tol_rel > 0.0 && res <= tol_rel * fnorm) {
            rep->converged = 1;
            status = ORC_OK;
            break;
        }
        if (res < best) { best = res; since_best = 0; }
        else if (stall > 0 && ++since_best >= stall) break;
    }
    if (a != u) memcpy(u, a, sizeof(double) * (size_t)N);
    rep->steps = steps;
    rep->res_final = orc_residual(N, type, idx, w, n_stride, n_row, f, u);
    return status;
}

/* ------------------------------------------------------------------------ */
/* FP32 inner sweeps inside an FP64 residual-correction loop.               */
/* One outer pass:  r = f - L64 u (FP64 weights, interior rows; 0 on         */
/* Dirichlet rows);  r32 = (float) r;  e = 0;  `inner` times                 */
/* e_new = e + dt32 (L32 e - r32) on interior rows with FP32 weights and     */
/* FP32 accumulation (Dirichlet rows keep e = 0);  u += (double) e.          */
/* With u_ref given, after each pass err = max |u - u_ref| over all nodes;   */
/* the loop stops when err <= err_target, or after max_outer passes.        */
/* Returns the number of passes run; errs[p] receives err after pass p.      */
/* ------------------------------------------------------------------------ */
int64_t orc_mixed(int64_t N, const int8_t *type, const int32_t *idx,
                  const double *w64, const float *w32, int n_stride, const int32_t *n_row,
                  const double *f, double dt, double *u, int64_t inner, int64_t max_outer,
                  const double *u_ref, double err_target, double *errs,
                  double *r /* [N] work */, float *e /* [N] */, float *e2 /* [N] */,
                  float *r32 /* [N] */)
{
    const float dt32 = (float)dt;
    int64_t pass = 0;
    for (; pass < max_outer; ++pass) {
        for (int64_t i = 0; i < N; ++i) {
            if (type[i] != 0) { r[i] = 0.0; continue; }
            int n = n_row ? n_row[i] : n_stride;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) {
                double prod = w64[i * n_stride + k] * u[idx[i * n_stride + k]];
                acc = acc + prod;
            }
            r[i] = f[i] - acc;
        }
        for (int64_t i = 0; i < N; ++i) { r32[i] = (float)r[i]; e[i] = 0.0f; }
        float *ea = e, *eb = e2;
        for (int64_t t = 0; t < inner; ++t) {
            for (int64_t i = 0; i < N; ++i) {
                if (type[i] != 0) { eb[i] = 0.0f; continue; }
                int n = n_row ? n_row[i] : n_stride;
                float acc = 0.0f;
                for (int k = 0; k < n; ++k) {
                    float prod = w32[i * n_stride + k] * ea[idx[i * n_stride + k]];
                    acc = acc + prod;
                }
                float rho = acc - r32[i];
                float step = dt32 * rho;
                eb[i] = ea[i] + step;
            }
            float *tmp = ea; ea = eb; eb = tmp;
        }
        for (int64_t i = 0; i < N; ++i)
            if (type[i] == 0) u[i] = u[i] + (double)ea[i];
        if (u_ref) {
            double err = 0.0;
            for (int64_t i = 0; i < N; ++i) err = nanmax_abs(err, u[i] - u_ref[i]);
            if (errs) errs[pass] = err;
            if (err <= err_target) { ++pass; break; }
        }
    }
    return pass;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of K explicit steps with respect to the source f.                */
/* The step is u_{j+1} = G u_j - dt f (+ dt L_IB g) on interior rows, with   */
/* G = I + dt L_II.  For J(u_K) with dJ/du_K = gK, the gradient is           */
/*   dJ/df = -dt sum_{j=0}^{K-1} (G^T)^j gK   (interior rows; 0 elsewhere). */
/* (G^T v)_c = v_c + dt sum_{r interior} sum_k [idx_rk = c] w_rk v_r for     */
/* interior c: a transpose scatter in which nothing flows into Dirichlet     */
/* columns.  Sequential loops, no atomics.                                   */
/* ------------------------------------------------------------------------ */
void orc_apply_transpose(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                         int n_stride, const int32_t *n_row, const double *v, double *out)
{
    for (int64_t c = 0; c < N; ++c) out[c] = 0.0;
    for (int64_t r = 0; r < N; ++r) {
        if (type[r] != 0) continue;
        int n = n_row ? n_row[r] : n_stride;
        for (int k = 0; k < n; ++k) {
            int32_t c = idx[r * n_stride + k];
            if (type[c] != 0) continue;
            double prod = w[r * n_stride + k] * v[r];
            out[c] = out[c] + prod;
        }
    }
}

void orc_adjoint_f(int64_t N, const int8_t *type, const int32_t *idx, const double *w,
                   int n_stride, const int32_t *n_row, double dt, int64_t K,
                   const double *gK, double *grad /* [N] */,
                   double *lam /* [N] work */, double *tmp /* [N] work */)
{
    double *sum = grad;
    for (int64_t i = 0; i < N; ++i) {
        lam[i] = (type[i] == 0) ? gK[i] : 0.0;
        sum[i] = lam[i];
    }
    for (int64_t j = 1; j < K; ++j) {
        orc_apply_transpose(N, type, idx, w, n_stride, n_row, lam, tmp);
        for (int64_t i = 0; i < N; ++i) {
            if (type[i] != 0) { lam[i] = 0.0; continue; }
            double step = dt * tmp[i];
            lam[i] = lam[i] + step;
            sum[i] = sum[i] + lam[i];
        }
    }
    for (int64_t i = 0; i < N; ++i) grad[i] = (type[i] == 0) ? -dt * sum[i] : 0.0;
}
