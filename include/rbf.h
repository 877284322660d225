/*
 * rbf.h - C ABI of an MI355X (gfx950) library for the explicit RBF-FD Poisson
 * iteration of Vehovar, Rot and Kosec, "Performance Trade-offs of High Order
 * Meshless Approximation on Distributed Memory Systems" (arXiv 2502.12878).
 *
 * The calls follow the paper's problem statement in order: build nodes,
 * build stencils (supports), compute weights, iterate to tolerance.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns an rbf_status (0 = RBF_OK).  Arguments are checked
 *   before any GPU work is queued (RBF_EINVAL).  Nothing aborts or throws
 *   across this boundary.  rbf_last_error() gives a message naming the
 *   offending node id or step where there is one.
 * - Pointers named *_dev are device pointers on the handle's device; pointers
 *   named *_host are host pointers.  The caller owns every pointer it passes;
 *   the library never frees caller memory and keeps no caller pointer after
 *   the call returns (it copies what it needs).
 * - Internal buffers (cell lists, packed operator, iteration vectors, graph
 *   state) come from the allocator given to rbf_create (hipMalloc when NULL)
 *   and are released by rbf_destroy.
 * - All GPU work is queued on the stream given to rbf_create (or set later).
 *   Calls returning host-visible results (statuses of setup calls, iteration
 *   reports, get/set of stencils and weights) synchronise that stream; the
 *   others return once their work is queued.
 * - Node numbering: canonical ids 0..N-1 as given to rbf_set_nodes.  Every
 *   array crossing the ABI is in canonical order.  The library may renumber
 *   internally; that never shows at the ABI.
 * - Coordinates are structure-of-arrays: xyz[a*N + i] is coordinate a of
 *   node i.  Node types: 0 interior, 1 Dirichlet, 2 Neumann (the mixed
 *   boundary variant of Sec. II-C; Neumann nodes need unit outward normals).
 * - One host thread at a time per handle.
 */
#ifndef RBF_MI355X_H
#define RBF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rbf_status;
enum {
    RBF_OK = 0,
    RBF_EINVAL = 1,        /* bad argument or call order                        */
    RBF_ENOMEM = 2,        /* allocator returned NULL                           */
    RBF_ESINGULAR = 3,     /* a local weight system has a (near-)zero pivot     */
    RBF_EDIVERGED = 4,     /* residual non-finite or grew 1e6-fold              */
    RBF_ENOTCONVERGED = 5, /* max_steps reached or progress stalled             */
    RBF_EOVERFLOW = 6,     /* neighbour search exceeded its candidate capacity  */
    RBF_EHIP = 7           /* a HIP runtime call failed                         */
};

typedef struct rbf_handle rbf_handle;

/* Device-memory allocator used for every internal buffer.  alloc returns a
 * device pointer of at least `bytes` bytes (256-byte aligned) or NULL; free
 * releases it.  ctx is passed back unchanged. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} rbf_allocator;

/* ---------------------------------------------------------------- handle */

/* Create a handle on `device` queuing work on `hip_stream` (a hipStream_t,
 * borrowed; NULL = the null stream).  `alloc` may be NULL (hipMalloc/hipFree);
 * the struct is copied. */
rbf_status rbf_create(rbf_handle **out, int device, void *hip_stream, const rbf_allocator *alloc);
rbf_status rbf_destroy(rbf_handle *h);
/* Switch the stream later calls queue on (borrowed). */
rbf_status rbf_set_stream(rbf_handle *h, void *hip_stream);
const char *rbf_status_string(rbf_status s);
/* Message of the last failing call on this handle ("" if none). */
const char *rbf_last_error(const rbf_handle *h);
/* Library version string. */
const char *rbf_version(void);

/* Sizes known to the handle (any pointer may be NULL). */
rbf_status rbf_get_sizes(const rbf_handle *h, int *dim, int64_t *N, int64_t *N_interior, int32_t *n_max);

/* ------------------------------------------------------------ build nodes */

/* Jittered Cartesian node set on [0,1]^dim standing in for the paper's
 * quasi-uniform node sets (Sec. II-C, node generation).  side^dim nodes,
 * id = i + side*j + side^2*k, pitch h = 1/(side-1).  Draw number id*dim + a
 * of the SplitMix64 stream `seed` (Steele, Lea and Flood, 2014) gives U in
 * [0,1) (top 53 bits times 2^-53); interior nodes move to
 * x = i*h + (2U - 1)*(jitter_frac*h), each product and sum rounded
 * separately; a node with any grid index 0 or side-1 is Dirichlet and stays
 * on the grid.
 * xyz_dev: [dim][side^dim] doubles; type_dev: [side^dim] int8.  Asynchronous.
 * EINVAL: dim not in 1..3, side < 2, side^dim > 2^31-1, jitter_frac not in
 * [0, 0.5), NULL pointers. */
rbf_status rbf_build_nodes(rbf_handle *h, int dim, int64_t side, double jitter_frac, uint64_t seed,
                           double *xyz_dev, int8_t *type_dev);

/* Give the handle its node set (copied).  Resets stencils and weights.
 * EINVAL: dim not in 1..3, N < 1 or N > 2^29-1 (the sweeps address the
 * gathered FP64 vector with 32-bit byte offsets), a type other than 0/1/2,
 * NULL pointers. */
rbf_status rbf_set_nodes(rbf_handle *h, int dim, int64_t N, const double *xyz_dev, const int8_t *type_dev);

/* Unit outward normals of the Neumann nodes (Sec. II-C, mixed boundary
 * conditions): normals_dev [dim][N] doubles (entries of other nodes are
 * ignored), copied.  Required before rbf_compute_weights when Neumann nodes
 * exist.  EINVAL: no nodes, a Neumann normal whose length differs from 1 by
 * more than 1e-12. */
rbf_status rbf_set_normals(rbf_handle *h, const double *normals_dev);

/* --------------------------------------------------------- build stencils */

/* Supports (Sec. II, after the weighted-sum form of the operator): for every
 * node, its n nearest nodes, the node itself first, in ascending order of the
 * key (d2, id) with d2 = (dx*dx + dy*dy) + dz*dz, dx = x_j - x_c, each
 * operation rounded separately; ties go to the lower id.  The search bins
 * nodes into a uniform cell grid and is exact.  A Neumann node's support is
 * itself and its nearest interior nodes (its boundary value is computed from
 * interior values only, Sec. II-C).
 * n_uniform: support size for every node, or 0 with n_per_node_dev
 * ([N] int16, device) giving each node's size.  Synchronises.
 * EINVAL: n < 1 or n > N or n > 256; EOVERFLOW: a node's candidate set
 * exceeded the search capacity (pathologically clustered nodes). */
rbf_status rbf_build_stencils(rbf_handle *h, int32_t n_uniform, const int16_t *n_per_node_dev);

/* -------------------------------------------------------- compute weights */

/* RBF-FD weights of the Laplacian (Sec. II, the augmented system
 * [A P; P^T 0][w; lambda] = [L Phi; L p]) for every interior node: cubic
 * polyharmonic spline phi(r) = r^3 plus all monomials of total degree <= m
 * (M = C(m+d, d), graded, x exponent then y exponent descending).  The system
 * is built in local coordinates y = (x - x_c)/s, s = the largest support
 * distance, solved in FP64, and w = x/(s*s).  Neumann rows get the weights of
 * the derivative along their normal nv instead: right-hand side
 * 3|y_k| ((0 - y_k) . nv) and nv_a for the monomial y_a, w = x/s.
 * m_uniform: order for every node, or -1 with m_per_node_dev ([N] int8).
 * keep_fp32: also keep an FP32 copy (needed by the mixed-precision mode).
 * Solvers:
 * - systems of more than 40 unknowns with m >= 1, 2 or 3 dimensions,
 *   n <= 255, M <= 84 and n - M + 1 <= 86 (3D) or M, n - M + 1 <= 64 (2D):
 *   a null-space method.
 *   P = [L1; L2] U by LU with partial pivoting (rows reordered pivots
 *   first), w = v + G z with G = [-L1^{-T} L2^T; I] spanning the null space
 *   of P^T and P^T v = Lp, and (G^T A G) z = G^T (L Phi - A v) by Cholesky
 *   (G^T A G is positive definite since r^3 is conditionally positive
 *   definite of order 2).  The same solution in another operation order: it
 *   agrees with the elimination to ~1e-12 relative per row, not bitwise;
 * - every other system: Gaussian elimination with partial pivoting (first row
 *   of largest |a_ik|) in the oracle's operation order, bit-equal to it.
 *   Above 40 unknowns it is factored by panels of 8 or 16 columns; the panel
 *   width is read from the tuning cache (key weights|arch|dim|S), else timed
 *   on a sample when there are at least 4096 such systems, else 16;
 *   RBF_WEIGHTS_PANEL=8 or 16 fixes it.  Every width performs the same
 *   floating-point operations in the same order, so the weights do not
 *   depend on it.
 * RBF_WEIGHTS_SOLVER=gepp in the environment sends every system to the
 * elimination.  rbf_get_operator_info reports how many systems each solver
 * took.
 * Synchronises.  ESINGULAR (with the node id in rbf_last_error) when a pivot
 * is zero or below 2^-45 times the largest matrix entry (a support with fewer
 * nodes than monomials, duplicate or collinear nodes; on the null-space path
 * a pivot of the factorisation of P at most 2^-45 max|P| or a Cholesky pivot
 * at most 2^-45 times the largest diagonal entry); EINVAL when m is not in
 * 0..6 or no stencils are set. */
rbf_status rbf_compute_weights(rbf_handle *h, int32_t m_uniform, const int8_t *m_per_node_dev, int keep_fp32);

/* ------------------------------------------------------ iterate (Sec. II-C) */

enum { RBF_MODE_FP64 = 0, RBF_MODE_MIXED = 1 };

typedef struct {
    double dt;             /* pseudo-time step, e.g. alpha*h^2/(2d)                 */
    int64_t max_steps;     /* upper bound on explicit steps                         */
    double tol_rel;        /* stop when max|L u - f| <= tol_rel*max|f| (interior);  */
                           /* <= 0: run exactly max_steps (unless diverged/err met) */
    int32_t chunk;         /* steps per residual check (one GPU graph per chunk)    */
    int32_t mode;          /* RBF_MODE_FP64 or RBF_MODE_MIXED                       */
    int32_t inner_steps;   /* mixed mode: FP32 steps per FP64 outer correction      */
    int32_t stall_chunks;  /* stop after this many chunks without a new best        */
                           /* residual (0 = never)                                  */
    const double *u_ref_dev; /* optional [N] reference for the error; NULL = none  */
    double err_target;     /* with u_ref: stop when max|u - u_ref| <= err_target    */
} rbf_iter_params;

typedef struct {
    int64_t steps;         /* explicit steps taken (mixed: inner steps of all passes) */
    double res0;           /* max|L u0 - f| over interior nodes                     */
    double res_last;       /* residual seen at the last check                       */
    double res_final;      /* max|L u - f| of the returned iterate                  */
    double fnorm;          /* max|f| over interior nodes                            */
    double err_inf;        /* max|u - u_ref| of the returned iterate (u_ref given)  */
    double err_mean_abs;   /* (1/N) sum |u - u_ref| (the paper's error measure)     */
    double seconds;        /* device time of the iteration (GPU events)             */
    int64_t diverged_step; /* step count at which divergence was seen, else -1      */
    int32_t converged;     /* tolerance or error target met                         */
    int32_t diverged;
    int32_t err_met;       /* error target met                                      */
    int32_t checks;        /* number of residual/error checks done                  */
} rbf_iter_report;

/* Explicit iteration u <- u + dt (L_h u - f) on interior nodes (the Jacobi
 * step of Sec. II-C); Dirichlet nodes keep their value.
 * u_dev: [N] in: u0 with Dirichlet values g; out: the final iterate.
 * f_dev: [N] (values on Dirichlet nodes are ignored).
 * Chunk semantics: after every `chunk` steps the residual of the iterate that
 * entered the chunk's last step is checked: non-finite or > 1e6*res0 ->
 * EDIVERGED; <= tol_rel*max|f| -> converged (RBF_OK).  A non-finite res0 is
 * divergence at step 0.  max_steps reached with tol_rel > 0 -> ENOTCONVERGED
 * (RBF_OK when tol_rel <= 0).  With u_ref and err_target > 0, the error is
 * checked at every chunk (mixed mode: after every outer pass) and reaching the
 * target ends the run with RBF_OK.
 * Mixed mode: per outer pass r = f - L64 u (FP64 weights), then inner_steps
 * FP32 steps e <- e + dt (L32 e - (float)r) from e = 0 with FP32 weights and
 * accumulation, then u += e; the last pass runs fewer inner steps when
 * max_steps is not a multiple of inner_steps.  Residual and error checks
 * happen once per outer pass (`chunk` does not apply).  Requires keep_fp32
 * at rbf_compute_weights.
 * Neumann nodes: f_dev on a Neumann node is its prescribed normal
 * derivative g_b.  Before every step each Neumann node takes
 * u_b = (g_b - sum_{k != b} w_bk u_k) / w_bb with the other support values of
 * the current iterate (all new values are computed before any is stored).
 * Mixed precision is implemented for problems without Neumann nodes only
 * (EINVAL).
 * Synchronises; the report is filled on every return path except EINVAL. */
rbf_status rbf_iterate(rbf_handle *h, const double *f_dev, double *u_dev, const rbf_iter_params *p,
                       rbf_iter_report *report);

/* ------------------------------------------------ single operator calls */

/* Lu_dev[r] = sum_k w_rk u_dev[idx_rk] for interior r (the Laplacian) and for
 * Neumann r (the normal derivative); 0 on Dirichlet rows. */
rbf_status rbf_apply(rbf_handle *h, const double *u_dev, double *Lu_dev);

/* out_dev[c] = sum over interior rows r and support entries k with
 * idx_rk = c of w_rk v_dev[r], for interior c; 0 on Dirichlet nodes (nothing
 * flows into Dirichlet columns).  The first transposed call builds L_II^T once
 * (entries of each column sorted by row), so results are deterministic; with
 * the environment variable RBF_TRANSPOSE_SCATTER=1 a scatter with FP64 atomics
 * is used instead (last bits may then vary between calls). */
rbf_status rbf_apply_transpose(rbf_handle *h, const double *v_dev, double *out_dev);

/* Max-norm residual max|L u - f| over interior nodes, written to *res_host.
 * Synchronises. */
rbf_status rbf_residual(rbf_handle *h, const double *f_dev, const double *u_dev, double *res_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result
 * of rbf_residual, max|L u - f| over interior nodes, written to the device
 * double *res_dev.  Queued on the handle's stream without synchronising; no
 * allocation of any kind.  The gathered copies of u and f and the reduction
 * slot live in a static workspace of 32 MiB that the library holds on each
 * device it runs on until the process ends, so the node count is limited to
 * 2^21 = 2,097,152 (EINVAL beyond, naming the limit).  Every call on a device
 * shares that workspace: calls that overlap on one device (other streams,
 * other handles, other host threads) race and must be serialised by the
 * caller.  f_dev, u_dev: [N] device, canonical order; res_dev: one device
 * double.  EINVAL without an operator or with NULL pointers; EHIP when the
 * workspace address could not be found on this device. */
rbf_status rbf_residual_noalloc(rbf_handle *h, const double *f_dev, const double *u_dev, double *res_dev);

/* ---------------------------------------- adjoint (inverse source problems) */

/* K explicit steps from u0 (Dirichlet values included) with checkpoints:
 * ckpt_dev receives u after steps 0, every, 2*every, ... (K/every + 1 rows of
 * N doubles, row j = state after j*every steps); uK_dev receives u after K
 * steps.  EINVAL unless 1 <= every <= K and K % every == 0. */
rbf_status rbf_forward_ckpt(rbf_handle *h, const double *f_dev, const double *u0_dev, int64_t K,
                            int64_t every, double *ckpt_dev, double *uK_dev, double dt);

/* Gradient of J(u_K) with respect to f for K explicit steps: with
 * G = I + dt L_II and gK = dJ/du_K, grad = -dt sum_{j=0}^{K-1} (G^T)^j gK on
 * interior nodes, 0 on Dirichlet nodes.  The sum is taken in Horner form,
 * T_0 = 0, T_{j+1} = T_j + dt (L_II^T T_j + gK) = dt gK + G^T T_j, so that
 * grad = -T_K: K forward sweeps over the transposed operator L_II^T (built
 * once, each column's entries sorted by row, so results are deterministic;
 * the first call also encodes it and picks its launch shape, cached like the
 * shapes of rbf_autotune) with -gK in place of f, in graphs of `every` steps
 * (one per checkpoint segment).  ckpt_dev may be NULL because this gradient
 * does not depend on the states.  RBF_TRANSPOSE_SCATTER=1 instead forms the
 * terms (G^T)^j gK one by one with the atomic scatter of
 * rbf_apply_transpose and sums them.  EINVAL when the node set has Neumann
 * nodes. */
rbf_status rbf_adjoint_f(rbf_handle *h, const double *gK_dev, int64_t K, int64_t every,
                         const double *ckpt_dev, double *grad_f_dev, double dt);

/* ------------------------------------------ import / export (canonical) */

/* Stencils as [N][n_max] int32, row r holding its n_r nearest ids (ascending
 * (d2, id)) then -1 padding.  Synchronises. */
rbf_status rbf_get_stencils(rbf_handle *h, int32_t *idx_host);
/* Weights as [N][n_max] doubles in stencil order, 0 on padding and on
 * Dirichlet rows.  Synchronises. */
rbf_status rbf_get_weights(rbf_handle *h, double *w_host);
/* Replace the stencils: [N][n_max] int32 canonical ids, -1 padding after the
 * first n_r entries (n_r >= 1).  Clears weights.  EINVAL: ids out of range,
 * an id repeated within a row, padding not -1.  Synchronises. */
rbf_status rbf_set_stencils(rbf_handle *h, const int32_t *idx_host, int32_t n_max);
/* Replace the weights ([N][n_max] doubles in stencil order; Dirichlet rows
 * ignored; Neumann rows are normal-derivative weights) and pack the
 * operator; keep_fp32 as in rbf_compute_weights.  EINVAL (and no operator)
 * when a Neumann row lacks its own node or its own weight is 0 or not
 * finite.  Synchronises. */
rbf_status rbf_set_weights(rbf_handle *h, const double *w_host, int keep_fp32);

/* ------------------------------------------------------------ tuning */

/* Time candidate kernel shapes for the current operator and keep the fastest
 * (sweep: rows per workgroup, unroll depth, XCD-aware block order, software
 * pipelining, zig-zag slice order, 16-bit column codes, non-temporal or
 * ordinary operator loads, FP32 weights in the code layout; weight solver:
 * panel width).  Results are cached in the JSON file named by the
 * RBF_AUTOTUNE_CACHE environment variable (none: not cached), keyed by device
 * architecture and problem shape; a shape found there is used without timing
 * (RBF_AUTOTUNE_FORCE=1 times again and replaces it).  RBF_SWEEP_ZIGZAG=0/1
 * and RBF_SWEEP_CODES=0/1 fix those two choices; RBF_SWEEP_SHAPE="waves,
 * unroll,xcd_remap,pipeline,zigzag,codes[,temporal[,quad]]" fixes the whole
 * sweep shape and turns the sweep timing off.  Synchronises. */
rbf_status rbf_autotune(rbf_handle *h);

/* Layout of the packed interior operator and the sweep shapes in use.
 * stream_bytes_* are the bytes one sweep reads and writes as the operator is
 * stored: column ids (4 B) or codes (2 B, plus the per-slice segment table)
 * and weights (8 B FP64 / 4 B FP32) of every slot including padding, slice
 * headers, and f, u and u_new of each interior row (8 B each in FP64; r, e
 * and e_new 4 B each in FP32).  The gathered values of u are not counted.
 * Every 16-bit code is decoded back and compared with its 32-bit id when the
 * codes are built; code_mismatches counts slices that failed (they are read
 * through their 32-bit ids instead; 0 is expected).  The t_* fields describe
 * the transposed interior operator L_II^T of the adjoint (all 0 until a
 * transposed call has built it); its rows are the columns of L_II, so their
 * length is a column's in-degree, which the support size does not bound. */
typedef struct {
    int64_t n_interior, n_neumann;
    int64_t slices, slots;          /* slots: packed entries incl. padding */
    int64_t coded_slices;           /* slices whose ids are also stored as codes */
    int32_t max_len, layout;
    int32_t f64_waves, f64_unroll, f64_xcd_remap, f64_pipeline, f64_zigzag, f64_codes;
    int32_t f32_waves, f32_unroll, f32_xcd_remap, f32_pipeline, f32_zigzag, f32_codes;
    double stream_bytes_f64, stream_bytes_f32;
    int32_t f64_temporal, f32_temporal;  /* code-reading sweeps: ordinary (1) or non-temporal (0) loads */
    int32_t f32_quad;                    /* FP32 weights of coded slices read in the code layout */
    int32_t code_mismatches;             /* slices whose codes failed the decode check */
    int64_t t_slices, t_slots, t_coded_slices, t_code_mismatches;
    int32_t t_max_len;                   /* longest transposed row (largest interior in-degree, even) */
    int32_t t_waves, t_unroll, t_codes;  /* launch shape of the transposed sweep */
    int64_t ns_systems;     /* weight systems solved by the null-space solver (last rbf_compute_weights) */
    int64_t elim_systems;   /* weight systems solved by Gaussian elimination (same call)               */
    int32_t t_lane_order;   /* transposed slices hold their rows on lanes by decreasing length */
    int32_t t_masked;       /* the transposed sweep skips each lane's loads past its own length */
} rbf_operator_info;

/* Fill *info for the current operator (EINVAL without one). */
rbf_status rbf_get_operator_info(const rbf_handle *h, rbf_operator_info *info);

/* Mean device time per FP64 sweep over the last rbf_iterate FP64 chunks
 * (GPU events around each graph launch divided by its step count), and the
 * number of sweeps timed.  For benchmarking. */
rbf_status rbf_last_sweep_time(const rbf_handle *h, double *seconds_per_sweep, int64_t *sweeps);

#ifdef __cplusplus
}
#endif
#endif /* RBF_MI355X_H */
