// Internal declarations of the gfx950 RBF-FD library: the handle, the packed
// operator layout, and the host-side launchers of every kernel family.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "rbf.h"

namespace rbf {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSlice = 64;       // rows per slice of the packed operator (= one wavefront)
constexpr int kMaxSupport = 256; // largest support size accepted
constexpr int kMaxOrder = 6;     // largest augmentation order accepted
// Largest node count: the sweeps gather FP64 values at 32-bit byte offsets.
constexpr int64_t kMaxNodes = ((int64_t)1 << 29) - 1;

// Device-side status word: set by kernels that detect a failure, read by the
// host at the next synchronisation.  code = rbf_status, info = node id.
struct DevStatus {
    int32_t code;
    int32_t pad;
    int64_t info;
};

// Launch shape of the sweep kernels (chosen by the autotuner).
struct SweepCfg {
    int waves_per_block = 4;  // slices (64 rows each) per workgroup
    int unroll = 8;           // support entries loaded ahead per lane
    int xcd_remap = 1;        // give each XCD a contiguous range of slices
    int pipeline = 0;         // request the next group's streams before the current gathers
    int zigzag = 0;           // odd sweeps of a sequence visit the slices in reverse order
    int codes = 0;            // read 16-bit segment codes instead of 32-bit column ids (Ell::code)
    int temporal = 0;         // with codes: ordinary instead of non-temporal operator loads
    int quad = 0;             // FP32 sweeps with codes: weights in the code layout (Ell::w32q)
    bool operator<(const SweepCfg &o) const {
        return std::tie(waves_per_block, unroll, xcd_remap, pipeline, zigzag, codes, temporal, quad) <
               std::tie(o.waves_per_block, o.unroll, o.xcd_remap, o.pipeline, o.zigzag, o.codes, o.temporal, o.quad);
    }
};

// Packed operator: interior rows renumbered first (grouped by support size,
// then canonical id), Dirichlet rows last.  Slice s covers internal rows
// [64 s, 64 s + 64); its entries live at slice_ptr[s] + k*64 + lane for
// k < slice_len[s].  Within a row, entries are sorted by internal column id
// so that the k-th gathers of neighbouring rows hit neighbouring addresses.
struct Ell {
    int layout = 1;                // 0: one element per lane per entry; 1: entry pairs as vectors (k_sweep.hip)
    int64_t nslices = 0;
    int64_t elems = 0;
    int64_t ncols = 0;             // length of the gathered vector (all nodes)
    int32_t max_len = 0;
    int32_t uniform_len = 0;       // the length of every slice when all are equal, else 0
    int64_t *slice_ptr = nullptr;  // [nslices + 1]
    int32_t *slice_len = nullptr;  // [nslices]
    int32_t *idx = nullptr;        // [elems] internal ids
    double *w = nullptr;           // [elems]
    float *w32 = nullptr;          // [elems] or null
    // Compressed column ids (layout 1 only): the columns of a slice fall in at
    // most kSegs aligned blocks of kSegSpan ids; entry k of a lane is the
    // 16-bit code (segment << 12 | column % 4096) at cptr[s] + 256 (k / 4) +
    // 4 lane + k % 4 (slice length padded to a multiple of 4), and
    // column = segbase[16 s + segment] + (code & 4095).  Slices touching more
    // blocks keep cmode[s] = 0 and are read from idx.
    uint16_t *code = nullptr;      // [celems]
    int64_t *cptr = nullptr;       // [nslices + 1]
    int32_t *segbase = nullptr;    // [16 nslices]
    int8_t *cmode = nullptr;       // [nslices] 1: slice has codes
    float *w32q = nullptr;         // [celems] FP32 weights of coded slices in the code layout, or null
    // Lane order of the transposed operator (rows of uneven length): the 64
    // rows of a slice sit on its lanes by decreasing length, and lane p of
    // slice s holds row 64 s + (lmeta[64 s + p] & 63), of lmeta[64 s + p] >> 6
    // (< 1024) entries.  The sweeps then mask each lane's loads past its own
    // length, so whole cache lines of padding are not fetched.  Null (also
    // when a row is longer): lane p holds row 64 s + p.
    uint16_t *lmeta = nullptr;     // [64 nslices] or null
    int64_t celems = 0;
    int64_t coded_slices = 0;      // slices with cmode 1
    int64_t code_mismatches = 0;   // slices whose codes failed the decode check (kept on 32-bit ids)
};

constexpr int kSegs = 16;
constexpr int kSegSpan = 4096;

}  // namespace rbf

struct rbf_handle {
    int device = 0;
    hipStream_t stream = nullptr;   // borrowed
    hipStream_t cap = nullptr;      // own stream used only for graph capture
    hipStream_t cap2 = nullptr;     // second capture stream (branch of a forked step)
    hipEvent_t evf[2] = {nullptr, nullptr};  // fork / join of a captured step
    rbf_allocator alloc{};
    bool custom_alloc = false;
    std::vector<std::pair<void *, size_t>> owned;  // live allocations
    std::string err;
    char arch[64] = {0};
    int num_cus = 0;

    // small device/host scratch
    unsigned long long *dslots = nullptr;  // [16] device
    unsigned long long *hslots = nullptr;  // [16] pinned host
    rbf::DevStatus *dstatus = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // nodes (canonical order)
    int dim = 0;
    int64_t N = 0, N_int = 0, N_neu = 0;
    double *xyz = nullptr;      // [dim][N]
    int8_t *type = nullptr;     // [N]: 0 interior, 1 Dirichlet, 2 Neumann
    double *normals = nullptr;  // [dim][N] unit outward normals (Neumann nodes)

    // stencils and weights (canonical order, row-major [N][n_max])
    int32_t n_max = 0;
    int32_t *sten = nullptr;
    int16_t *nrow = nullptr;  // [N]
    double *w_can = nullptr;
    bool have_sten = false, have_w = false, have_w32 = false;

    // internal numbering and packed operator
    int32_t *perm = nullptr;   // internal -> canonical
    int32_t *iperm = nullptr;  // canonical -> internal
    rbf::Ell ell;
    rbf::Ell ellT;             // transposed interior operator (built on first use)
    rbf::Ell ellN;             // Neumann rows (internal N_int ..), own entry zeroed
    double *wself = nullptr;   // [N_neu] own weight of each Neumann row
    double *nb = nullptr;      // [N_neu] new Neumann values of a step
    bool neu_direct = false;   // Neumann supports hold interior nodes only: update in place
    int64_t far_slices = 0;    // leading slices whose rows read no Neumann node

    // iteration vectors (internal order)
    double *ua = nullptr, *ub = nullptr, *fint = nullptr, *tmp = nullptr, *uref = nullptr;
    double *part = nullptr;   // per-block partial sums
    float *ea = nullptr, *eb = nullptr, *r32 = nullptr;

    rbf::SweepCfg cfg;    // FP64 sweep family
    rbf::SweepCfg cfg32;  // FP32 inner sweeps
    rbf::SweepCfg cfgT;   // sweep on the transposed operator (adjoint)
    bool tunedT = false;
    int weights_panel = 16;
    hipError_t noalloc_status = hipSuccess;  // lookup of the no-allocation workspace at creation
    int64_t w_ns_systems = 0, w_elim_systems = 0;  // solver paths of the last weight computation
    double last_sweep_sec = 0.0;
    int64_t last_sweeps = 0;

    // cached graphs: key = (kind, steps, start buffer, dt bits) -> executable
    std::map<std::tuple<int, int64_t, int, uint64_t>, hipGraphExec_t> graphs;

    // host copies used for validation and layout
    std::vector<int8_t> type_h;
    std::vector<int16_t> nrow_h;
};

namespace rbf {

// ---------------------------------------------------------------- memory
void *dalloc(rbf_handle *h, size_t bytes);
void dfree(rbf_handle *h, void *p);
template <typename T>
T *dalloc_n(rbf_handle *h, size_t n) { return static_cast<T *>(dalloc(h, n * sizeof(T) + 256)); }

// ---------------------------------------------------------------- nodes
hipError_t launch_build_nodes(hipStream_t s, int dim, int64_t side, double h, double t, uint64_t seed,
                              double *xyz, int8_t *type);

// ---------------------------------------------------------------- neighbours
struct CellGrid {
    int dim;
    int nc[3];
    double lo[3];
    double edge[3];
    int64_t ncells;
};
hipError_t launch_bbox_partials(hipStream_t s, int dim, int64_t N, const double *xyz, double *partials, int nblk);
hipError_t launch_bin_nodes(hipStream_t s, const CellGrid &g, int64_t N, const double *xyz, int32_t *cell_of,
                            int32_t *cell_count, int32_t *cell_start, int32_t *ids_by_cell, int32_t *cursor,
                            int32_t *scan_tmp);
hipError_t launch_coords_by_cell(hipStream_t s, int dim, int64_t N, const double *xyz, const int32_t *ids,
                                 double *xyz_c);
hipError_t launch_knn_query(hipStream_t s, const CellGrid &g, int64_t N, const double *xyz, const double *xyz_c,
                            const int32_t *cell_of, const int32_t *cell_start, const int32_t *ids_by_cell,
                            int32_t n_uniform, const int16_t *n_per_node, int32_t n_max, double ball_coef,
                            double margin, int32_t *sten, int16_t *nrow_out, const int8_t *type,
                            DevStatus *status);

// ---------------------------------------------------------------- weights
// Row stride (doubles) of a LARGE system's slab: S + 1 columns rounded up to 4.
__host__ __device__ constexpr int blocked_ld(int S) { return (S + 1 + 3) & ~3; }
int64_t weights_slab(int S_large);
int weights_small_limit();
int weights_grid(int S_small, int S_large, int panel);
size_t weights_item_bytes();
void weights_make_item(void *dst, int kind, int count, int64_t first);
hipError_t launch_weights_items(hipStream_t s, int dim, int64_t N, const double *xyz, const int32_t *sten,
                                const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                                const int8_t *type, const double *normals, double *w_out, double *scratch,
                                int64_t slab, int panel, DevStatus *status, const void *items, int64_t nitems,
                                int32_t *counter, int S_small, int S_large, int grid, int nslabs,
                                size_t *lds_used);

// Null-space solver (k_weights_ns.hip) for systems with m >= 1 whose sizes
// fit its register arrays and LDS layout; one launch per register-array size.
int ns_bucket(int dim, int n, int M);         // register-array size of the launch for (n, M); 0: no fit
int ns_lds_doubles(int n, int M, int bucket);  // LDS of one system, in doubles
bool ns_fits(int dim, int n, int M, size_t lds_limit);
int weights_ns_grid(int dim, int bucket, size_t lds_bytes);
hipError_t launch_weights_ns(hipStream_t s, int dim, int bucket, int64_t N, const double *xyz, const int32_t *sten,
                             const int16_t *nrow, int32_t n_max, const int32_t *rows, const int8_t *mrow,
                             const int8_t *type, const double *normals, double *w_out, DevStatus *status,
                             const void *items, int64_t nitems, int32_t *counter, size_t lds_bytes, int grid);

// ---------------------------------------------------------------- sweep family
hipError_t launch_pack_ell(hipStream_t s, int64_t row0, int64_t nrows, int32_t n_max, const int32_t *perm,
                           const int32_t *iperm, const int32_t *sten, const int16_t *nrow, const double *w_can,
                           const Ell &e, double *wself, int32_t *foreign);
hipError_t launch_encode_codes(hipStream_t s, const Ell &e);
hipError_t launch_check_codes(hipStream_t s, const Ell &e, unsigned long long *bad);
hipError_t launch_flag_near(hipStream_t s, int64_t N, int32_t n_max, const int32_t *sten, const int16_t *nrow,
                            const int8_t *type, int8_t *near);
hipError_t launch_neumann_update(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                 const double *g, double *u_cur, double *u_next, double *nb, bool direct);
hipError_t launch_neumann_apply(hipStream_t s, const Ell &e, int64_t N_int, int64_t N_neu, const double *wself,
                                const double *u, double *out);
// parity: index of the sweep within its sequence (odd sweeps run reversed when c.zigzag is set)
// s0, ns: the launch covers slices [s0, s0 + ns) (ns < 0: all slices from s0)
hipError_t launch_sweep_f64(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *f,
                            const double *u_old, double *u_new, double dt, unsigned long long *res_slot,
                            int parity, int64_t s0 = 0, int64_t ns = -1);
hipError_t launch_sweep_f32(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const float *r,
                            const float *e_old, float *e_new, float dt, int parity);
hipError_t launch_sweep_f32q(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const float *r,
                             const float *e_old, float *e_new, float dt, int parity);
hipError_t launch_apply_f64(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *u,
                            double *Lu, const double *f, unsigned long long *res_slot);
hipError_t launch_outer_residual(hipStream_t s, const SweepCfg &c, const Ell &e, int64_t N_int, const double *f,
                                 const double *u, float *r32, float *e0, unsigned long long *res_slot);
hipError_t launch_add_correction(hipStream_t s, int64_t N_int, double *u, const float *e);
hipError_t launch_tcount(hipStream_t s, int64_t N, int32_t n_max, int64_t N_int, const int8_t *type,
                         const int32_t *iperm, const int32_t *sten, const int16_t *nrow, int32_t *cnt);
hipError_t launch_tfill(hipStream_t s, int64_t N, int32_t n_max, int64_t N_int, const int8_t *type,
                        const int32_t *iperm, const int32_t *sten, const int16_t *nrow, const double *w_can,
                        const int64_t *start, int32_t *cursor, int32_t *rows_t, double *w_t);
hipError_t launch_tpack(hipStream_t s, int64_t N_int, const int64_t *start, int32_t *rows_t, double *w_t,
                        const Ell &e);
hipError_t launch_err_norm(hipStream_t s, int64_t N, const double *u, const double *uref, double *partials,
                           int nblk, unsigned long long *max_slot);
hipError_t launch_sum_partials(hipStream_t s, const double *partials, int n, double *out);
hipError_t launch_transpose_scatter(hipStream_t s, const Ell &e, int64_t N_int, const double *v, double *out);
hipError_t launch_adjoint_update(hipStream_t s, int64_t N_int, double dt, double *lam, double *acc, double *tmp);
hipError_t launch_gather(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst);
hipError_t launch_scatter(hipStream_t s, int64_t n, const int32_t *perm, const double *src, double *dst);
hipError_t launch_fill_f64(hipStream_t s, int64_t n, double v, double *p);
hipError_t launch_fill_f32(hipStream_t s, int64_t n, float v, float *p);
hipError_t launch_fill_u64(hipStream_t s, int64_t n, unsigned long long v, unsigned long long *p);
hipError_t launch_slot_to_double(hipStream_t s, const unsigned long long *slot, double *out);
hipError_t launch_scale_interior(hipStream_t s, int64_t N, int64_t N_int, double a, const double *src, double *dst);

}  // namespace rbf
