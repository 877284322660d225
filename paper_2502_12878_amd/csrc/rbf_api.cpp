// Host runtime of the gfx950 RBF-FD library: the C ABI declared in rbf.h.
// Argument checks, memory management, the internal node numbering, the
// iteration controller (chunks of explicit steps captured as HIP graphs, one
// 16-byte device-to-host read per chunk), the checkpointed forward run and the
// adjoint, and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "rbf_internal.h"

using namespace rbf;

namespace {

rbf_status fail(rbf_handle *h, rbf_status st, const char *fmt, ...) {
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return st;
}

#define HIPCHK(h, expr)                                                                         \
    do {                                                                                        \
        hipError_t _e = (expr);                                                                 \
        if (_e != hipSuccess) return fail((h), RBF_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

#define ALLOC(h, ptr, T, n)                                                                    \
    do {                                                                                       \
        (ptr) = dalloc_n<T>((h), (size_t)(n));                                                 \
        if (!(ptr)) return fail((h), RBF_ENOMEM, "allocation of %zu bytes failed", (size_t)(n) * sizeof(T)); \
    } while (0)

// Switch to the handle's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

uint64_t double_bits(double d) {
    uint64_t b;
    std::memcpy(&b, &d, sizeof b);
    return b;
}

int num_monomials(int dim, int m) {
    int64_t num = 1, den = 1;
    for (int i = 1; i <= dim; ++i) {
        num *= (m + i);
        den *= i;
    }
    return (int)(num / den);
}

void free_ptr(rbf_handle *h, void *&p) {
    if (p) dfree(h, p);
    p = nullptr;
}

template <typename T>
void free_t(rbf_handle *h, T *&p) {
    void *q = (void *)p;
    free_ptr(h, q);
    p = nullptr;
}

void drop_graphs(rbf_handle *h) {
    for (auto &kv : h->graphs) hipGraphExecDestroy(kv.second);
    h->graphs.clear();
}

void drop_operator(rbf_handle *h) {
    drop_graphs(h);
    free_t(h, h->perm);
    free_t(h, h->iperm);
    free_t(h, h->ell.slice_ptr);
    free_t(h, h->ell.slice_len);
    free_t(h, h->ell.idx);
    free_t(h, h->ell.w);
    free_t(h, h->ell.w32);
    free_t(h, h->ell.code);
    free_t(h, h->ell.cptr);
    free_t(h, h->ell.segbase);
    free_t(h, h->ell.cmode);
    free_t(h, h->ell.w32q);
    h->ell = Ell{};
    free_t(h, h->ellT.slice_ptr);
    free_t(h, h->ellT.slice_len);
    free_t(h, h->ellT.idx);
    free_t(h, h->ellT.w);
    free_t(h, h->ellT.code);
    free_t(h, h->ellT.cptr);
    free_t(h, h->ellT.segbase);
    free_t(h, h->ellT.cmode);
    free_t(h, h->ellT.lmeta);
    h->ellT = Ell{};
    h->cfgT = SweepCfg{};
    h->tunedT = false;
    free_t(h, h->ellN.slice_ptr);
    free_t(h, h->ellN.slice_len);
    free_t(h, h->ellN.idx);
    free_t(h, h->ellN.w);
    h->ellN = Ell{};
    free_t(h, h->wself);
    free_t(h, h->nb);
    free_t(h, h->ua);
    free_t(h, h->ub);
    free_t(h, h->fint);
    free_t(h, h->tmp);
    free_t(h, h->uref);
    free_t(h, h->part);
    free_t(h, h->ea);
    free_t(h, h->eb);
    free_t(h, h->r32);
    h->have_w32 = false;
}

void drop_weights(rbf_handle *h) {
    drop_operator(h);
    free_t(h, h->w_can);
    h->have_w = false;
}

void drop_stencils(rbf_handle *h) {
    drop_weights(h);
    free_t(h, h->sten);
    free_t(h, h->nrow);
    h->nrow_h.clear();
    h->n_max = 0;
    h->have_sten = false;
}

rbf_status reset_status(rbf_handle *h) {
    DevStatus s{0, 0, std::numeric_limits<int64_t>::max()};
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::memcpy(h->hslots + 8, &s, sizeof s);
    HIPCHK(h, hipMemcpyAsync(h->dstatus, h->hslots + 8, sizeof s, hipMemcpyHostToDevice, h->stream));
    return RBF_OK;
}

rbf_status read_status(rbf_handle *h, DevStatus *out) {
    HIPCHK(h, hipMemcpyAsync(out, h->dstatus, sizeof *out, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return RBF_OK;
}

constexpr int kErrBlocks = 1024;

// ------------------------------------------------------------------ tuning cache
std::string cache_path() {
    const char *p = std::getenv("RBF_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

std::string read_file(const std::string &path) {
    std::ifstream f(path);
    if (!f) return std::string();
    std::stringstream ss;
    ss << f.rdbuf();
    return ss.str();
}

// The cache file is a JSON object of "key": [a, b, c] entries.
bool cache_lookup(const std::string &key, int *vals, int nv) {
    const std::string path = cache_path();
    if (path.empty()) return false;
    const std::string s = read_file(path);
    const std::string pat = "\"" + key + "\": [";
    const size_t at = s.find(pat);
    if (at == std::string::npos) return false;
    const char *c = s.c_str() + at + pat.size();
    for (int i = 0; i < nv; ++i) {
        char *end = nullptr;
        vals[i] = (int)std::strtol(c, &end, 10);
        if (end == c) return false;
        c = end;
        while (*c == ',' || *c == ' ') ++c;
    }
    return true;
}

// Rewrites the file with one entry per line: every "key": [ints] entry found
// in it (values may span lines), except the old entry of `key`, then `key`.
void cache_store(const std::string &key, const int *vals, int nv) {
    const std::string path = cache_path();
    if (path.empty()) return;
    const std::string s = read_file(path);
    std::vector<std::string> lines;
    for (size_t at = 0;;) {
        const size_t k0 = s.find('"', at);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t b0 = s.find_first_not_of(" \t\r\n", k1 + 1);
        if (b0 == std::string::npos || s[b0] != ':') { at = k1 + 1; continue; }
        const size_t v0 = s.find_first_not_of(" \t\r\n", b0 + 1);
        if (v0 == std::string::npos || s[v0] != '[') { at = k1 + 1; continue; }
        const size_t v1 = s.find(']', v0);
        if (v1 == std::string::npos) break;
        at = v1 + 1;
        const std::string k = s.substr(k0 + 1, k1 - k0 - 1);
        if (k == key) continue;
        std::string l = "  \"" + k + "\": [";
        std::stringstream vs(s.substr(v0 + 1, v1 - v0 - 1));
        std::string tok;
        bool first = true, ok = true;
        while (std::getline(vs, tok, ',')) {
            const size_t t0 = tok.find_first_not_of(" \t\r\n"), t1 = tok.find_last_not_of(" \t\r\n");
            if (t0 == std::string::npos) { ok = false; break; }
            l += (first ? "" : ", ") + tok.substr(t0, t1 - t0 + 1);
            first = false;
        }
        if (ok && !first) lines.push_back(l + "]");
    }
    std::string entry = "  \"" + key + "\": [";
    for (int i = 0; i < nv; ++i) entry += (i ? ", " : "") + std::to_string(vals[i]);
    entry += "]";
    lines.push_back(entry);
    std::ofstream f(path + ".tmp");
    f << "{\n";
    for (size_t i = 0; i < lines.size(); ++i) f << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
    f << "}\n";
    f.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

}  // namespace

// ====================================================================== memory
namespace rbf {

void *dalloc(rbf_handle *h, size_t bytes) {
    void *p = nullptr;
    if (h->custom_alloc) {
        p = h->alloc.alloc(bytes, h->alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) h->owned.emplace_back(p, bytes);
    return p;
}

void dfree(rbf_handle *h, void *p) {
    if (!p) return;
    auto it = std::find_if(h->owned.begin(), h->owned.end(), [p](const std::pair<void *, size_t> &e) { return e.first == p; });
    if (it == h->owned.end()) return;
    h->owned.erase(it);
    if (h->custom_alloc) h->alloc.free(p, h->alloc.ctx);
    else hipFree(p);
}

}  // namespace rbf

// ====================================================================== handle
extern "C" {

const char *rbf_version(void) { return "rbf-mi355x 0.1 (gfx950)"; }

const char *rbf_status_string(rbf_status s) {
    switch (s) {
        case RBF_OK: return "ok";
        case RBF_EINVAL: return "invalid argument";
        case RBF_ENOMEM: return "out of memory";
        case RBF_ESINGULAR: return "singular local system";
        case RBF_EDIVERGED: return "iteration diverged";
        case RBF_ENOTCONVERGED: return "not converged";
        case RBF_EOVERFLOW: return "neighbour search capacity exceeded";
        case RBF_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char *rbf_last_error(const rbf_handle *h) { return h ? h->err.c_str() : "null handle"; }

// Workspace of rbf_residual_noalloc (for callers that cannot allocate): the
// iterate and the source in internal order, kNoAllocMaxNodes doubles each,
// then the max-residual slot.  A file-scope device array, so every device the
// library runs on holds one copy (32 MiB + 256 B) until the process ends.
// Host code never uses the array's name as an address: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// when the first handle on the device is created, and kept in g_noalloc_ws.
constexpr int64_t kNoAllocMaxNodes = (int64_t)1 << 21;
constexpr int64_t kNoAllocDoubles = 2 * kNoAllocMaxNodes + 32;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];
static std::mutex g_noalloc_mu;
static double *g_noalloc_ws[kNoAllocMaxDevices];

// Look up this device's workspace address (the device is current).
static hipError_t init_noalloc_workspace(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ws[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ws[device] = static_cast<double *>(ptr);
    return hipSuccess;
}

static double *noalloc_workspace(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc_ws[device];
}

rbf_status rbf_create(rbf_handle **out, int device, void *hip_stream, const rbf_allocator *alloc) {
    if (!out) return RBF_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RBF_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->free)) return RBF_EINVAL;
    rbf_handle *h = new rbf_handle();
    h->device = device;
    DeviceGuard g(device);
    h->stream = (hipStream_t)hip_stream;
    if (alloc) {
        h->alloc = *alloc;
        h->custom_alloc = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete h;
        return RBF_EHIP;
    }
    std::snprintf(h->arch, sizeof h->arch, "%s", prop.gcnArchName);
    h->num_cus = prop.multiProcessorCount;
    // the no-allocation entry point's workspace on this device (a failure
    // here only disables that entry point, which then reports it)
    h->noalloc_status = init_noalloc_workspace(device);
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&h->cap2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->evf[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->evf[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
        hipHostMalloc((void **)&h->hslots, 16 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return RBF_EHIP;
    }
    h->dslots = dalloc_n<unsigned long long>(h, 16);
    h->dstatus = dalloc_n<DevStatus>(h, 1);
    if (!h->dslots || !h->dstatus) {
        rbf_destroy(h);
        return RBF_ENOMEM;
    }
    *out = h;
    return RBF_OK;
}

rbf_status rbf_destroy(rbf_handle *h) {
    if (!h) return RBF_EINVAL;
    {
        DeviceGuard g(h->device);
        if (h->stream) hipStreamSynchronize(h->stream);
        else hipDeviceSynchronize();
        drop_graphs(h);
        while (!h->owned.empty()) dfree(h, h->owned.back().first);
        if (h->cap) hipStreamDestroy(h->cap);
        if (h->cap2) hipStreamDestroy(h->cap2);
        for (hipEvent_t ev : h->evf)
            if (ev) hipEventDestroy(ev);
        if (h->ev0) hipEventDestroy(h->ev0);
        if (h->ev1) hipEventDestroy(h->ev1);
        if (h->hslots) hipHostFree(h->hslots);
    }
    delete h;
    return RBF_OK;
}

rbf_status rbf_set_stream(rbf_handle *h, void *hip_stream) {
    if (!h) return RBF_EINVAL;
    h->stream = (hipStream_t)hip_stream;
    return RBF_OK;
}

rbf_status rbf_get_sizes(const rbf_handle *h, int *dim, int64_t *N, int64_t *N_interior, int32_t *n_max) {
    if (!h) return RBF_EINVAL;
    if (dim) *dim = h->dim;
    if (N) *N = h->N;
    if (N_interior) *N_interior = h->N_int;
    if (n_max) *n_max = h->n_max;
    return RBF_OK;
}

// ====================================================================== nodes
rbf_status rbf_build_nodes(rbf_handle *h, int dim, int64_t side, double jitter_frac, uint64_t seed,
                           double *xyz_dev, int8_t *type_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (dim < 1 || dim > 3 || side < 2) return fail(h, RBF_EINVAL, "dim must be 1..3 and side >= 2");
    if (!(jitter_frac >= 0.0 && jitter_frac < 0.5)) return fail(h, RBF_EINVAL, "jitter_frac must be in [0, 0.5)");
    if (!xyz_dev || !type_dev) return fail(h, RBF_EINVAL, "null output pointer");
    int64_t N = 1;
    for (int a = 0; a < dim; ++a) {
        if (N > (int64_t)INT32_MAX / side) return fail(h, RBF_EINVAL, "side^dim exceeds 2^31-1");
        N *= side;
    }
    DeviceGuard g(h->device);
    const double pitch = 1.0 / (double)(side - 1);
    const double t = jitter_frac * pitch;
    HIPCHK(h, launch_build_nodes(h->stream, dim, side, pitch, t, seed, xyz_dev, type_dev));
    return RBF_OK;
}

rbf_status rbf_set_nodes(rbf_handle *h, int dim, int64_t N, const double *xyz_dev, const int8_t *type_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (dim < 1 || dim > 3) return fail(h, RBF_EINVAL, "dim must be 1..3");
    if (N < 1 || N > kMaxNodes) return fail(h, RBF_EINVAL, "N must be in 1..%" PRId64, (int64_t)kMaxNodes);
    if (!xyz_dev || !type_dev) return fail(h, RBF_EINVAL, "null node pointer");
    DeviceGuard g(h->device);
    drop_stencils(h);
    free_t(h, h->xyz);
    free_t(h, h->type);
    h->dim = 0;
    h->N = h->N_int = 0;
    std::vector<int8_t> th((size_t)N);
    HIPCHK(h, hipMemcpyAsync(th.data(), type_dev, (size_t)N, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    int64_t nint = 0, nneu = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (th[i] < 0 || th[i] > 2)
            return fail(h, RBF_EINVAL, "node %" PRId64 " has type %d (must be 0, 1 or 2)", i, (int)th[i]);
        nint += th[i] == 0;
        nneu += th[i] == 2;
    }
    free_t(h, h->normals);
    ALLOC(h, h->xyz, double, (size_t)dim * N);
    ALLOC(h, h->type, int8_t, N);
    HIPCHK(h, hipMemcpyAsync(h->xyz, xyz_dev, sizeof(double) * dim * N, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->type, type_dev, (size_t)N, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->dim = dim;
    h->N = N;
    h->N_int = nint;
    h->N_neu = nneu;
    h->type_h.swap(th);
    return RBF_OK;
}

rbf_status rbf_set_normals(rbf_handle *h, const double *normals_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (h->N == 0) return fail(h, RBF_EINVAL, "no nodes set");
    if (!normals_dev) return fail(h, RBF_EINVAL, "null normals");
    DeviceGuard g(h->device);
    const int64_t N = h->N;
    const int dim = h->dim;
    std::vector<double> nh((size_t)dim * N);
    HIPCHK(h, hipMemcpyAsync(nh.data(), normals_dev, sizeof(double) * dim * N, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < N; ++i) {
        if (h->type_h[i] != 2) continue;
        double s2 = 0.0;
        for (int a = 0; a < dim; ++a) s2 += nh[a * N + i] * nh[a * N + i];
        if (!(std::fabs(s2 - 1.0) <= 1e-12)) return fail(h, RBF_EINVAL, "Neumann node %" PRId64 ": normal is not a unit vector", i);
    }
    drop_weights(h);
    free_t(h, h->normals);
    ALLOC(h, h->normals, double, (size_t)dim * N);
    HIPCHK(h, hipMemcpyAsync(h->normals, normals_dev, sizeof(double) * dim * N, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return RBF_OK;
}

// ====================================================================== stencils
rbf_status rbf_build_stencils(rbf_handle *h, int32_t n_uniform, const int16_t *n_per_node_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (h->N == 0) return fail(h, RBF_EINVAL, "no nodes set");
    const int64_t N = h->N;
    const int dim = h->dim;
    DeviceGuard g(h->device);
    int32_t n_max = 0;
    if (n_uniform > 0) {
        if (n_uniform > N || n_uniform > kMaxSupport)
            return fail(h, RBF_EINVAL, "support size %d must be <= N (%" PRId64 ") and <= %d", n_uniform, N, kMaxSupport);
        n_max = n_uniform;
    } else {
        if (n_uniform != 0 || !n_per_node_dev) return fail(h, RBF_EINVAL, "need n_uniform > 0 or per-node sizes");
        std::vector<int16_t> nh((size_t)N);
        HIPCHK(h, hipMemcpyAsync(nh.data(), n_per_node_dev, sizeof(int16_t) * N, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int64_t i = 0; i < N; ++i) {
            if (nh[i] < 1 || nh[i] > N || nh[i] > kMaxSupport)
                return fail(h, RBF_EINVAL, "node %" PRId64 ": support size %d out of range", i, (int)nh[i]);
            n_max = std::max<int32_t>(n_max, nh[i]);
        }
    }
    // a Neumann node draws its support from itself and the interior nodes
    if (h->N_neu > 0 && n_max > h->N_int + 1)
        return fail(h, RBF_EINVAL, "Neumann supports of %d nodes need at least %d interior nodes", n_max, n_max - 1);
    drop_stencils(h);

    // bounding box
    const int nb = 512;
    double *partials = nullptr;
    ALLOC(h, partials, double, nb * 6);
    HIPCHK(h, launch_bbox_partials(h->stream, dim, N, h->xyz, partials, nb));
    std::vector<double> ph(nb * 6);
    HIPCHK(h, hipMemcpyAsync(ph.data(), partials, sizeof(double) * nb * 6, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    dfree(h, partials);
    CellGrid cg{};
    cg.dim = dim;
    double lo[3], hi[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
        for (int b = 0; b < nb; ++b) {
            lo[a] = std::min(lo[a], ph[b * 6 + 2 * a]);
            hi[a] = std::max(hi[a], ph[b * 6 + 2 * a + 1]);
        }
    }
    double maxext = 0.0;
    for (int a = 0; a < dim; ++a) {
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a])) return fail(h, RBF_EINVAL, "non-finite coordinates");
        maxext = std::max(maxext, hi[a] - lo[a]);
    }
    if (!(maxext > 0.0)) maxext = 1.0;
    int active = 0;
    for (int a = 0; a < dim; ++a)
        if (hi[a] - lo[a] > 1e-12 * maxext) {
            vol *= (hi[a] - lo[a]);
            ++active;
        }
    const double cell = active ? std::pow(vol / (double)N, 1.0 / active) : maxext;
    cg.ncells = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            const double ext = hi[a] - lo[a];
            int nc = ext > 1e-12 * maxext ? (int)std::floor(ext / cell) : 1;
            nc = std::max(1, std::min(nc, 1 << 20));
            cg.nc[a] = nc;
            cg.lo[a] = lo[a];
            cg.edge[a] = ext > 1e-12 * maxext ? ext / nc : maxext;
        } else {
            cg.nc[a] = 1;
            cg.lo[a] = 0.0;
            cg.edge[a] = 1.0;
        }
        cg.ncells *= cg.nc[a];
    }
    if (cg.ncells > INT32_MAX / 2) return fail(h, RBF_EINVAL, "cell grid too large");
    // n nodes at density N/vol fill a ball of radius (n * ball_coef)^(1/d)
    const double unit_ball = dim == 1 ? 2.0 : (dim == 2 ? M_PI : 4.0 * M_PI / 3.0);
    const double ball_coef = (active == dim ? vol : std::pow(maxext, dim)) / ((double)N * unit_ball);
    const double margin = 1e-12 * maxext;

    int32_t *cell_of = nullptr, *count = nullptr, *start = nullptr, *ids = nullptr, *cursor = nullptr, *scan = nullptr;
    double *xyz_c = nullptr;
    const int64_t nscan = (cg.ncells + 1023) / 1024 + 1;
    ALLOC(h, cell_of, int32_t, N);
    ALLOC(h, count, int32_t, cg.ncells);
    ALLOC(h, start, int32_t, cg.ncells + 1);
    ALLOC(h, ids, int32_t, N);
    ALLOC(h, cursor, int32_t, cg.ncells);
    ALLOC(h, scan, int32_t, nscan);
    ALLOC(h, xyz_c, double, (size_t)dim * N);
    HIPCHK(h, hipMemsetAsync(count, 0, sizeof(int32_t) * cg.ncells, h->stream));
    HIPCHK(h, hipMemsetAsync(cursor, 0, sizeof(int32_t) * cg.ncells, h->stream));
    HIPCHK(h, launch_bin_nodes(h->stream, cg, N, h->xyz, cell_of, count, start, ids, cursor, scan));
    HIPCHK(h, launch_coords_by_cell(h->stream, dim, N, h->xyz, ids, xyz_c));

    ALLOC(h, h->sten, int32_t, (size_t)N * n_max);
    ALLOC(h, h->nrow, int16_t, N);
    rbf_status st = reset_status(h);
    if (st) return st;
    HIPCHK(h, launch_knn_query(h->stream, cg, N, h->xyz, xyz_c, cell_of, start, ids, n_uniform, n_per_node_dev,
                               n_max, ball_coef, margin, h->sten, h->nrow, h->type, h->dstatus));
    DevStatus ds;
    st = read_status(h, &ds);
    dfree(h, cell_of);
    dfree(h, count);
    dfree(h, start);
    dfree(h, ids);
    dfree(h, cursor);
    dfree(h, scan);
    dfree(h, xyz_c);
    if (st) return st;
    if (ds.code != 0) {
        drop_stencils(h);
        return fail(h, ds.code, "neighbour search failed at node %" PRId64 " (%s)", ds.info, rbf_status_string(ds.code));
    }
    h->n_max = n_max;
    h->nrow_h.resize((size_t)N);
    HIPCHK(h, hipMemcpyAsync(h->nrow_h.data(), h->nrow, sizeof(int16_t) * N, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->have_sten = true;
    return RBF_OK;
}

// ====================================================================== packed operator
// Sliced operator over internal rows [row0, row0 + nrows) (perm gives their
// canonical ids); with wself, each row's own weight is split out (Neumann rows).
// 16-bit segment codes for the column ids of a packed operator in layout 1
// (the sweeps' index stream at half the bytes); the block number of an id
// must fit in 16 bits.  slen: the slice lengths.  RBF_ELL_CODES=0 skips them.
static rbf_status attach_codes(rbf_handle *h, Ell &e, const std::vector<int32_t> &slen) {
    const char *cenv = std::getenv("RBF_ELL_CODES");
    if (e.layout != 1 || !e.nslices || (cenv && cenv[0] == '0') || h->N >= ((int64_t)1 << 28)) return RBF_OK;
    std::vector<int64_t> cp((size_t)e.nslices + 1);
    cp[0] = 0;
    for (int64_t s = 0; s < e.nslices; ++s) cp[s + 1] = cp[s] + (int64_t)kSlice * ((slen[s] + 3) & ~3);
    e.celems = cp[e.nslices];
    ALLOC(h, e.code, uint16_t, e.celems);
    ALLOC(h, e.cptr, int64_t, e.nslices + 1);
    ALLOC(h, e.segbase, int32_t, (size_t)kSegs * e.nslices);
    ALLOC(h, e.cmode, int8_t, e.nslices);
    if (e.w32) ALLOC(h, e.w32q, float, e.celems);
    HIPCHK(h, hipMemcpyAsync(e.cptr, cp.data(), sizeof(int64_t) * (e.nslices + 1), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_encode_codes(h->stream, e));
    // every code decoded back and compared with its 32-bit id; a slice that
    // fails keeps reading its ids
    HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, h->dslots + 4));
    HIPCHK(h, launch_check_codes(h->stream, e, h->dslots + 4));
    HIPCHK(h, hipMemcpyAsync(h->hslots + 4, h->dslots + 4, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             h->stream));
    std::vector<int8_t> cm((size_t)e.nslices);
    HIPCHK(h, hipMemcpyAsync(cm.data(), e.cmode, (size_t)e.nslices, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    e.code_mismatches = (int64_t)h->hslots[4];
    e.coded_slices = 0;
    for (int8_t c : cm) e.coded_slices += c;
    return RBF_OK;
}

static rbf_status make_ell(rbf_handle *h, int64_t row0, int64_t nrows, const std::vector<int32_t> &perm, int layout,
                           int keep_fp32, Ell *out, double *wself, bool with_codes, int32_t *foreign = nullptr) {
    Ell e;
    e.layout = layout;
    e.ncols = h->N;
    e.nslices = (nrows + kSlice - 1) / kSlice;
    std::vector<int64_t> sptr((size_t)e.nslices + 1);
    std::vector<int32_t> slen((size_t)e.nslices);
    int64_t acc = 0;
    int32_t mx = 0;
    for (int64_t s = 0; s < e.nslices; ++s) {
        int32_t len = 0;
        for (int64_t i = s * kSlice; i < std::min<int64_t>(nrows, (s + 1) * kSlice); ++i)
            len = std::max<int32_t>(len, h->nrow_h[perm[row0 + i]]);
        if (e.layout == 1) len += len & 1;
        slen[s] = len;
        sptr[s] = acc;
        acc += (int64_t)len * kSlice;
        mx = std::max(mx, len);
    }
    sptr[e.nslices] = acc;
    e.elems = acc;
    e.max_len = mx;
    e.uniform_len = mx;
    for (int64_t s = 0; s < e.nslices; ++s)
        if (slen[s] != mx) e.uniform_len = 0;
    ALLOC(h, e.slice_ptr, int64_t, e.nslices + 1);
    ALLOC(h, e.slice_len, int32_t, std::max<int64_t>(1, e.nslices));
    ALLOC(h, e.idx, int32_t, std::max<int64_t>(1, e.elems));
    ALLOC(h, e.w, double, std::max<int64_t>(1, e.elems));
    if (keep_fp32) ALLOC(h, e.w32, float, std::max<int64_t>(1, e.elems));
    *out = e;
    HIPCHK(h, hipMemcpyAsync(e.slice_ptr, sptr.data(), sizeof(int64_t) * (e.nslices + 1), hipMemcpyHostToDevice, h->stream));
    if (e.nslices) {
        HIPCHK(h, hipMemcpyAsync(e.slice_len, slen.data(), sizeof(int32_t) * e.nslices, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, launch_pack_ell(h->stream, row0, nrows, h->n_max, h->perm, h->iperm, h->sten, h->nrow, h->w_can, e,
                                  wself, foreign));
    }
    if (with_codes) {
        const rbf_status st = attach_codes(h, e, slen);
        if (st) return st;
        *out = e;
    }
    return RBF_OK;
}

// Autotuner cache key of the sweep shape for the current operator (prec 0:
// FP64 sweeps, 1: FP32).
static void sweep_key(const rbf_handle *h, int prec, char *key, size_t len) {
    const Ell &e = h->ell;
    // problems with Neumann rows sweep in two parts around the Neumann update:
    // their own key, even where the interior operator has the same shape
    char neu[32] = "";
    if (h->N_neu > 0) std::snprintf(neu, sizeof neu, "|nn%" PRId64, h->N_neu);
    std::snprintf(key, len, "%s|%s|L%d|%" PRId64 "|%" PRId64 "|%d|c%" PRId64 "%s", prec ? "sweep32" : "sweep", h->arch,
                  e.layout, h->N_int, e.elems, e.max_len, e.coded_slices, neu);
}

// Apply cached shape values v[8] to c.
static void apply_shape(SweepCfg &c, const int *v, const Ell &e) {
    c.waves_per_block = v[0];
    c.unroll = v[1];
    c.xcd_remap = v[2];
    c.pipeline = e.layout ? v[3] : 0;
    c.zigzag = v[4];
    c.codes = e.cmode ? v[5] : 0;
    c.temporal = c.codes ? v[6] : 0;
    c.quad = (c.codes && e.w32q) ? v[7] : 0;
}

// Cached shape of `key` into v[8]; older entries hold 6 or 7 values (the
// missing choices 0).
static bool lookup_shape(const char *key, int *v) {
    v[6] = v[7] = 0;
    return cache_lookup(key, v, 8) || cache_lookup(key, v, 7) || cache_lookup(key, v, 6);
}

// RBF_SWEEP_ZIGZAG=0/1 fixes the sweep order (forward only / alternating) and
// RBF_SWEEP_CODES=0/1 whether the sweeps read the 16-bit codes; unset, the
// autotuner chooses.  -1 when unset.
static int env_flag(const char *name) {
    const char *z = std::getenv(name);
    if (!z || !z[0]) return -1;
    return z[0] == '1' ? 1 : 0;
}
static int zigzag_override() { return env_flag("RBF_SWEEP_ZIGZAG"); }
// RBF_NEUMANN_OVERLAP=1 forks each step of a Neumann problem (the far
// interior slices swept beside the Neumann update, then the rest).  Off by
// default: on MI355X the sequential step measured faster (0.139 vs 0.148 ms
// at 1M interior rows), the second sweep launch costing more than the hidden
// update.
static bool overlap_neumann() { return env_flag("RBF_NEUMANN_OVERLAP") == 1; }
static int codes_override() { return env_flag("RBF_SWEEP_CODES"); }

// RBF_SWEEP_SHAPE="waves,unroll,xcd_remap,pipeline,zigzag,codes[,temporal[,quad]]"
// fixes the whole sweep shape (both precisions) and turns the sweep
// autotuner off.
static bool shape_override(SweepCfg *c) {
    const char *z = std::getenv("RBF_SWEEP_SHAPE");
    if (!z || !z[0]) return false;
    int v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int got =
        std::sscanf(z, "%d,%d,%d,%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7]);
    if (got < 6) return false;
    // 32-entry groups exist only for the FP32 sweep reading weights in the code
    // layout; the FP64 sweeps then use 16
    const bool quad = got >= 8 && v[7] && v[5];
    if ((v[0] != 2 && v[0] != 4 && v[0] != 8) || (v[1] != 4 && v[1] != 8 && v[1] != 16 && !(v[1] == 32 && quad)))
        return false;
    c->waves_per_block = v[0];
    c->unroll = v[1];
    c->xcd_remap = v[2] != 0;
    c->pipeline = v[3] != 0;
    c->zigzag = v[4] != 0;
    c->codes = v[5] != 0;
    c->temporal = c->codes && v[6] != 0;
    c->quad = c->codes && v[7] != 0;
    return true;
}

// Internal order: interior rows by descending support size then canonical id,
// then Neumann rows likewise, then Dirichlet rows by canonical id.
static rbf_status finalize_operator(rbf_handle *h, int keep_fp32) {
    drop_operator(h);
    const int64_t N = h->N, N_int = h->N_int, N_neu = h->N_neu;
    std::vector<int32_t> perm((size_t)N), iperm((size_t)N);
    // With Neumann nodes, interior rows whose supports hold no Neumann node
    // ("far" rows) come first, so a step can sweep them while the Neumann
    // values are being updated.
    std::vector<int8_t> near((size_t)N, 0);
    if (N_neu > 0) {
        int8_t *d_near = nullptr;
        ALLOC(h, d_near, int8_t, N);
        HIPCHK(h, launch_flag_near(h->stream, N, h->n_max, h->sten, h->nrow, h->type, d_near));
        HIPCHK(h, hipMemcpyAsync(near.data(), d_near, (size_t)N, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        dfree(h, d_near);
    }
    int64_t n_far = 0;
    {
        // groups: 0 far interior, 1 near interior, 2 Neumann; each by descending
        // support size, then canonical id
        auto group = [&](int64_t i) { return h->type_h[i] == 2 ? 2 : (int)near[i]; };
        const int G = kMaxSupport + 2;
        std::vector<int64_t> cnt(3 * G, 0);
        for (int64_t i = 0; i < N; ++i)
            if (h->type_h[i] != 1) cnt[group(i) * G + h->nrow_h[i]]++;
        std::vector<int64_t> off(3 * G, 0);
        int64_t acc = 0;
        for (int g = 0; g < 3; ++g)
            for (int n = kMaxSupport; n >= 1; --n) {
                off[g * G + n] = acc;
                acc += cnt[g * G + n];
                if (g == 0) n_far += cnt[g * G + n];
            }
        int64_t bpos = N_int + N_neu;
        for (int64_t i = 0; i < N; ++i) {
            if (h->type_h[i] == 1) perm[bpos++] = (int32_t)i;
            else perm[off[group(i) * G + h->nrow_h[i]]++] = (int32_t)i;
        }
        for (int64_t k = 0; k < N; ++k) iperm[perm[k]] = (int32_t)k;
    }
    h->far_slices = N_neu > 0 ? n_far / kSlice : 0;
    ALLOC(h, h->perm, int32_t, N);
    ALLOC(h, h->iperm, int32_t, N);
    HIPCHK(h, hipMemcpyAsync(h->perm, perm.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->iperm, iperm.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, h->stream));
    // packed layout: entry pairs as vectors unless RBF_ELL_LAYOUT=0
    const char *lay = std::getenv("RBF_ELL_LAYOUT");
    const int layout = (lay && lay[0] == '0') ? 0 : 1;
    rbf_status st = make_ell(h, 0, N_int, perm, layout, keep_fp32, &h->ell, nullptr, true);
    if (st) return st;
    Ell &e = h->ell;
    if (N_neu > 0) {
        ALLOC(h, h->wself, double, N_neu);
        ALLOC(h, h->nb, double, N_neu);
        HIPCHK(h, launch_fill_f64(h->stream, N_neu, 0.0, h->wself));
        HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, h->dslots + 3));
        st = make_ell(h, N_int, N_neu, perm, layout, 0, &h->ellN, h->wself, false, (int32_t *)(h->dslots + 3));
        if (st) return st;
        HIPCHK(h, hipMemcpyAsync(h->hslots + 3, h->dslots + 3, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->neu_direct = h->hslots[3] == 0;
        // each Neumann row divides by its own weight: it must be present and nonzero
        std::vector<double> ws((size_t)N_neu);
        HIPCHK(h, hipMemcpyAsync(ws.data(), h->wself, sizeof(double) * N_neu, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int64_t j = 0; j < N_neu; ++j)
            if (!(std::fabs(ws[j]) > 0.0) || !std::isfinite(ws[j])) {
                const int64_t r = perm[N_int + j];
                drop_operator(h);
                h->have_w = false;
                return fail(h, RBF_EINVAL, "Neumann node %" PRId64 ": own weight missing, zero or not finite", r);
            }
    }
    ALLOC(h, h->ua, double, N);
    ALLOC(h, h->ub, double, N);
    ALLOC(h, h->fint, double, N);
    ALLOC(h, h->tmp, double, N);
    ALLOC(h, h->uref, double, N);
    ALLOC(h, h->part, double, kErrBlocks + 8);
    ALLOC(h, h->ea, float, N);
    ALLOC(h, h->eb, float, N);
    ALLOC(h, h->r32, float, N);
    HIPCHK(h, launch_fill_f32(h->stream, N, 0.0f, h->ea));
    HIPCHK(h, launch_fill_f32(h->stream, N, 0.0f, h->eb));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->have_w32 = keep_fp32 != 0;
    // a tuned shape for this operator, if cached
    char key[160];
    int v[8];
    for (int prec = 0; prec < 2; ++prec) {
        sweep_key(h, prec, key, sizeof key);
        if (lookup_shape(key, v)) apply_shape(prec ? h->cfg32 : h->cfg, v, e);
    }
    const int zz = zigzag_override();
    if (zz >= 0) h->cfg.zigzag = h->cfg32.zigzag = zz;
    const int cd = codes_override();
    if (cd >= 0) h->cfg.codes = h->cfg32.codes = (cd && e.cmode) ? 1 : 0;
    SweepCfg forced;
    if (shape_override(&forced)) {
        if (!e.layout) forced.pipeline = 0;
        if (!e.cmode) forced.codes = forced.temporal = 0;
        if (!forced.codes || !e.w32q) forced.quad = 0;
        if (!forced.quad && forced.unroll > 16) forced.unroll = 16;
        h->cfg = h->cfg32 = forced;
        h->cfg.quad = 0;
        h->cfg.unroll = std::min(h->cfg.unroll, 16);
    }
    return RBF_OK;
}

// ====================================================================== weights
// RBF_WEIGHTS_SOLVER=gepp: every system larger than the one-wavefront size
// by the blocked elimination in the oracle's operation order (bit-equal to
// the oracle); unset or "ns": the null-space solver where it applies.
static bool weights_solver_ns() {
    const char *v = std::getenv("RBF_WEIGHTS_SOLVER");
    return !(v && std::strcmp(v, "gepp") == 0);
}

extern "C" rbf_status rbf_compute_weights(rbf_handle *h, int32_t m_uniform, const int8_t *m_per_node_dev,
                                          int keep_fp32) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_sten) return fail(h, RBF_EINVAL, "no stencils set");
    const int64_t N = h->N;
    const int dim = h->dim;
    DeviceGuard g(h->device);
    std::vector<int8_t> mh((size_t)N, (int8_t)m_uniform);
    if (m_uniform < 0) {
        if (!m_per_node_dev) return fail(h, RBF_EINVAL, "need m_uniform >= 0 or per-node orders");
        HIPCHK(h, hipMemcpyAsync(mh.data(), m_per_node_dev, (size_t)N, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    for (int64_t i = 0; i < N; ++i)
        if (h->type_h[i] != 1 && (mh[i] < 0 || mh[i] > kMaxOrder))
            return fail(h, RBF_EINVAL, "node %" PRId64 ": order %d not in 0..%d", i, (int)mh[i], kMaxOrder);
    if (h->N_neu > 0 && !h->normals) return fail(h, RBF_EINVAL, "Neumann nodes need normals (rbf_set_normals)");
    drop_weights(h);

    // group interior rows by (n, m) (a counting sort on the key 8 n + m, rows
    // in ascending id within a class); classes by descending system size
    constexpr int kKeys = 8 * (kMaxSupport + 1);
    std::vector<int64_t> kcount(kKeys + 1, 0);
    for (int64_t i = 0; i < N; ++i)
        if (h->type_h[i] != 1) ++kcount[8 * h->nrow_h[i] + mh[i] + 1];
    for (int k = 0; k < kKeys; ++k) kcount[k + 1] += kcount[k];
    std::vector<int32_t> grouped((size_t)kcount[kKeys]);
    {
        std::vector<int64_t> pos(kcount.begin(), kcount.end() - 1);
        for (int64_t i = 0; i < N; ++i)
            if (h->type_h[i] != 1) grouped[(size_t)pos[8 * h->nrow_h[i] + mh[i]]++] = (int32_t)i;
    }
    struct Cls { int S, n, m; int64_t begin, end; };
    std::vector<Cls> order;
    for (int k = 0; k < kKeys; ++k)
        if (kcount[k + 1] > kcount[k])
            order.push_back({k / 8 + num_monomials(dim, k % 8), k / 8, k % 8, kcount[k], kcount[k + 1]});
    std::sort(order.begin(), order.end(), [](const Cls &a, const Cls &b) { return a.S > b.S || (a.S == b.S && a.n > b.n); });
    std::vector<int32_t> rows;
    std::vector<int8_t> mrows;
    const size_t isz = weights_item_bytes();
    std::vector<char> items;
    // null-space systems: one launch per register-array size (items, largest
    // system's LDS in doubles)
    std::map<int, std::pair<std::vector<char>, int>> ns_launch;
    int S_small = 0, S_large = 0;
    int64_t nitems = 0, nlarge = 0, nitems_ns = 0;
    const bool ns_on = weights_solver_ns();
    size_t lds_limit = 0;
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess)
            lds_limit = (size_t)v;
    }
    for (auto &c : order) {
        // systems of at most weights_small_limit() unknowns: one wavefront
        // each, matrix in LDS; larger ones with m >= 1 whose working set fits
        // the null-space solver's LDS layout: that solver, one workgroup each;
        // the rest: blocked elimination, one workgroup each
        int kind = c.S <= weights_small_limit() ? 0 : 1;
        if (kind == 1 && ns_on && c.m >= 1 && ns_fits(dim, c.n, c.S - c.n, lds_limit - 64)) kind = 2;
        if (kind == 0) S_small = std::max(S_small, c.S);
        if (kind == 1) S_large = std::max(S_large, c.S);
        const int bucket = kind == 2 ? ns_bucket(dim, c.n, c.S - c.n) : 0;
        if (kind == 2) {
            int &mx = ns_launch[bucket].second;
            mx = std::max(mx, ns_lds_doubles(c.n, c.S - c.n, bucket));
        }
        const int per = kind == 0 ? 4 : 1;
        const int64_t first = (int64_t)rows.size(), cnt = c.end - c.begin;
        rows.insert(rows.end(), grouped.begin() + c.begin, grouped.begin() + c.end);
        mrows.insert(mrows.end(), (size_t)cnt, (int8_t)c.m);
        std::vector<char> &dst = kind == 2 ? ns_launch[bucket].first : items;
        size_t at = dst.size();
        dst.resize(at + (size_t)((cnt + per - 1) / per) * isz);
        for (int64_t q = 0; q < cnt; q += per, at += isz) {
            weights_make_item(dst.data() + at, kind == 2 ? 1 : kind, (int)std::min<int64_t>(per, cnt - q), first + q);
            if (kind == 2) {
                ++nitems_ns;
            } else {
                ++nitems;
                nlarge += kind == 1;
            }
        }
    }
    h->w_ns_systems = nitems_ns;
    h->w_elim_systems = (int64_t)rows.size() - nitems_ns;
    ALLOC(h, h->w_can, double, (size_t)N * h->n_max);
    HIPCHK(h, launch_fill_f64(h->stream, N * (int64_t)h->n_max, 0.0, h->w_can));
    if (nitems_ns > 0) {
        // null-space systems (one persistent launch per register-array size), before the others
        int32_t *d_rows = nullptr, *counter = nullptr;
        int8_t *d_m = nullptr;
        ALLOC(h, d_rows, int32_t, rows.size());
        ALLOC(h, d_m, int8_t, mrows.size());
        ALLOC(h, counter, int32_t, 4);
        HIPCHK(h, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(d_m, mrows.data(), mrows.size(), hipMemcpyHostToDevice, h->stream));
        rbf_status st = reset_status(h);
        if (st) return st;
        std::vector<char *> d_items;
        for (auto &kv : ns_launch) {
            const std::vector<char> &its = kv.second.first;
            char *di = nullptr;
            ALLOC(h, di, char, its.size());
            d_items.push_back(di);
            HIPCHK(h, hipMemcpyAsync(di, its.data(), its.size(), hipMemcpyHostToDevice, h->stream));
            const size_t lds = ((size_t)kv.second.second * sizeof(double) + 255) & ~(size_t)255;
            const int grid = weights_ns_grid(dim, kv.first, lds);
            if (grid <= 0) return fail(h, RBF_EHIP, "null-space weight solver does not fit on the device");
            HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, (unsigned long long *)counter));
            HIPCHK(h, launch_weights_ns(h->stream, dim, kv.first, N, h->xyz, h->sten, h->nrow, h->n_max, d_rows, d_m,
                                        h->type, h->normals, h->w_can, h->dstatus, di,
                                        (int64_t)(its.size() / isz), counter, lds, grid));
        }
        DevStatus ds;
        st = read_status(h, &ds);
        dfree(h, d_rows);
        dfree(h, d_m);
        for (char *di : d_items) dfree(h, di);
        dfree(h, counter);
        if (st) return st;
        if (ds.code != 0) {
            free_t(h, h->w_can);
            return fail(h, ds.code, "singular local system at node %" PRId64, ds.info);
        }
    }
    if (nitems > 0) {
        int32_t *d_rows = nullptr, *counter = nullptr;
        int8_t *d_m = nullptr;
        char *d_items = nullptr;
        double *scratch = nullptr;
        ALLOC(h, d_rows, int32_t, rows.size());
        ALLOC(h, d_m, int8_t, mrows.size());
        ALLOC(h, d_items, char, items.size());
        ALLOC(h, counter, int32_t, 4);
        HIPCHK(h, hipMemcpyAsync(d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(d_m, mrows.data(), mrows.size(), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(d_items, items.data(), items.size(), hipMemcpyHostToDevice, h->stream));
        const int64_t slab = weights_slab(S_large);
        const int cand[2] = {8, 16};
        auto fits = [&](int pc) {
            return weights_grid(S_small, S_large, pc) > 0 && (S_large == 0 || weights_grid(0, S_large, pc) > 0);
        };
        // Every LARGE workgroup indexes its own scratch slab by blockIdx, so the
        // slab count must cover the largest grid launched below: the full
        // launch (all item kinds) and the panel-timing launches (LARGE items
        // only, smaller LDS footprint, hence possibly more resident groups).
        int grid_max = 0;
        for (int pc : cand) {
            grid_max = std::max(grid_max, weights_grid(S_small, S_large, pc));
            if (S_large > 0) grid_max = std::max(grid_max, weights_grid(0, S_large, pc));
        }
        if (grid_max <= 0) return fail(h, RBF_EHIP, "weight solver does not fit on the device");
        int panel_fit = 0;  // largest panel width whose LDS footprint fits
        for (int pc : cand)
            if (fits(pc)) panel_fit = pc;
        if (panel_fit == 0) return fail(h, RBF_EHIP, "weight solver does not fit on the device");
        if (S_large > 0) ALLOC(h, scratch, double, (size_t)slab * grid_max);
        // panel width: cached choice, else time the candidates on a sample
        int panel = h->weights_panel;
        if (S_large > 0) {
            char key[160];
            std::snprintf(key, sizeof key, "weights|%s|%d|%d", h->arch, dim, S_large);
            int v[1];
            const int forced = std::getenv("RBF_WEIGHTS_PANEL") ? std::atoi(std::getenv("RBF_WEIGHTS_PANEL")) : 0;
            if ((forced == 8 || forced == 16) && fits(forced)) {
                panel = forced;
            } else if (cache_lookup(key, v, 1) && (v[0] == 8 || v[0] == 16) && fits(v[0])) {
                panel = v[0];
            } else if (nlarge >= 4096) {
                float best = 1e30f;
                const int64_t sample = std::min<int64_t>(nlarge, 4 * grid_max);
                for (int pc : cand) {
                    if (!fits(pc)) continue;
                    HIPCHK(h, hipMemsetAsync(counter, 0, sizeof(int32_t), h->stream));
                    HIPCHK(h, hipEventRecord(h->ev0, h->stream));
                    HIPCHK(h, launch_weights_items(h->stream, dim, N, h->xyz, h->sten, h->nrow, h->n_max, d_rows, d_m,
                                                   h->type, h->normals, h->w_can, scratch, slab, pc, h->dstatus,
                                                   d_items, sample, counter,
                                                   0, S_large, weights_grid(0, S_large, pc), grid_max,
                                                   nullptr));
                    HIPCHK(h, hipEventRecord(h->ev1, h->stream));
                    HIPCHK(h, hipEventSynchronize(h->ev1));
                    float ms = 0.f;
                    HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
                    if (ms < best) {
                        best = ms;
                        panel = pc;
                    }
                }
                v[0] = panel;
                cache_store(key, v, 1);
            }
            if (!fits(panel)) panel = panel_fit;
            h->weights_panel = panel;
        }
        rbf_status st = reset_status(h);
        if (st) return st;
        HIPCHK(h, hipMemsetAsync(counter, 0, sizeof(int32_t), h->stream));
        HIPCHK(h, launch_weights_items(h->stream, dim, N, h->xyz, h->sten, h->nrow, h->n_max, d_rows, d_m, h->type,
                                       h->normals, h->w_can, scratch, slab, panel, h->dstatus, d_items, nitems,
                                       counter, S_small,
                                       S_large, weights_grid(S_small, S_large, panel), grid_max, nullptr));
        DevStatus ds;
        st = read_status(h, &ds);
        dfree(h, d_rows);
        dfree(h, d_m);
        dfree(h, d_items);
        dfree(h, counter);
        if (scratch) dfree(h, scratch);
        if (st) return st;
        if (ds.code != 0) {
            free_t(h, h->w_can);
            return fail(h, ds.code, "singular local system at node %" PRId64, ds.info);
        }
    }
    h->have_w = true;
    return finalize_operator(h, keep_fp32);
}

// ====================================================================== import / export
extern "C" rbf_status rbf_get_stencils(rbf_handle *h, int32_t *idx_host) {
    if (!h || !idx_host) return RBF_EINVAL;
    if (!h->have_sten) return fail(h, RBF_EINVAL, "no stencils set");
    DeviceGuard g(h->device);
    HIPCHK(h, hipMemcpyAsync(idx_host, h->sten, sizeof(int32_t) * h->N * h->n_max, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return RBF_OK;
}

extern "C" rbf_status rbf_get_weights(rbf_handle *h, double *w_host) {
    if (!h || !w_host) return RBF_EINVAL;
    if (!h->have_w) return fail(h, RBF_EINVAL, "no weights set");
    DeviceGuard g(h->device);
    HIPCHK(h, hipMemcpyAsync(w_host, h->w_can, sizeof(double) * h->N * h->n_max, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return RBF_OK;
}

extern "C" rbf_status rbf_set_stencils(rbf_handle *h, const int32_t *idx_host, int32_t n_max) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (h->N == 0) return fail(h, RBF_EINVAL, "no nodes set");
    if (!idx_host || n_max < 1 || n_max > kMaxSupport) return fail(h, RBF_EINVAL, "bad stencil array or n_max");
    const int64_t N = h->N;
    std::vector<int16_t> nr((size_t)N);
    std::vector<int32_t> row;
    for (int64_t r = 0; r < N; ++r) {
        int n = 0;
        while (n < n_max && idx_host[r * n_max + n] >= 0) ++n;
        if (n == 0) return fail(h, RBF_EINVAL, "row %" PRId64 " has an empty stencil", r);
        for (int k = 0; k < n_max; ++k) {
            const int32_t v = idx_host[r * n_max + k];
            if (k < n && v >= N) return fail(h, RBF_EINVAL, "row %" PRId64 ": id %d out of range", r, v);
            if (k >= n && v != -1) return fail(h, RBF_EINVAL, "row %" PRId64 ": padding must be -1", r);
        }
        // the packed layout places each entry by its rank among the row's ids
        row.assign(idx_host + r * n_max, idx_host + r * n_max + n);
        std::sort(row.begin(), row.end());
        if (std::adjacent_find(row.begin(), row.end()) != row.end())
            return fail(h, RBF_EINVAL, "row %" PRId64 ": repeated node id in the stencil", r);
        nr[r] = (int16_t)n;
    }
    DeviceGuard g(h->device);
    drop_stencils(h);
    ALLOC(h, h->sten, int32_t, (size_t)N * n_max);
    ALLOC(h, h->nrow, int16_t, N);
    HIPCHK(h, hipMemcpyAsync(h->sten, idx_host, sizeof(int32_t) * N * n_max, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->nrow, nr.data(), sizeof(int16_t) * N, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->n_max = n_max;
    h->nrow_h.swap(nr);
    h->have_sten = true;
    return RBF_OK;
}

extern "C" rbf_status rbf_set_weights(rbf_handle *h, const double *w_host, int keep_fp32) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    h->w_ns_systems = h->w_elim_systems = 0;
    if (!h->have_sten) return fail(h, RBF_EINVAL, "no stencils set");
    if (!w_host) return fail(h, RBF_EINVAL, "null weights");
    const int64_t N = h->N, nm = h->n_max;
    std::vector<double> w((size_t)N * nm);
    for (int64_t r = 0; r < N; ++r)
        for (int64_t k = 0; k < nm; ++k) {
            const bool live = h->type_h[r] != 1 && k < h->nrow_h[r];
            w[r * nm + k] = live ? w_host[r * nm + k] : 0.0;
        }
    DeviceGuard g(h->device);
    drop_weights(h);
    ALLOC(h, h->w_can, double, (size_t)N * nm);
    HIPCHK(h, hipMemcpyAsync(h->w_can, w.data(), sizeof(double) * N * nm, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->have_w = true;
    return finalize_operator(h, keep_fp32);
}

// ====================================================================== operators
extern "C" rbf_status rbf_apply(rbf_handle *h, const double *u_dev, double *Lu_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!u_dev || !Lu_dev) return fail(h, RBF_EINVAL, "null pointer");
    DeviceGuard g(h->device);
    const int64_t N = h->N, Ni = h->N_int;
    HIPCHK(h, launch_gather(h->stream, N, h->perm, u_dev, h->ua));
    HIPCHK(h, launch_fill_f64(h->stream, N - Ni, 0.0, h->tmp + Ni));
    if (Ni) HIPCHK(h, launch_apply_f64(h->stream, h->cfg, h->ell, Ni, h->ua, h->tmp, nullptr, nullptr));
    if (h->N_neu) HIPCHK(h, launch_neumann_apply(h->stream, h->ellN, Ni, h->N_neu, h->wself, h->ua, h->tmp));
    HIPCHK(h, launch_scatter(h->stream, N, h->perm, h->tmp, Lu_dev));
    return RBF_OK;
}

// The transposed interior operator in the sliced layout (built once per
// operator): column c of L_II becomes row c of L_II^T, its entries sorted by
// row so that the gather sums in a fixed order.
static rbf_status build_transpose(rbf_handle *h) {
    if (h->ellT.idx || !h->N_int) return RBF_OK;
    const int64_t N = h->N, Ni = h->N_int;
    int32_t *cnt = nullptr, *cursor = nullptr, *rows_t = nullptr;
    int64_t *start = nullptr;
    double *w_t = nullptr;
    ALLOC(h, cnt, int32_t, Ni);
    HIPCHK(h, hipMemsetAsync(cnt, 0, sizeof(int32_t) * Ni, h->stream));
    HIPCHK(h, launch_tcount(h->stream, N, h->n_max, Ni, h->type, h->iperm, h->sten, h->nrow, cnt));
    std::vector<int32_t> ch((size_t)Ni);
    HIPCHK(h, hipMemcpyAsync(ch.data(), cnt, sizeof(int32_t) * Ni, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::vector<int64_t> st((size_t)Ni + 1);
    st[0] = 0;
    for (int64_t c = 0; c < Ni; ++c) st[c + 1] = st[c] + ch[c];
    const int64_t nnz = st[Ni];
    Ell e;
    e.layout = 1;
    e.ncols = N;
    e.nslices = (Ni + kSlice - 1) / kSlice;
    std::vector<int64_t> sptr((size_t)e.nslices + 1);
    std::vector<int32_t> slen((size_t)e.nslices);
    int64_t acc = 0;
    for (int64_t s = 0; s < e.nslices; ++s) {
        int32_t len = 0;
        for (int64_t c = s * kSlice; c < std::min<int64_t>(Ni, (s + 1) * kSlice); ++c) len = std::max(len, ch[c]);
        len += len & 1;
        slen[s] = len;
        sptr[s] = acc;
        acc += (int64_t)len * kSlice;
        e.max_len = std::max(e.max_len, len);
    }
    sptr[e.nslices] = acc;
    e.elems = acc;
    // lanes of each slice by decreasing row length (ties by row), so that the
    // padding of a slice sits in whole cache lines of its last lanes; none if
    // a row has 1024 entries or more (16-bit lane descriptors)
    std::vector<uint16_t> lm;
    if (e.max_len < 1024) {
        lm.resize((size_t)e.nslices * kSlice);
        int q[kSlice];
        for (int64_t s = 0; s < e.nslices; ++s) {
            for (int r = 0; r < kSlice; ++r) q[r] = r;
            auto cnt_of = [&](int r) { return s * kSlice + r < Ni ? ch[s * kSlice + r] : 0; };
            std::stable_sort(q, q + kSlice, [&](int a, int b) { return cnt_of(a) > cnt_of(b); });
            for (int p = 0; p < kSlice; ++p) lm[s * kSlice + p] = (uint16_t)(q[p] | (cnt_of(q[p]) << 6));
        }
    }
    ALLOC(h, start, int64_t, Ni + 1);
    ALLOC(h, cursor, int32_t, Ni);
    ALLOC(h, rows_t, int32_t, std::max<int64_t>(1, nnz));
    ALLOC(h, w_t, double, std::max<int64_t>(1, nnz));
    ALLOC(h, e.slice_ptr, int64_t, e.nslices + 1);
    ALLOC(h, e.slice_len, int32_t, e.nslices);
    ALLOC(h, e.idx, int32_t, std::max<int64_t>(1, e.elems));
    ALLOC(h, e.w, double, std::max<int64_t>(1, e.elems));
    if (!lm.empty()) ALLOC(h, e.lmeta, uint16_t, e.nslices * kSlice);
    HIPCHK(h, hipMemcpyAsync(start, st.data(), sizeof(int64_t) * (Ni + 1), hipMemcpyHostToDevice, h->stream));
    if (e.lmeta)
        HIPCHK(h, hipMemcpyAsync(e.lmeta, lm.data(), sizeof(uint16_t) * lm.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(e.slice_ptr, sptr.data(), sizeof(int64_t) * (e.nslices + 1), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(e.slice_len, slen.data(), sizeof(int32_t) * e.nslices, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemsetAsync(cursor, 0, sizeof(int32_t) * Ni, h->stream));
    HIPCHK(h, launch_tfill(h->stream, N, h->n_max, Ni, h->type, h->iperm, h->sten, h->nrow, h->w_can, start, cursor,
                           rows_t, w_t));
    HIPCHK(h, launch_tpack(h->stream, Ni, start, rows_t, w_t, e));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    dfree(h, cnt);
    dfree(h, cursor);
    dfree(h, start);
    dfree(h, rows_t);
    dfree(h, w_t);
    h->ellT = e;
    const rbf_status cst = attach_codes(h, e, slen);
    h->ellT = e;
    return cst;
}

static bool use_scatter_transpose() {
    const char *v = std::getenv("RBF_TRANSPOSE_SCATTER");
    return v && v[0] == '1';
}

extern "C" rbf_status rbf_apply_transpose(rbf_handle *h, const double *v_dev, double *out_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!v_dev || !out_dev) return fail(h, RBF_EINVAL, "null pointer");
    DeviceGuard g(h->device);
    const int64_t N = h->N, Ni = h->N_int;
    HIPCHK(h, launch_gather(h->stream, N, h->perm, v_dev, h->ua));
    HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->tmp));
    if (Ni && use_scatter_transpose()) {
        HIPCHK(h, launch_transpose_scatter(h->stream, h->ell, Ni, h->ua, h->tmp));
    } else if (Ni) {
        rbf_status st = build_transpose(h);
        if (st) return st;
        HIPCHK(h, launch_apply_f64(h->stream, h->cfg, h->ellT, Ni, h->ua, h->tmp, nullptr, nullptr));
    }
    HIPCHK(h, launch_scatter(h->stream, N, h->perm, h->tmp, out_dev));
    return RBF_OK;
}

static rbf_status residual_internal(rbf_handle *h, const double *u_int, double *res) {
    HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, h->dslots));
    if (h->N_int)
        HIPCHK(h, launch_apply_f64(h->stream, h->cfg, h->ell, h->N_int, u_int, nullptr, h->fint, h->dslots));
    HIPCHK(h, hipMemcpyAsync(h->hslots, h->dslots, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *res = bits_to_double(h->hslots[0]);
    return RBF_OK;
}

extern "C" rbf_status rbf_residual(rbf_handle *h, const double *f_dev, const double *u_dev, double *res_host) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!f_dev || !u_dev || !res_host) return fail(h, RBF_EINVAL, "null pointer");
    DeviceGuard g(h->device);
    HIPCHK(h, launch_gather(h->stream, h->N, h->perm, u_dev, h->ua));
    HIPCHK(h, launch_gather(h->stream, h->N, h->perm, f_dev, h->fint));
    return residual_internal(h, h->ua, res_host);
}

// rbf_residual without allocating and without synchronising: the same
// gathers into internal order and the same residual kernel, with the staging
// vectors and the reduction slot in the static per-device workspace instead
// of the handle's buffers; the result goes to a device double.
extern "C" rbf_status rbf_residual_noalloc(rbf_handle *h, const double *f_dev, const double *u_dev, double *res_dev) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!f_dev || !u_dev || !res_dev) return fail(h, RBF_EINVAL, "null pointer");
    if (h->N > kNoAllocMaxNodes)
        return fail(h, RBF_EINVAL,
                    "rbf_residual_noalloc: %" PRId64 " nodes exceed its static workspace (at most %" PRId64 " nodes)",
                    h->N, kNoAllocMaxNodes);
    double *ws = noalloc_workspace(h->device);
    if (!ws)
        return fail(h, RBF_EHIP, "rbf_residual_noalloc: workspace address unavailable on device %d (%s)", h->device,
                    hipGetErrorString(h->noalloc_status));
    DeviceGuard g(h->device);
    double *u_int = ws, *f_int = ws + kNoAllocMaxNodes;
    unsigned long long *slot = reinterpret_cast<unsigned long long *>(ws + 2 * kNoAllocMaxNodes);
    HIPCHK(h, launch_gather(h->stream, h->N, h->perm, u_dev, u_int));
    HIPCHK(h, launch_gather(h->stream, h->N, h->perm, f_dev, f_int));
    HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, slot));  // the slot keeps the previous call's maximum
    if (h->N_int) HIPCHK(h, launch_apply_f64(h->stream, h->cfg, h->ell, h->N_int, u_int, nullptr, f_int, slot));
    HIPCHK(h, launch_slot_to_double(h->stream, slot, res_dev));
    return RBF_OK;
}

// ====================================================================== graphs
enum GraphKind { kGraphF64 = 0, kGraphMixed = 1, kGraphAdjoint = 2, kGraphF64Quiet = 3, kGraphAdjointHorner = 4 };

// FP64 chunk: reset the residual slot, `steps` sweeps alternating ua/ub
// (starting from ua when start == 0), the last one reporting max |rho|; with
// inner == 1 (the first chunk of a run) the first sweep also reports its
// max |rho|, the residual of the starting iterate, into slot 5.
static rbf_status get_graph(rbf_handle *h, int kind, int64_t steps, int start, double dt, int inner,
                            hipGraphExec_t *out) {
    const auto key = std::make_tuple(kind, steps, start + 2 * inner, double_bits(dt));
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return RBF_OK;
    }
    const int64_t Ni = h->N_int;
    hipStream_t s = h->cap;
    HIPCHK(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (kind == kGraphF64 || kind == kGraphF64Quiet) {
        const bool first = kind == kGraphF64 && inner == 1;
        if (kind == kGraphF64) e = launch_fill_u64(s, 1, 0ull, h->dslots);
        if (first && e == hipSuccess) e = launch_fill_u64(s, 1, 0ull, h->dslots + 5);
        double *a = start ? h->ub : h->ua, *b = start ? h->ua : h->ub;
        // With Neumann nodes updated in place, a step forks: the far interior
        // slices (whose rows read no Neumann value) are swept on a second
        // capture stream while the Neumann values are updated, then the
        // remaining slices are swept.  Same per-row arithmetic as one sweep.
        const bool fork = h->N_neu > 0 && h->neu_direct && h->far_slices > 0 && overlap_neumann();
        for (int64_t i = 0; i < steps && e == hipSuccess; ++i) {
            const bool report = kind == kGraphF64 && i == steps - 1;
            unsigned long long *slot = report ? h->dslots : (first && i == 0 ? h->dslots + 5 : nullptr);
            const int par = (int)(i & 1);
            if (fork) {
                // the small Neumann launch is queued first so its workgroups
                // are placed before the far sweep fills the device
                e = hipEventRecord(h->evf[0], s);
                if (e == hipSuccess) e = hipStreamWaitEvent(h->cap2, h->evf[0], 0);
                if (e == hipSuccess)
                    e = launch_neumann_update(s, h->ellN, Ni, h->N_neu, h->wself, h->fint, a, b, h->nb, true);
                if (e == hipSuccess)
                    e = launch_sweep_f64(h->cap2, h->cfg, h->ell, Ni, h->fint, a, b, dt, slot, par, 0, h->far_slices);
                if (e == hipSuccess) e = hipEventRecord(h->evf[1], h->cap2);
                if (e == hipSuccess) e = hipStreamWaitEvent(s, h->evf[1], 0);
                if (e == hipSuccess)
                    e = launch_sweep_f64(s, h->cfg, h->ell, Ni, h->fint, a, b, dt, slot, par, h->far_slices, -1);
            } else {
                // Neumann rows first take their values from the current iterate
                if (h->N_neu > 0)
                    e = launch_neumann_update(s, h->ellN, Ni, h->N_neu, h->wself, h->fint, a, b, h->nb,
                                              h->neu_direct);
                if (e == hipSuccess) e = launch_sweep_f64(s, h->cfg, h->ell, Ni, h->fint, a, b, dt, slot, par);
            }
            std::swap(a, b);
        }
    } else if (kind == kGraphMixed) {
        // one outer pass: r = f - L64 u (its max into slot 0), `inner` FP32
        // sweeps on e from 0, u += e, error against the reference into slot 1
        e = launch_fill_u64(s, 2, 0ull, h->dslots);
        if (e == hipSuccess) e = launch_outer_residual(s, h->cfg, h->ell, Ni, h->fint, h->ua, h->r32, h->ea, h->dslots);
        float *a = h->ea, *b = h->eb;
        const float dt32 = (float)dt;
        for (int i = 0; i < inner && e == hipSuccess; ++i) {
            e = (h->cfg32.quad ? launch_sweep_f32q : launch_sweep_f32)(s, h->cfg32, h->ell, Ni, h->r32, a, b, dt32,
                                                                       i & 1);
            std::swap(a, b);
        }
        if (e == hipSuccess) e = launch_add_correction(s, Ni, h->ua, a);
        if (e == hipSuccess && steps)  // steps != 0: the reference is set
            e = launch_err_norm(s, h->N, h->ua, h->uref, h->part, kErrBlocks, h->dslots + 1);
    } else if (kind == kGraphAdjoint) {
        // `steps` transposed steps by scattering: tmp += L^T lam (FP64
        // atomics), lam += dt tmp, acc += lam, tmp = 0.  ua = lam, ub = acc.
        for (int64_t i = 0; i < steps && e == hipSuccess; ++i) {
            e = launch_transpose_scatter(s, h->ell, Ni, h->ua, h->tmp);
            if (e == hipSuccess) e = launch_adjoint_update(s, Ni, dt, h->ua, h->ub, h->tmp);
        }
    } else if (kind == kGraphAdjointHorner) {
        // `steps` transposed steps in Horner form, T <- T + dt (L_II^T T + gK):
        // the forward sweep on the transposed operator with tmp = -gK as its
        // source; T alternates between ua and ub (from `start`).
        double *a = start ? h->ub : h->ua, *b = start ? h->ua : h->ub;
        for (int64_t i = 0; i < steps && e == hipSuccess; ++i) {
            e = launch_sweep_f64(s, h->cfgT, h->ellT, Ni, h->tmp, a, b, dt, nullptr, (int)(i & 1));
            std::swap(a, b);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return fail(h, RBF_EHIP, "graph capture: %s", hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(h, RBF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, RBF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (h->graphs.size() > 64) drop_graphs(h);
    h->graphs[key] = exec;
    *out = exec;
    return RBF_OK;
}

// ====================================================================== iterate
extern "C" rbf_status rbf_iterate(rbf_handle *h, const double *f_dev, double *u_dev, const rbf_iter_params *p,
                                  rbf_iter_report *rep) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!p || !rep || !f_dev || !u_dev) return fail(h, RBF_EINVAL, "null pointer");
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator: compute or set weights first");
    if (!std::isfinite(p->dt)) return fail(h, RBF_EINVAL, "dt must be finite");
    if (p->max_steps < 0 || p->chunk < 1) return fail(h, RBF_EINVAL, "max_steps >= 0 and chunk >= 1 required");
    if (p->mode != RBF_MODE_FP64 && p->mode != RBF_MODE_MIXED) return fail(h, RBF_EINVAL, "unknown mode %d", p->mode);
    if (p->mode == RBF_MODE_MIXED && (p->inner_steps < 1 || !h->have_w32))
        return fail(h, RBF_EINVAL, "mixed mode needs inner_steps >= 1 and FP32 weights (keep_fp32)");
    if (p->mode == RBF_MODE_MIXED && h->N_neu > 0)
        return fail(h, RBF_EINVAL, "mixed precision is implemented for Dirichlet problems only");
    if (p->stall_chunks < 0) return fail(h, RBF_EINVAL, "stall_chunks must be >= 0");
    DeviceGuard g(h->device);
    std::memset(rep, 0, sizeof *rep);
    rep->diverged_step = -1;
    const int64_t N = h->N, Ni = h->N_int;
    const bool use_ref = p->u_ref_dev != nullptr;
    const bool err_stop = use_ref && p->err_target > 0.0;
    const bool mixed = p->mode == RBF_MODE_MIXED;

    HIPCHK(h, launch_gather(h->stream, N, h->perm, u_dev, h->ua));
    HIPCHK(h, hipMemcpyAsync(h->ub, h->ua, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, launch_gather(h->stream, N, h->perm, f_dev, h->fint));
    if (use_ref) HIPCHK(h, launch_gather(h->stream, N, h->perm, p->u_ref_dev, h->uref));
    // max |f| over interior rows (tmp = 0 as the reference), read back with
    // the first chunk's report
    HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->tmp));
    HIPCHK(h, launch_fill_u64(h->stream, 2, 0ull, h->dslots));
    if (Ni) HIPCHK(h, launch_err_norm(h->stream, Ni, h->fint, h->tmp, h->part, kErrBlocks, h->dslots + 1));
    HIPCHK(h, hipMemcpyAsync(h->hslots + 6, h->dslots + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));

    auto finish_errors = [&](double *cur) -> rbf_status {
        if (!use_ref) return RBF_OK;
        HIPCHK(h, launch_fill_u64(h->stream, 2, 0ull, h->dslots));
        HIPCHK(h, launch_err_norm(h->stream, N, cur, h->uref, h->part, kErrBlocks, h->dslots + 1));
        HIPCHK(h, launch_sum_partials(h->stream, h->part, kErrBlocks, (double *)(h->dslots + 2)));
        HIPCHK(h, hipMemcpyAsync(h->hslots, h->dslots, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        rep->err_inf = bits_to_double(h->hslots[1]);
        rep->err_mean_abs = bits_to_double(h->hslots[2]) / (double)N;
        return RBF_OK;
    };
    // a non-finite residual of u0 is divergence at step 0: u_dev keeps u0
    auto diverged_at_start = [&](double res0) -> rbf_status {
        rep->diverged = 1;
        rep->diverged_step = 0;
        rep->steps = 0;
        rep->res0 = rep->res_last = rep->res_final = res0;
        HIPCHK(h, launch_gather(h->stream, N, h->perm, u_dev, h->ua));
        rbf_status st = finish_errors(h->ua);
        if (st) return st;
        return fail(h, RBF_EDIVERGED, "non-finite initial residual (diverged at step 0)");
    };

    // The residual of u0 is the max |rho| of the first sweep (FP64 mode, no
    // Neumann rows: the first chunk's graph reports it) or the first outer
    // residual (mixed mode); otherwise, and when no step runs, it is
    // evaluated here.
    const bool fused_res0 = p->max_steps > 0 && (mixed || h->N_neu == 0);
    double res0 = NAN;
    if (!fused_res0) {
        rbf_status st = residual_internal(h, h->ua, &res0);  // synchronises: fnorm is in hslots[6]
        if (st) return st;
        rep->res0 = res0;
        rep->res_last = res0;
        rep->fnorm = bits_to_double(h->hslots[6]);
        if (!std::isfinite(res0)) return diverged_at_start(res0);
    }

    const bool tol_stop = p->tol_rel > 0.0;
    double best = INFINITY;
    int64_t since_best = 0;
    int64_t steps = 0;
    int cur = 0;  // 0: iterate in ua, 1: in ub
    double dev_ms = 0.0, sweep_ms = 0.0;
    int64_t sweeps_timed = 0;
    rbf_status status = (tol_stop || err_stop) ? RBF_ENOTCONVERGED : RBF_OK;
    bool first = true;

    while (steps < p->max_steps) {
        // FP64: a chunk of sweeps; mixed: one outer pass (u stays in ua), the
        // last one shortened so that max_steps is not exceeded
        const int64_t s = mixed ? std::min<int64_t>(p->inner_steps, p->max_steps - steps)
                                : std::min<int64_t>(p->chunk, p->max_steps - steps);
        hipGraphExec_t ex;
        rbf_status st = mixed ? get_graph(h, kGraphMixed, use_ref ? 1 : 0, 0, p->dt, (int)s, &ex)
                              : get_graph(h, kGraphF64, s, cur, p->dt, (first && fused_res0) ? 1 : 0, &ex);
        if (st) return st;
        HIPCHK(h, hipEventRecord(h->ev0, h->stream));
        HIPCHK(h, hipGraphLaunch(ex, h->stream));
        HIPCHK(h, hipEventRecord(h->ev1, h->stream));
        if (!mixed && (s & 1)) cur ^= 1;
        int nslot = mixed ? 2 : 1;
        if (!mixed && err_stop) {
            double *u_now = cur ? h->ub : h->ua;
            HIPCHK(h, launch_fill_u64(h->stream, 1, 0ull, h->dslots + 1));
            HIPCHK(h, launch_err_norm(h->stream, N, u_now, h->uref, h->part, kErrBlocks, h->dslots + 1));
            nslot = 2;
        }
        HIPCHK(h, hipMemcpyAsync(h->hslots, h->dslots, nslot * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
        if (first && fused_res0 && !mixed)
            HIPCHK(h, hipMemcpyAsync(h->hslots + 5, h->dslots + 5, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                     h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
        dev_ms += ms;
        const double res = bits_to_double(h->hslots[0]);  // residual of the iterate entering the last step
        if (first && fused_res0) {
            // a chunk of one step (and every mixed pass) reports the residual
            // of its starting iterate in slot 0
            res0 = (mixed || s == 1) ? res : bits_to_double(h->hslots[5]);
            rep->res0 = res0;
            rep->fnorm = bits_to_double(h->hslots[6]);
            if (!std::isfinite(res0)) return diverged_at_start(res0);
        }
        first = false;
        if (!mixed) {
            sweep_ms += ms;
            sweeps_timed += s;
        }
        steps += s;
        rep->checks++;
        rep->res_last = res;
        if (!std::isfinite(res) || res > 1e6 * res0) {
            rep->diverged = 1;
            rep->diverged_step = steps;
            status = RBF_EDIVERGED;
            break;
        }
        if (err_stop && bits_to_double(h->hslots[1]) <= p->err_target) {
            rep->err_met = 1;
            rep->converged = 1;
            status = RBF_OK;
            break;
        }
        if (tol_stop && res <= p->tol_rel * rep->fnorm) {
            rep->converged = 1;
            status = RBF_OK;
            break;
        }
        if (res < best) {
            best = res;
            since_best = 0;
        } else if (p->stall_chunks > 0 && ++since_best >= p->stall_chunks) {
            break;
        }
    }
    if (!mixed) {
        h->last_sweep_sec = sweeps_timed ? sweep_ms * 1e-3 / (double)sweeps_timed : 0.0;
        h->last_sweeps = sweeps_timed;
    }
    double *u_fin = cur ? h->ub : h->ua;
    rep->steps = steps;
    rep->seconds = dev_ms * 1e-3;
    HIPCHK(h, launch_scatter(h->stream, N, h->perm, u_fin, u_dev));
    double resf = 0.0;
    rbf_status st = residual_internal(h, u_fin, &resf);
    if (st) return st;
    rep->res_final = resf;
    st = finish_errors(u_fin);
    if (st) return st;
    const double tol_abs = p->tol_rel * rep->fnorm;
    if (status == RBF_EDIVERGED)
        return fail(h, status, "diverged: residual %g at step %" PRId64 " (initial %g)", rep->res_last, rep->diverged_step, res0);
    if (status == RBF_ENOTCONVERGED)
        return fail(h, status, "not converged after %" PRId64 " steps (residual %g, target %g)", steps, rep->res_last, tol_abs);
    return RBF_OK;
}

// Bytes one sweep streams through the packed operator as stored (see the
// header), for FP64 (wbytes 8, vbytes 8) or FP32 (4, 4) with or without codes.
static double stream_bytes(const rbf_handle *h, int wbytes, int vbytes, bool codes, bool quad) {
    const Ell &e = h->ell;
    if (!e.nslices) return 0.0;
    std::vector<int32_t> slen((size_t)e.nslices);
    std::vector<int8_t> cm;
    if (hipMemcpy(slen.data(), e.slice_len, sizeof(int32_t) * e.nslices, hipMemcpyDeviceToHost) != hipSuccess)
        return 0.0;
    if (codes) {
        cm.resize((size_t)e.nslices);
        if (hipMemcpy(cm.data(), e.cmode, (size_t)e.nslices, hipMemcpyDeviceToHost) != hipSuccess) return 0.0;
    }
    double b = 0.0;
    for (int64_t s = 0; s < e.nslices; ++s) {
        const double len = slen[s], len4 = (slen[s] + 3) & ~3;
        b += 12.0 + kSlice * ((quad && cm[s]) ? len4 : len) * wbytes;       // header, weights
        if (codes && cm[s]) b += 1.0 + 4.0 * kSegs + 8.0 + kSlice * len4 * 2.0;  // mode, segments, offset, codes
        else b += kSlice * len * 4.0;                                       // ids
    }
    return b + 3.0 * vbytes * (double)h->N_int;
}

extern "C" rbf_status rbf_get_operator_info(const rbf_handle *h, rbf_operator_info *info) {
    if (!h || !info) return RBF_EINVAL;
    if (!h->have_w || !h->ua) return RBF_EINVAL;
    DeviceGuard g(h->device);
    std::memset(info, 0, sizeof *info);
    const Ell &e = h->ell;
    info->n_interior = h->N_int;
    info->n_neumann = h->N_neu;
    info->slices = e.nslices;
    info->slots = e.elems;
    info->coded_slices = e.cmode ? e.coded_slices : 0;
    info->max_len = e.max_len;
    info->layout = e.layout;
    const SweepCfg &a = h->cfg, &b = h->cfg32;
    info->f64_waves = a.waves_per_block;
    info->f64_unroll = a.unroll;
    info->f64_xcd_remap = a.xcd_remap;
    info->f64_pipeline = a.pipeline;
    info->f64_zigzag = a.zigzag;
    info->f64_codes = a.codes && e.cmode ? 1 : 0;
    info->f32_waves = b.waves_per_block;
    info->f32_unroll = b.unroll;
    info->f32_xcd_remap = b.xcd_remap;
    info->f32_pipeline = b.pipeline;
    info->f32_zigzag = b.zigzag;
    info->f32_codes = b.codes && e.cmode ? 1 : 0;
    info->f64_temporal = info->f64_codes && a.temporal;
    info->f32_temporal = info->f32_codes && b.temporal;
    info->f32_quad = info->f32_codes && b.quad && e.w32q ? 1 : 0;
    info->stream_bytes_f64 = stream_bytes(h, 8, 8, info->f64_codes, false);
    info->stream_bytes_f32 = h->have_w32 ? stream_bytes(h, 4, 4, info->f32_codes, info->f32_quad) : 0.0;
    info->code_mismatches = (int32_t)e.code_mismatches;
    const Ell &t = h->ellT;
    if (t.idx) {
        info->t_slices = t.nslices;
        info->t_slots = t.elems;
        info->t_coded_slices = t.cmode ? t.coded_slices : 0;
        info->t_code_mismatches = t.code_mismatches;
        info->t_max_len = t.max_len;
        info->t_waves = h->cfgT.waves_per_block;
        info->t_unroll = h->cfgT.unroll;
        info->t_codes = h->cfgT.codes && t.cmode ? 1 : 0;
        info->t_lane_order = t.lmeta ? 1 : 0;
        info->t_masked = info->t_codes && t.lmeta && h->cfgT.temporal && h->cfgT.pipeline ? 1 : 0;
    }
    info->ns_systems = h->w_ns_systems;
    info->elim_systems = h->w_elim_systems;
    return RBF_OK;
}

extern "C" rbf_status rbf_last_sweep_time(const rbf_handle *h, double *seconds_per_sweep, int64_t *sweeps) {
    if (!h) return RBF_EINVAL;
    if (seconds_per_sweep) *seconds_per_sweep = h->last_sweep_sec;
    if (sweeps) *sweeps = h->last_sweeps;
    return RBF_OK;
}

// ====================================================================== adjoint
extern "C" rbf_status rbf_forward_ckpt(rbf_handle *h, const double *f_dev, const double *u0_dev, int64_t K,
                                       int64_t every, double *ckpt_dev, double *uK_dev, double dt) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!f_dev || !u0_dev || !uK_dev) return fail(h, RBF_EINVAL, "null pointer");
    if (K < 1 || every < 1 || every > K || K % every) return fail(h, RBF_EINVAL, "need 1 <= every <= K, K %% every == 0");
    if (!std::isfinite(dt)) return fail(h, RBF_EINVAL, "dt must be finite");
    DeviceGuard g(h->device);
    const int64_t N = h->N;
    HIPCHK(h, launch_gather(h->stream, N, h->perm, u0_dev, h->ua));
    HIPCHK(h, hipMemcpyAsync(h->ub, h->ua, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, launch_gather(h->stream, N, h->perm, f_dev, h->fint));
    if (ckpt_dev) HIPCHK(h, launch_scatter(h->stream, N, h->perm, h->ua, ckpt_dev));
    int cur = 0;
    for (int64_t seg = 1; seg <= K / every; ++seg) {
        hipGraphExec_t ex;
        rbf_status st = get_graph(h, kGraphF64Quiet, every, cur, dt, 0, &ex);
        if (st) return st;
        HIPCHK(h, hipGraphLaunch(ex, h->stream));
        if (every & 1) cur ^= 1;
        if (ckpt_dev) HIPCHK(h, launch_scatter(h->stream, N, h->perm, cur ? h->ub : h->ua, ckpt_dev + seg * N));
    }
    HIPCHK(h, launch_scatter(h->stream, N, h->perm, cur ? h->ub : h->ua, uK_dev));
    return RBF_OK;
}

// Sweep shape of the transposed gather (its rows are the interior columns of
// L, of uneven length): cached like the forward shapes under "sweepT|...",
// else timed over the same candidates on the handle's work vectors.
static rbf_status tune_transpose(rbf_handle *h) {
    const Ell &e = h->ellT;
    if (!e.nslices || h->tunedT) return RBF_OK;
    char key[160];
    std::snprintf(key, sizeof key, "sweepT|%s|L%d|%" PRId64 "|%" PRId64 "|%d|c%" PRId64, h->arch, e.layout,
                  h->N_int, e.elems, e.max_len, e.coded_slices);
    int v[8];
    SweepCfg forced;
    if (shape_override(&forced)) {
        if (!e.cmode) forced.codes = forced.temporal = 0;
        forced.quad = 0;
        forced.unroll = std::min(forced.unroll, 16);
        h->cfgT = forced;
    } else if (env_flag("RBF_AUTOTUNE_FORCE") != 1 && lookup_shape(key, v)) {
        apply_shape(h->cfgT, v, e);
    } else {
        const int64_t Ni = h->N_int;
        HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->ua));
        HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->ub));
        HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->tmp));
        float best = 1e30f;
        SweepCfg bestc = h->cfgT;
        for (int wv : {2, 4, 8})
            for (int un : {4, 8, 16})
                for (int rm : {0, 1})
                    for (int pl : {0, 1})
                    for (int zz : {0, 1})
                    for (int cd : {0, 1})
                    for (int tp : {0, 1}) {
                        if ((cd && !e.cmode) || (tp && !cd)) continue;
                        SweepCfg c;
                        c.waves_per_block = wv;
                        c.unroll = un;
                        c.xcd_remap = rm;
                        c.pipeline = pl;
                        c.zigzag = zz;
                        c.codes = cd;
                        c.temporal = tp;
                        auto launch = [&](int r) {
                            return launch_sweep_f64(h->stream, c, e, Ni, h->tmp, (r & 1) ? h->ub : h->ua,
                                                    (r & 1) ? h->ua : h->ub, 0.0, nullptr, r & 1);
                        };
                        HIPCHK(h, launch(0));
                        HIPCHK(h, hipEventRecord(h->ev0, h->stream));
                        for (int r = 0; r < 20; ++r) HIPCHK(h, launch(r));
                        HIPCHK(h, hipEventRecord(h->ev1, h->stream));
                        HIPCHK(h, hipEventSynchronize(h->ev1));
                        float ms = 0.f;
                        HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
                        if (ms < best) {
                            best = ms;
                            bestc = c;
                        }
                    }
        h->cfgT = bestc;
        int vv[8] = {bestc.waves_per_block, bestc.unroll, bestc.xcd_remap, bestc.pipeline, bestc.zigzag, bestc.codes,
                     bestc.temporal, 0};
        cache_store(key, vv, 8);
    }
    h->tunedT = true;
    return RBF_OK;
}

extern "C" rbf_status rbf_adjoint_f(rbf_handle *h, const double *gK_dev, int64_t K, int64_t every,
                                    const double *ckpt_dev, double *grad_f_dev, double dt) {
    (void)ckpt_dev;  // the gradient with respect to f does not depend on the states
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua) return fail(h, RBF_EINVAL, "no operator");
    if (!gK_dev || !grad_f_dev) return fail(h, RBF_EINVAL, "null pointer");
    if (h->N_neu > 0) return fail(h, RBF_EINVAL, "the adjoint is implemented for Dirichlet problems only");
    if (K < 1 || every < 1 || every > K || K % every) return fail(h, RBF_EINVAL, "need 1 <= every <= K, K %% every == 0");
    if (!std::isfinite(dt)) return fail(h, RBF_EINVAL, "dt must be finite");
    DeviceGuard g(h->device);
    const int64_t N = h->N, Ni = h->N_int;
    const int64_t nseg = K / every;
    if (use_scatter_transpose()) {
        // lam = gK on interior rows (0 elsewhere) in ua, acc = lam in ub, the
        // scatter target tmp = 0; K-1 scattered steps lam <- G^T lam, acc += lam
        HIPCHK(h, launch_gather(h->stream, N, h->perm, gK_dev, h->ua));
        HIPCHK(h, launch_fill_f64(h->stream, N - Ni, 0.0, h->ua + Ni));
        HIPCHK(h, hipMemcpyAsync(h->ub, h->ua, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->tmp));
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t steps = seg == 0 ? every - 1 : every;
            if (steps <= 0) continue;
            hipGraphExec_t ex;
            rbf_status st = get_graph(h, kGraphAdjoint, steps, 0, dt, 0, &ex);
            if (st) return st;
            HIPCHK(h, hipGraphLaunch(ex, h->stream));
        }
        HIPCHK(h, launch_scale_interior(h->stream, N, Ni, -dt, h->ub, h->tmp));
        HIPCHK(h, launch_scatter(h->stream, N, h->perm, h->tmp, grad_f_dev));
        HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->tmp));
        return RBF_OK;
    }
    rbf_status st = build_transpose(h);
    if (!st) st = tune_transpose(h);
    if (st) return st;
    // Horner form of grad = -dt sum_{j<K} (G^T)^j gK: with T_0 = 0 and
    // T_{j+1} = T_j + dt (L_II^T T_j + gK) = dt gK + G^T T_j, T_K = dt times
    // the sum, so grad = -T_K.  Each step is the forward sweep on L_II^T with
    // source -gK (in tmp); T lives in ua / ub, 0 on Dirichlet nodes.
    HIPCHK(h, launch_gather(h->stream, N, h->perm, gK_dev, h->ua));
    HIPCHK(h, launch_scale_interior(h->stream, N, Ni, -1.0, h->ua, h->tmp));
    HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->ua));
    HIPCHK(h, launch_fill_f64(h->stream, N, 0.0, h->ub));
    // K steps in graphs of `every` (one per checkpoint segment, run from the
    // last segment back to the first)
    int cur = 0;
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        hipGraphExec_t ex;
        st = get_graph(h, kGraphAdjointHorner, every, cur, dt, 0, &ex);
        if (st) return st;
        HIPCHK(h, hipGraphLaunch(ex, h->stream));
        if (every & 1) cur ^= 1;
    }
    double *T = cur ? h->ub : h->ua, *out = cur ? h->ua : h->ub;
    HIPCHK(h, launch_scale_interior(h->stream, N, Ni, -1.0, T, out));
    HIPCHK(h, launch_scatter(h->stream, N, h->perm, out, grad_f_dev));
    return RBF_OK;
}

// ====================================================================== autotune
// Time every candidate shape of the FP64 sweep (and of the FP32 sweep when an
// FP32 copy exists) on the real operator and keep the fastest of each.
extern "C" rbf_status rbf_autotune(rbf_handle *h) {
    if (!h) return RBF_EINVAL;
    h->err.clear();
    if (!h->have_w || !h->ua || !h->N_int) return fail(h, RBF_EINVAL, "no operator");
    DeviceGuard g(h->device);
    drop_graphs(h);
    const int64_t Ni = h->N_int;
    HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->ua));
    HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->ub));
    HIPCHK(h, launch_fill_f64(h->stream, h->N, 0.0, h->fint));
    HIPCHK(h, launch_fill_f32(h->stream, h->N, 0.0f, h->r32));
    const int reps = 20;
    SweepCfg forced;
    const int nprec = shape_override(&forced) ? 0 : (h->have_w32 ? 2 : 1);
    const bool force = env_flag("RBF_AUTOTUNE_FORCE") == 1;
    for (int prec = 0; prec < nprec; ++prec) {
        char key[160];
        sweep_key(h, prec, key, sizeof key);
        int cached[8];
        if (!force && lookup_shape(key, cached)) {  // tuned before for this shape
            apply_shape(prec ? h->cfg32 : h->cfg, cached, h->ell);
            continue;
        }
        float best = 1e30f;
        SweepCfg bestc = prec ? h->cfg32 : h->cfg;
        auto launch = [&](const SweepCfg &c, int r) -> hipError_t {
            if (prec)
                return (c.quad ? launch_sweep_f32q : launch_sweep_f32)(h->stream, c, h->ell, Ni, h->r32,
                                                                       (r & 1) ? h->eb : h->ea,
                                                                       (r & 1) ? h->ea : h->eb, 0.0f, r & 1);
            return launch_sweep_f64(h->stream, c, h->ell, Ni, h->fint, (r & 1) ? h->ub : h->ua,
                                    (r & 1) ? h->ua : h->ub, 0.0, nullptr, r & 1);
        };
        for (int wv : {2, 4, 8})
            for (int un : {4, 8, 16, 32})
                for (int rm : {0, 1})
                    for (int pl : {0, 1})
                    for (int zz : {0, 1})
                    for (int cd : {0, 1})
                    for (int tp : {0, 1})
                    for (int qd : {0, 1}) {
                        if (pl && h->ell.layout == 0) continue;
                        if (tp && !cd) continue;
                        if (qd && (!prec || !cd || !h->ell.w32q)) continue;
                        if (un == 32 && !qd) continue;  // only the FP32 code-layout sweep has 32-entry groups
                        if (zigzag_override() >= 0 && zz != zigzag_override()) continue;
                        if (cd && !h->ell.cmode) continue;
                        if (codes_override() >= 0 && cd != codes_override() && h->ell.cmode) continue;
                        SweepCfg c;
                        c.waves_per_block = wv;
                        c.unroll = un;
                        c.xcd_remap = rm;
                        c.pipeline = pl;
                        c.zigzag = zz;
                        c.codes = cd;
                        c.temporal = tp;
                        c.quad = qd;
                        HIPCHK(h, launch(c, 0));
                        HIPCHK(h, hipEventRecord(h->ev0, h->stream));
                        for (int r = 0; r < reps; ++r) HIPCHK(h, launch(c, r));
                        HIPCHK(h, hipEventRecord(h->ev1, h->stream));
                        HIPCHK(h, hipEventSynchronize(h->ev1));
                        float ms = 0.f;
                        HIPCHK(h, hipEventElapsedTime(&ms, h->ev0, h->ev1));
                        if (ms < best) {
                            best = ms;
                            bestc = c;
                        }
                    }
        (prec ? h->cfg32 : h->cfg) = bestc;
        int v[8] = {bestc.waves_per_block, bestc.unroll, bestc.xcd_remap, bestc.pipeline, bestc.zigzag, bestc.codes,
                    bestc.temporal, bestc.quad};
        cache_store(key, v, 8);
    }
    // leave the FP32 work vectors as the mixed loop expects them (0 beyond N_int)
    HIPCHK(h, launch_fill_f32(h->stream, h->N, 0.0f, h->ea));
    HIPCHK(h, launch_fill_f32(h->stream, h->N, 0.0f, h->eb));
    return RBF_OK;
}

}  // extern "C"
