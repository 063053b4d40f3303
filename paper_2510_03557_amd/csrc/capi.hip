// C ABI of the short-range step: argument validation, contexts, trees,
// device-error latching, graph capture and event timing.  The arithmetic
// lives in tree.hip, lists.hip, passes.hip and integrate.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "crk_internal.h"

// Scratch of crk_density_noalloc: the masses of the gas particles in tree
// order (up to CRK_NOALLOC_MAX_GAS values of the context precision), as a
// file-scope device array so that the entry point allocates nothing.  Each
// GPU holds its own copy until the process ends.  In host code the name is
// only a stand-in for the symbol, not a device address: its address on a
// device comes from hipGetSymbolAddress, once per device (at the first
// crk_ctx_create on it), and only that address is ever passed to kernels.
static __device__ __align__(256) unsigned char
    scratch[(size_t)CRK_NOALLOC_MAX_GAS * sizeof(double)];

namespace crk {

namespace {
thread_local std::string g_last_error;

bool aligned(const void *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}
}  // namespace

int set_error(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

namespace {
std::atomic<uint64_t> g_alloc_gen{1};

// per-device address of the scratch array (null until looked up; a failed
// lookup is remembered with its message)
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
std::string g_scratch_err[MAX_DEVICES];
bool g_scratch_done[MAX_DEVICES] = {};

// Looks the scratch array up on the current device (which must be dev).
void *scratch_address(int dev, std::string *err) {
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p) {
            g_scratch_ptr[dev] = p;
        } else {
            g_scratch_ptr[dev] = nullptr;
            g_scratch_err[dev] = std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e);
        }
        g_scratch_done[dev] = true;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}
}  // namespace

uint64_t alloc_generation() { return g_alloc_gen.load(std::memory_order_acquire); }
void alloc_generation_bump() { g_alloc_gen.fetch_add(1, std::memory_order_acq_rel); }

int DevBuf::ensure(size_t n, bool capturing) {
    if (n <= bytes && p) return CRK_OK;
    if (capturing)
        return set_error(CRK_ECAPACITY,
                         "a buffer would have to grow during graph capture; "
                         "run the step once eagerly at this size first");
    if (p) {
        alloc_generation_bump();
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    size_t want = (n + 255) & ~size_t(255);
    if (want == 0) want = 256;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return set_error(CRK_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    bytes = want;
    return CRK_OK;
}

void DevBuf::release() {
    if (p) {
        alloc_generation_bump();
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
}

int HostBuf::ensure(size_t n) {
    if (n <= bytes && p) return CRK_OK;
    if (p) {
        alloc_generation_bump();
        (void)hipHostFree(p);
    }
    p = nullptr;
    bytes = 0;
    size_t want = std::max<size_t>((n + 255) & ~size_t(255), 256);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        return set_error(CRK_EDEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    bytes = want;
    return CRK_OK;
}

void HostBuf::release() {
    if (p) {
        alloc_generation_bump();
        (void)hipHostFree(p);
    }
    p = nullptr;
    bytes = 0;
}

void span_begin(crk_ctx *ctx, int pass, bool kernel, hipEvent_t *ev) {
    *ev = nullptr;
    if (!ctx->timing || ctx->capturing) return;
    if (hipEventCreate(ev) != hipSuccess) {
        *ev = nullptr;
        return;
    }
    (void)hipEventRecord(*ev, ctx->stream);
    (void)pass;
    (void)kernel;
}

void span_end(crk_ctx *ctx, int pass, bool kernel, hipEvent_t ev) {
    if (!ev) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return;
    }
    (void)hipEventRecord(b, ctx->stream);
    ctx->spans.push_back(TimedSpan{pass, kernel, ev, b});
}

}  // namespace crk

using namespace crk;

namespace crk {
// halo.hip
int fof_properties(crk_ctx *ctx, int64_t n_gas, int64_t n_dm,
                   const int32_t *labels_gas, const int32_t *labels_dm,
                   const void *const g[3], const void *m_gas,
                   const void *const d[3], const void *m_dm, int32_t *count,
                   double *mass, double *centre);
}  // namespace crk

namespace {

int check_ctx(const crk_ctx *ctx) {
    if (!ctx) return set_error(CRK_EINVAL, "null context");
    return CRK_OK;
}

int check_ptr(const void *p, size_t align, const char *name, bool required) {
    if (!p) {
        if (required) return set_error(CRK_EINVAL, std::string("null pointer: ") + name);
        return CRK_OK;
    }
    if (!aligned(p, align))
        return set_error(CRK_EINVAL, std::string("misaligned pointer: ") + name);
    return CRK_OK;
}

int check_tree_ready(const crk_ctx *ctx, const crk_tree *t, bool need_lists) {
    CRK_TRY(check_ctx(ctx));
    if (!t) return set_error(CRK_EINVAL, "null tree");
    if (t->owner != ctx) return set_error(CRK_ESTATE, "tree belongs to another context");
    if (t->leaf_cap == 0) return set_error(CRK_ESTATE, "tree not built");
    if (need_lists && !t->lists_built)
        return set_error(CRK_ESTATE, "interaction lists not built for this tree");
    return CRK_OK;
}

struct PassSpan {
    crk_ctx *ctx;
    int pass;
    hipEvent_t ev;
    PassSpan(crk_ctx *c, int p) : ctx(c), pass(p), ev(nullptr) {
        span_begin(ctx, pass, false, &ev);
    }
    ~PassSpan() { span_end(ctx, pass, false, ev); }
};

}  // namespace

extern "C" {

const char *crk_last_error(void) { return g_last_error.c_str(); }

int crk_ctx_create(crk_ctx **out, int precision, void *stream,
                   const crk_params *params) {
    if (!out) return set_error(CRK_EINVAL, "null output pointer");
    *out = nullptr;
    if (precision != CRK_FP32 && precision != CRK_FP64)
        return set_error(CRK_EINVAL, "precision must be CRK_FP32 or CRK_FP64");
    crk_params p = {5.0 / 3.0, 1.0, 2.0, 0.01, 1.0};
    if (params) {
        p = *params;
        if (!(p.gamma > 1.0) || !(p.Cl >= 0.0) || !(p.Cq >= 0.0) ||
            !(p.epsQ > 0.0) || !std::isfinite(p.G))
            return set_error(CRK_EINVAL, "invalid physical parameters");
    }
    crk_ctx *c = new (std::nothrow) crk_ctx();
    if (!c) return set_error(CRK_EDEVICE, "out of host memory");
    c->precision = precision;
    c->stream = static_cast<hipStream_t>(stream);
    c->params = p;
    c->tuning.leaf_max = 64;
    c->tuning.cm_factor = 0.0;
    c->tuning.grid_mult = 0;
    c->tuning.xcd_remap = 1;
    c->tuning.walk_mask = 0;
    c->tuning.sub_sweep = 2;
    c->tuning.tree_lds = 1;
    c->tuning.tile = 0;
    c->tuning.act_groups = 1;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount,
                                  c->device);
    if (e != hipSuccess) {
        delete c;
        return set_error(CRK_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
    }
    // the allocation-free entry point's scratch on this (current) device
    c->noalloc_scratch = scratch_address(c->device, &c->noalloc_error);
    int s = c->err.ensure(64, false);
    if (s == CRK_OK) s = c->err_host.ensure(4096);
    if (s != CRK_OK) {
        delete c;
        return s;
    }
    e = hipMemset(c->err.p, 0, 64);
    if (e != hipSuccess) {
        c->err.release();
        c->err_host.release();
        delete c;
        return set_error(CRK_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    *out = c;
    return CRK_OK;
}

int crk_ctx_destroy(crk_ctx *ctx) {
    if (!ctx) return CRK_OK;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (auto &s : ctx->spans) {
        (void)hipEventDestroy(s.a);
        (void)hipEventDestroy(s.b);
    }
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    pm_release(ctx->pm);
    ctx->err.release();
    ctx->err_host.release();
    ctx->scratch.release();
    delete ctx;
    return CRK_OK;
}

int crk_set_tuning(crk_ctx *ctx, const crk_tuning *t) {
    CRK_TRY(check_ctx(ctx));
    if (!t) return set_error(CRK_EINVAL, "null tuning");
    if (t->leaf_max < 16 || t->leaf_max > 256)
        return set_error(CRK_EINVAL, "leaf_max must be in [16, 256]");
    if (!(t->cm_factor == 0.0 || (t->cm_factor >= 1.0 && t->cm_factor <= 64.0)))
        return set_error(CRK_EINVAL, "cm_factor must be 0 (auto) or in [1, 64]");
    if (t->grid_mult < 0 || t->grid_mult > 64)
        return set_error(CRK_EINVAL, "grid_mult must be in [0, 64]");
    if (t->xcd_remap != 0 && t->xcd_remap != 1)
        return set_error(CRK_EINVAL, "xcd_remap must be 0 or 1");
    if (t->walk_mask < 0 || t->walk_mask > 31)
        return set_error(CRK_EINVAL, "walk_mask must be in [0, 31]");
    if (t->sub_sweep < 0 || t->sub_sweep > 3)
        return set_error(CRK_EINVAL, "sub_sweep must be 0, 1, 2 or 3");
    if (t->tree_lds != 0 && t->tree_lds != 1)
        return set_error(CRK_EINVAL, "tree_lds must be 0 or 1");
    if (!(t->tile == 0 || t->tile == 1 || t->tile == 2 || t->tile == 4 ||
          t->tile == 8))
        return set_error(CRK_EINVAL, "tile must be 0, 1, 2, 4 or 8");
    if (t->act_groups < 0 || t->act_groups > 4096)
        return set_error(CRK_EINVAL, "act_groups must be in [0, 4096]");
    if (ctx->capturing) return set_error(CRK_ESTATE, "tuning change during capture");
    ctx->tuning = *t;
    return CRK_OK;
}

int crk_get_tuning(const crk_ctx *ctx, crk_tuning *t) {
    CRK_TRY(check_ctx(ctx));
    if (!t) return set_error(CRK_EINVAL, "null tuning");
    *t = ctx->tuning;
    return CRK_OK;
}

int crk_sync(crk_ctx *ctx, int64_t *required) {
    CRK_TRY(check_ctx(ctx));
    if (ctx->capturing) return set_error(CRK_ESTATE, "crk_sync during graph capture");
    int32_t *hb = ctx->err_host.as<int32_t>();
    CRK_HIP(hipMemcpyAsync(hb, ctx->err.p, 16, hipMemcpyDeviceToHost, ctx->stream));
    CRK_HIP(hipStreamSynchronize(ctx->stream));
    int word = hb[0];
    if (required) *required = 0;
    if (word) {
        CRK_HIP(fill_i32(ctx->err.as<int32_t>(), 0, 4, ctx->stream));
        CRK_HIP(hipStreamSynchronize(ctx->stream));
        if (word & DEV_ERR_INPUT)
            return set_error(CRK_EINVAL,
                             "device check: a position outside [1,2), a "
                             "non-finite value, a non-positive h or a group "
                             "label outside the particle range");
        if (word & DEV_ERR_HMAX)
            return set_error(CRK_EINVAL,
                             "device check: a smoothing length above the "
                             "declared per-box h_max");
        if (word & DEV_ERR_CAPACITY)
            return set_error(CRK_ECAPACITY,
                             "a capacity fixed at graph capture was exceeded; "
                             "rebuild eagerly and capture again");
    }
    return CRK_OK;
}

int build_tree(crk_ctx *ctx, const crk_boxes *boxes, const void *gx,
               const void *gy, const void *gz, const void *gh, const void *dx,
               const void *dy, const void *dz, crk_tree **tree) {
    CRK_TRY(check_ctx(ctx));
    if (!boxes || !tree) return set_error(CRK_EINVAL, "null boxes or tree pointer");
    const int nb = boxes->n_boxes;
    if (nb < 1) return set_error(CRK_EINVAL, "n_boxes must be >= 1");
    if (!boxes->gas_off || !boxes->dm_off || !boxes->r_c || !boxes->eps ||
        !boxes->h_max)
        return set_error(CRK_EINVAL, "null array in crk_boxes");
    if (boxes->gas_off[0] != 0 || boxes->dm_off[0] != 0)
        return set_error(CRK_EINVAL, "box offsets must start at 0");
    for (int b = 0; b < nb; ++b) {
        if (boxes->gas_off[b + 1] < boxes->gas_off[b] ||
            boxes->dm_off[b + 1] < boxes->dm_off[b])
            return set_error(CRK_EINVAL, "box offsets must be non-decreasing");
        const double rc = boxes->r_c[b], eps = boxes->eps[b], hm = boxes->h_max[b];
        if (!(rc > 0.0) || !(rc < 0.5))
            return set_error(CRK_EINVAL, "r_c must satisfy 0 < r_c < 0.5");
        if (!(eps >= 0.0) || !(eps < rc))
            return set_error(CRK_EINVAL, "eps must satisfy 0 <= eps < r_c");
        if (!(hm > 0.0) || !(2.0 * hm < 0.5))
            return set_error(CRK_EINVAL, "h_max must satisfy 0 < 2 h_max < 0.5");
    }
    const int64_t ng = boxes->gas_off[nb], nd = boxes->dm_off[nb];
    const size_t el = ctx->elem();
    CRK_TRY(check_ptr(gx, el, "gx", ng > 0));
    CRK_TRY(check_ptr(gy, el, "gy", ng > 0));
    CRK_TRY(check_ptr(gz, el, "gz", ng > 0));
    CRK_TRY(check_ptr(gh, el, "gh", ng > 0));
    CRK_TRY(check_ptr(dx, el, "dx", nd > 0));
    CRK_TRY(check_ptr(dy, el, "dy", nd > 0));
    CRK_TRY(check_ptr(dz, el, "dz", nd > 0));
    if (ng + nd == 0) return set_error(CRK_EINVAL, "no particles");
    crk_tree *t = *tree;
    if (!t) {
        if (ctx->capturing) return set_error(CRK_ESTATE, "tree creation during capture");
        t = new (std::nothrow) crk_tree();
        if (!t) return set_error(CRK_EDEVICE, "out of host memory");
        t->owner = ctx;
        *tree = t;
    } else if (t->owner != ctx) {
        return set_error(CRK_ESTATE, "tree belongs to another context");
    }
    PassSpan sp(ctx, P_TREE);
    t->act_on = false;  // a new tree starts with every leaf active
    t->grp_on = false;
    t->slist_on = false;
    return tree_build(ctx, t, boxes, gx, gy, gz, gh, dx, dy, dz);
}

int build_interaction_lists(crk_ctx *ctx, crk_tree *t) {
    CRK_TRY(check_tree_ready(ctx, t, false));
    PassSpan sp(ctx, P_LISTS);
    return lists_build(ctx, t);
}

int crk_density(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                void *rho_tilde) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    CRK_TRY(check_ptr(m, el, "m", g));
    CRK_TRY(check_ptr(V, el, "V", g));
    CRK_TRY(check_ptr(rho_tilde, el, "rho_tilde", g));
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_DENSITY);
    return pass_density(ctx, t, m, V, rho_tilde);
}

int crk_density_noalloc(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                        void *rho_tilde) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    CRK_TRY(check_ptr(m, el, "m", g));
    CRK_TRY(check_ptr(V, el, "V", g));
    CRK_TRY(check_ptr(rho_tilde, el, "rho_tilde", g));
    if (t->n_gas > (int64_t)CRK_NOALLOC_MAX_GAS)
        return set_error(CRK_EINVAL,
                         "crk_density_noalloc: " + std::to_string(t->n_gas) +
                             " gas particles exceed its scratch of " +
                             std::to_string((int64_t)CRK_NOALLOC_MAX_GAS) +
                             "; use crk_density");
    if (!ctx->noalloc_scratch)
        return set_error(CRK_EDEVICE, "crk_density_noalloc: no scratch on this "
                                      "device (" + ctx->noalloc_error + ")");
    if (!g) return CRK_OK;
    return pass_density_scratch(ctx, t, m, V, rho_tilde, ctx->noalloc_scratch);
}

int crk_coefficients(crk_ctx *ctx, crk_tree *t, const void *m, const void *V,
                     const void *u, void *A, void *B, void *gradA, void *gradB,
                     void *rho, void *P, void *cs) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    const void *ins[] = {m, V, u};
    const char *in_names[] = {"m", "V", "u"};
    for (int k = 0; k < 3; ++k) CRK_TRY(check_ptr(ins[k], el, in_names[k], g));
    void *outs[] = {A, B, gradA, gradB, rho, P, cs};
    const char *out_names[] = {"A", "B", "gradA", "gradB", "rho", "P", "cs"};
    for (int k = 0; k < 7; ++k) CRK_TRY(check_ptr(outs[k], el, out_names[k], g));
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_COEFF);
    return pass_coefficients(ctx, t, m, V, u, A, B, gradA, gradB, rho, P, cs);
}

int crk_hydro_forces(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
                     const void *vy, const void *vz, const void *V,
                     const void *rho, const void *P, const void *cs,
                     const void *A, const void *B, const void *gradA,
                     const void *gradB, void *ax, void *ay, void *az,
                     void *dudt) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    const void *ins[] = {m, vx, vy, vz, V, rho, P, cs, A, B, gradA, gradB};
    const char *in_names[] = {"m", "vx", "vy", "vz", "V", "rho", "P", "cs",
                              "A", "B", "gradA", "gradB"};
    for (int k = 0; k < 12; ++k) CRK_TRY(check_ptr(ins[k], el, in_names[k], g));
    void *outs[] = {ax, ay, az, dudt};
    const char *out_names[] = {"ax", "ay", "az", "dudt"};
    for (int k = 0; k < 4; ++k) CRK_TRY(check_ptr(outs[k], el, out_names[k], g));
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_HYDRO);
    return pass_hydro(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA, gradB,
                      nullptr, 0.0, 1.0, ax, ay, az, dudt);
}

namespace {

// the checks and the launch of both compatible-energy entry points; bins
// (caller order) selects per-particle kick widths, nullptr the width dt
int energy_compatible(crk_ctx *ctx, crk_tree *t, const void *m,
                      const void *vx, const void *vy, const void *vz,
                      const void *V, const void *rho, const void *P,
                      const void *cs, const void *A, const void *B,
                      const void *gradA, const void *gradB, const void *dv,
                      double eta_crit, double eta_fold, double dt,
                      const int32_t *bins, int max_level, int64_t substep,
                      const void *const a_grav[3],
                      const void *const a_hydro[3], void *dudt) {
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    const void *ins[] = {m, vx, vy, vz, V, rho, P, cs, A, B, gradA, gradB};
    const char *in_names[] = {"m", "vx", "vy", "vz", "V", "rho", "P", "cs",
                              "A", "B", "gradA", "gradB"};
    for (int k = 0; k < 12; ++k) CRK_TRY(check_ptr(ins[k], el, in_names[k], g));
    CRK_TRY(check_ptr(dudt, el, "dudt", g));
    if (!std::isfinite(dt)) return set_error(CRK_EINVAL, "dt must be finite");
    if (g && !a_grav) return set_error(CRK_EINVAL, "null pointer array a_grav");
    for (int a = 0; a < 3 && g; ++a) {
        CRK_TRY(check_ptr(a_grav[a], el, "a_grav", true));
        if (a_hydro) CRK_TRY(check_ptr(a_hydro[a], el, "a_hydro", true));
    }
    if (dv) {
        CRK_TRY(check_ptr(dv, el, "dv", g));
        if (!(eta_crit >= 0.0) || !std::isfinite(eta_crit) ||
            !(eta_fold > 0.0) || !std::isfinite(eta_fold))
            return set_error(CRK_EINVAL,
                             "eta_crit must be finite and >= 0, eta_fold finite and > 0");
    }
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_ENERGY);
    return pass_energy_compatible(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B,
                                  gradA, gradB, dv, eta_crit, eta_fold, dt,
                                  bins, max_level, substep, a_grav, a_hydro,
                                  dudt);
}

}  // namespace

int crk_hydro_energy_compatible(crk_ctx *ctx, crk_tree *t, const void *m,
                                const void *vx, const void *vy, const void *vz,
                                const void *V, const void *rho, const void *P,
                                const void *cs, const void *A, const void *B,
                                const void *gradA, const void *gradB,
                                const void *dv, double eta_crit,
                                double eta_fold, double dt,
                                const void *const a_grav[3],
                                const void *const a_hydro[3], void *dudt) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    return energy_compatible(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA,
                             gradB, dv, eta_crit, eta_fold, dt, nullptr, 0, -1,
                             a_grav, a_hydro, dudt);
}

int crk_hydro_energy_compatible_block(
    crk_ctx *ctx, crk_tree *t, const void *m, const void *vx, const void *vy,
    const void *vz, const void *V, const void *rho, const void *P,
    const void *cs, const void *A, const void *B, const void *gradA,
    const void *gradB, const void *dv, double eta_crit, double eta_fold,
    double dt, int32_t max_level, const int32_t *bins_gas, int64_t substep,
    const void *const a_grav[3], const void *const a_hydro[3], void *dudt) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    if (max_level < 0 || max_level > 30)
        return set_error(CRK_EINVAL, "max_level must be in [0, 30]");
    if (substep < -1 || substep >= ((int64_t)1 << max_level))
        return set_error(CRK_EINVAL, "substep must be in [-1, 2^max_level)");
    if (!(dt > 0.0) || !std::isfinite(dt))
        return set_error(CRK_EINVAL, "dt must be finite and > 0");
    CRK_TRY(check_ptr(bins_gas, 4, "bins_gas", t->n_gas > 0));
    // the pass writes the particles crk_tree_set_active selected: they must
    // be the ones this kick moves
    if (substep < 0 ? t->act_on
                    : (!t->act_on || t->act_substep != substep ||
                       t->act_level != max_level))
        return set_error(CRK_ESTATE,
                         "crk_tree_set_active must select the same substep "
                         "and max_level (everything for substep -1)");
    return energy_compatible(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA,
                             gradB, dv, eta_crit, eta_fold, dt, bins_gas,
                             max_level, substep, a_grav, a_hydro, dudt);
}

int crk_velocity_gradient(crk_ctx *ctx, crk_tree *t, const void *vx,
                          const void *vy, const void *vz, const void *V,
                          const void *A, const void *B, const void *gradA,
                          const void *gradB, void *dv) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    const void *ins[] = {vx, vy, vz, V, A, B, gradA, gradB};
    const char *in_names[] = {"vx", "vy", "vz", "V", "A", "B", "gradA", "gradB"};
    for (int k = 0; k < 8; ++k) CRK_TRY(check_ptr(ins[k], el, in_names[k], g));
    CRK_TRY(check_ptr(dv, el, "dv", g));
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_VGRAD);
    return pass_velocity_gradient(ctx, t, vx, vy, vz, V, A, B, gradA, gradB, dv);
}

int crk_hydro_forces_limited(crk_ctx *ctx, crk_tree *t, const void *m,
                             const void *vx, const void *vy, const void *vz,
                             const void *V, const void *rho, const void *P,
                             const void *cs, const void *A, const void *B,
                             const void *gradA, const void *gradB,
                             const void *dv, double eta_crit, double eta_fold,
                             void *ax, void *ay, void *az, void *dudt) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0;
    const void *ins[] = {m, vx, vy, vz, V, rho, P, cs, A, B, gradA, gradB, dv};
    const char *in_names[] = {"m", "vx", "vy", "vz", "V", "rho", "P", "cs",
                              "A", "B", "gradA", "gradB", "dv"};
    for (int k = 0; k < 13; ++k) CRK_TRY(check_ptr(ins[k], el, in_names[k], g));
    void *outs[] = {ax, ay, az, dudt};
    const char *out_names[] = {"ax", "ay", "az", "dudt"};
    for (int k = 0; k < 4; ++k) CRK_TRY(check_ptr(outs[k], el, out_names[k], g));
    if (!(eta_crit >= 0.0) || !std::isfinite(eta_crit) || !(eta_fold > 0.0) ||
        !std::isfinite(eta_fold))
        return set_error(CRK_EINVAL,
                         "eta_crit must be finite and >= 0, eta_fold finite and > 0");
    if (!g) return CRK_OK;
    PassSpan sp(ctx, P_HYDRO);
    return pass_hydro(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA, gradB,
                      dv, eta_crit, eta_fold, ax, ay, az, dudt);
}

int shortrange_gravity(crk_ctx *ctx, crk_tree *t, const void *m_gas,
                       const void *m_dm, void *ax_gas, void *ay_gas,
                       void *az_gas, void *ax_dm, void *ay_dm, void *az_dm) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0, d = t->n_dm > 0;
    CRK_TRY(check_ptr(m_gas, el, "m_gas", g));
    CRK_TRY(check_ptr(ax_gas, el, "ax_gas", g));
    CRK_TRY(check_ptr(ay_gas, el, "ay_gas", g));
    CRK_TRY(check_ptr(az_gas, el, "az_gas", g));
    CRK_TRY(check_ptr(m_dm, el, "m_dm", d));
    CRK_TRY(check_ptr(ax_dm, el, "ax_dm", d));
    CRK_TRY(check_ptr(ay_dm, el, "ay_dm", d));
    CRK_TRY(check_ptr(az_dm, el, "az_dm", d));
    PassSpan sp(ctx, P_GRAV);
    return pass_gravity(ctx, t, m_gas, m_dm, ax_gas, ay_gas, az_gas, ax_dm,
                        ay_dm, az_dm);
}

int crk_integrate(crk_ctx *ctx, int64_t n, double dt, double *x64, double *v64,
                  double *u64, const void *const a_grav[3],
                  const void *const a_hydro[3], const void *dudt,
                  void *const x[3], void *const v[3], void *u) {
    CRK_TRY(check_ctx(ctx));
    if (n < 0) return set_error(CRK_EINVAL, "n must be >= 0");
    if (!std::isfinite(dt)) return set_error(CRK_EINVAL, "dt must be finite");
    if (n == 0) return CRK_OK;
    if (!a_grav || !x || !v) return set_error(CRK_EINVAL, "null pointer array");
    const size_t el = ctx->elem();
    CRK_TRY(check_ptr(x64, 8, "x64", true));
    CRK_TRY(check_ptr(v64, 8, "v64", true));
    CRK_TRY(check_ptr(u64, 8, "u64", false));
    for (int a = 0; a < 3; ++a) {
        CRK_TRY(check_ptr(a_grav[a], el, "a_grav", true));
        CRK_TRY(check_ptr(x[a], el, "x", true));
        CRK_TRY(check_ptr(v[a], el, "v", true));
        if (a_hydro) CRK_TRY(check_ptr(a_hydro[a], el, "a_hydro", true));
    }
    if (u64) {
        CRK_TRY(check_ptr(dudt, el, "dudt", true));
        CRK_TRY(check_ptr(u, el, "u", true));
    }
    PassSpan sp(ctx, P_INTEG);
    return integrate(ctx, n, dt, x64, v64, u64, a_grav, a_hydro, dudt, x, v, u);
}

int crk_timestep_bins(crk_ctx *ctx, int64_t n, double dt, int32_t max_level,
                      double eps, double c_cfl, double eta,
                      const void *const a_grav[3], const void *const a_hydro[3],
                      const void *h, const void *cs, int32_t *bins) {
    CRK_TRY(check_ctx(ctx));
    if (n < 0) return set_error(CRK_EINVAL, "n must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(CRK_EINVAL, "dt must be > 0");
    if (max_level < 0 || max_level > 30)
        return set_error(CRK_EINVAL, "max_level must be in [0, 30]");
    if (!(eps > 0.0) || !(eta > 0.0) || !std::isfinite(eps) || !std::isfinite(eta))
        return set_error(CRK_EINVAL, "eps and eta must be > 0");
    if ((h == nullptr) != (cs == nullptr))
        return set_error(CRK_EINVAL, "h and cs: both or neither");
    if (h && !(c_cfl > 0.0)) return set_error(CRK_EINVAL, "c_cfl must be > 0");
    if (n == 0) return CRK_OK;
    if (!a_grav) return set_error(CRK_EINVAL, "null a_grav");
    const size_t el = ctx->elem();
    for (int a = 0; a < 3; ++a) {
        CRK_TRY(check_ptr(a_grav[a], el, "a_grav", true));
        if (a_hydro) CRK_TRY(check_ptr(a_hydro[a], el, "a_hydro", true));
    }
    CRK_TRY(check_ptr(h, el, "h", false));
    CRK_TRY(check_ptr(cs, el, "cs", false));
    CRK_TRY(check_ptr(bins, 4, "bins", true));
    return timestep_bins(ctx, n, dt, max_level, eps, c_cfl, eta, a_grav, a_hydro,
                         h, cs, bins);
}

int crk_tree_set_active(crk_ctx *ctx, crk_tree *t, const int32_t *bins_gas,
                        const int32_t *bins_dm, int32_t max_level,
                        int64_t substep) {
    CRK_TRY(check_tree_ready(ctx, t, false));
    if (ctx->capturing) return set_error(CRK_ESTATE, "set_active during capture");
    if (substep >= 0) {
        if (max_level < 0 || max_level > 30)
            return set_error(CRK_EINVAL, "max_level must be in [0, 30]");
        if (substep >= ((int64_t)1 << max_level))
            return set_error(CRK_EINVAL, "substep must be < 2^max_level");
        CRK_TRY(check_ptr(bins_gas, 4, "bins_gas", t->n_gas > 0));
        CRK_TRY(check_ptr(bins_dm, 4, "bins_dm", t->n_dm > 0));
    }
    return tree_set_active(ctx, t, bins_gas, bins_dm, max_level, substep);
}

int crk_tree_refit(crk_ctx *ctx, crk_tree *t, const void *gx, const void *gy,
                   const void *gz, const void *dx, const void *dy,
                   const void *dz) {
    CRK_TRY(check_tree_ready(ctx, t, false));
    if (ctx->capturing) return set_error(CRK_ESTATE, "refit during capture");
    const size_t el = ctx->elem();
    const bool g = t->n_gas > 0, d = t->n_dm > 0;
    CRK_TRY(check_ptr(gx, el, "gx", g));
    CRK_TRY(check_ptr(gy, el, "gy", g));
    CRK_TRY(check_ptr(gz, el, "gz", g));
    CRK_TRY(check_ptr(dx, el, "dx", d));
    CRK_TRY(check_ptr(dy, el, "dy", d));
    CRK_TRY(check_ptr(dz, el, "dz", d));
    PassSpan sp(ctx, P_TREE);
    return tree_refit(ctx, t, gx, gy, gz, dx, dy, dz);
}

int crk_kick(crk_ctx *ctx, int64_t n, double dt, int32_t max_level,
             int64_t substep, int32_t phase, const int32_t *bins, double *v64,
             double *u64, const void *const a_grav[3],
             const void *const a_hydro[3], const void *dudt, void *const v[3],
             void *u) {
    CRK_TRY(check_ctx(ctx));
    if (n < 0) return set_error(CRK_EINVAL, "n must be >= 0");
    if (!std::isfinite(dt)) return set_error(CRK_EINVAL, "dt must be finite");
    if (max_level < 0 || max_level > 30)
        return set_error(CRK_EINVAL, "max_level must be in [0, 30]");
    if (substep < 0 || substep >= ((int64_t)1 << max_level))
        return set_error(CRK_EINVAL, "substep must be in [0, 2^max_level)");
    if (phase != 0 && phase != 1) return set_error(CRK_EINVAL, "phase must be 0 or 1");
    if (n == 0) return CRK_OK;
    if (!a_grav || !v) return set_error(CRK_EINVAL, "null pointer array");
    const size_t el = ctx->elem();
    CRK_TRY(check_ptr(bins, 4, "bins", true));
    CRK_TRY(check_ptr(v64, 8, "v64", true));
    CRK_TRY(check_ptr(u64, 8, "u64", false));
    for (int a = 0; a < 3; ++a) {
        CRK_TRY(check_ptr(a_grav[a], el, "a_grav", true));
        CRK_TRY(check_ptr(v[a], el, "v", true));
        if (a_hydro) CRK_TRY(check_ptr(a_hydro[a], el, "a_hydro", true));
    }
    if (u64) {
        CRK_TRY(check_ptr(dudt, el, "dudt", true));
        CRK_TRY(check_ptr(u, el, "u", true));
    }
    PassSpan sp(ctx, P_INTEG);
    return block_kick(ctx, n, dt, max_level, substep, phase, bins, v64, u64,
                      a_grav, a_hydro, dudt, v, u);
}

int crk_drift(crk_ctx *ctx, int64_t n, double delta, int32_t wrap, double *x64,
              const double *v64, void *const x[3]) {
    CRK_TRY(check_ctx(ctx));
    if (n < 0) return set_error(CRK_EINVAL, "n must be >= 0");
    if (!std::isfinite(delta)) return set_error(CRK_EINVAL, "delta must be finite");
    if (n == 0) return CRK_OK;
    if (!x) return set_error(CRK_EINVAL, "null pointer array");
    const size_t el = ctx->elem();
    CRK_TRY(check_ptr(x64, 8, "x64", true));
    CRK_TRY(check_ptr(v64, 8, "v64", true));
    for (int a = 0; a < 3; ++a) CRK_TRY(check_ptr(x[a], el, "x", true));
    PassSpan sp(ctx, P_INTEG);
    return drift(ctx, n, delta, wrap ? 1 : 0, x64, v64, x);
}

int crk_pm_gravity(crk_ctx *ctx, int32_t n_mesh, double r_c, int64_t n_gas,
                   const void *gx, const void *gy, const void *gz,
                   const void *m_gas, int64_t n_dm, const void *dx,
                   const void *dy, const void *dz, const void *m_dm,
                   void *const a_gas[3], void *const a_dm[3]) {
    CRK_TRY(check_ctx(ctx));
    if (n_mesh < 4 || n_mesh > 2048 || (n_mesh & 1))
        return set_error(CRK_EINVAL, "n_mesh must be even, in [4, 2048]");
    if (!(r_c > 0.0) || !(r_c < 0.5) || !std::isfinite(r_c))
        return set_error(CRK_EINVAL, "r_c must be in (0, 0.5)");
    if (n_gas < 0 || n_dm < 0) return set_error(CRK_EINVAL, "counts must be >= 0");
    if (ctx->capturing) return set_error(CRK_ESTATE, "pm_gravity during capture");
    const size_t el = ctx->elem();
    const bool g = n_gas > 0, d = n_dm > 0;
    CRK_TRY(check_ptr(gx, el, "gx", g));
    CRK_TRY(check_ptr(gy, el, "gy", g));
    CRK_TRY(check_ptr(gz, el, "gz", g));
    CRK_TRY(check_ptr(m_gas, el, "m_gas", g));
    CRK_TRY(check_ptr(dx, el, "dx", d));
    CRK_TRY(check_ptr(dy, el, "dy", d));
    CRK_TRY(check_ptr(dz, el, "dz", d));
    CRK_TRY(check_ptr(m_dm, el, "m_dm", d));
    if ((g && !a_gas) || (d && !a_dm)) return set_error(CRK_EINVAL, "null pointer array");
    for (int a = 0; a < 3; ++a) {
        if (g) CRK_TRY(check_ptr(a_gas[a], el, "a_gas", true));
        if (d) CRK_TRY(check_ptr(a_dm[a], el, "a_dm", true));
    }
    PassSpan sp(ctx, P_GRAV);
    return pm_gravity(ctx, n_mesh, r_c, n_gas, gx, gy, gz, m_gas, n_dm, dx, dy,
                      dz, m_dm, a_gas, a_dm);
}

int crk_fof(crk_ctx *ctx, crk_tree *t, double b, int32_t *labels_gas,
            int32_t *labels_dm) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    if (ctx->capturing) return set_error(CRK_ESTATE, "fof during capture");
    if (t->act_on) return set_error(CRK_ESTATE, "fof with an active subset set");
    if (!(b > 0.0) || !std::isfinite(b))
        return set_error(CRK_EINVAL, "linking length must be > 0");
    for (double rc : t->cur_rc)
        if (b > rc)
            return set_error(CRK_EINVAL,
                             "linking length above r_c (the gravity lists' range)");
    if (t->n >= ((int64_t)1 << 31) - 1)
        return set_error(CRK_EINVAL, "fof: too many particles for int32 labels");
    CRK_TRY(check_ptr(labels_gas, 4, "labels_gas", t->n_gas > 0));
    CRK_TRY(check_ptr(labels_dm, 4, "labels_dm", t->n_dm > 0));
    return fof_groups(ctx, t, b, labels_gas, labels_dm);
}

int crk_fof_properties(crk_ctx *ctx, int64_t n_gas, int64_t n_dm,
                       const int32_t *labels_gas, const int32_t *labels_dm,
                       const void *const gas_x[3], const void *m_gas,
                       const void *const dm_x[3], const void *m_dm,
                       int32_t *count, double *mass, double *centre) {
    CRK_TRY(check_ctx(ctx));
    if (n_gas < 0 || n_dm < 0) return set_error(CRK_EINVAL, "counts must be >= 0");
    if (n_gas + n_dm >= ((int64_t)1 << 31) - 1)
        return set_error(CRK_EINVAL, "fof_properties: too many particles for int32 labels");
    const size_t el = ctx->elem();
    const bool g = n_gas > 0, d = n_dm > 0;
    if ((g && !gas_x) || (d && !dm_x)) return set_error(CRK_EINVAL, "null pointer array");
    for (int a = 0; a < 3; ++a) {
        if (g) CRK_TRY(check_ptr(gas_x[a], el, "gas_x", true));
        if (d) CRK_TRY(check_ptr(dm_x[a], el, "dm_x", true));
    }
    CRK_TRY(check_ptr(labels_gas, 4, "labels_gas", g));
    CRK_TRY(check_ptr(labels_dm, 4, "labels_dm", d));
    CRK_TRY(check_ptr(m_gas, el, "m_gas", g));
    CRK_TRY(check_ptr(m_dm, el, "m_dm", d));
    const bool any = g || d;
    CRK_TRY(check_ptr(count, 4, "count", any));
    CRK_TRY(check_ptr(mass, 8, "mass", any));
    CRK_TRY(check_ptr(centre, 8, "centre", any));
    if (!any) return CRK_OK;
    return fof_properties(ctx, n_gas, n_dm, labels_gas, labels_dm,
                          g ? gas_x : nullptr, m_gas, d ? dm_x : nullptr, m_dm,
                          count, mass, centre);
}

int crk_count_pairs(crk_ctx *ctx, crk_tree *t, int64_t totals[6]) {
    CRK_TRY(check_tree_ready(ctx, t, true));
    if (!totals) return set_error(CRK_EINVAL, "null totals");
    if (ctx->capturing) return set_error(CRK_ESTATE, "count during capture");
    return count_pairs(ctx, t, totals);
}

int crk_tree_get_info(const crk_tree *t, crk_tree_info *info) {
    if (!t || !info) return set_error(CRK_EINVAL, "null tree or info");
    info->n_gas = t->n_gas;
    info->n_dm = t->n_dm;
    info->n_leaves = t->n_leaves;
    info->n_gas_leaves = t->n_gas_leaves;
    info->n_bins = t->total_bins;
    info->grav_entries = t->grav_entries;
    info->hydro_entries = t->hydro_entries;
    info->kd_levels = t->kd_levels;
    info->act_leaves = t->act_on ? t->act_nall : 0;
    info->act_particles = t->act_on ? t->act_npart : 0;
    info->act_grouped = t->act_on && t->grp_on ? 1 : 0;
    return CRK_OK;
}

int crk_tree_get_leaves(crk_ctx *ctx, const crk_tree *t, int64_t *perm,
                        int64_t *leaf_start, int64_t *leaf_count) {
    CRK_TRY(check_tree_ready(ctx, t, false));
    if (ctx->capturing) return set_error(CRK_ESTATE, "query during capture");
    CRK_HIP(hipStreamSynchronize(ctx->stream));
    const int cur = t->cur_nodes;
    if (perm && t->n > 0) {
        std::vector<int32_t> tmp(t->n);
        CRK_HIP(hipMemcpy(tmp.data(), t->perm.p, t->n * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < t->n; ++i) perm[i] = tmp[i];
    }
    if ((leaf_start || leaf_count) && t->n_leaves > 0) {
        std::vector<int32_t> a(t->n_leaves), b(t->n_leaves);
        CRK_HIP(hipMemcpy(a.data(), t->nd_start[cur].p, t->n_leaves * 4,
                          hipMemcpyDeviceToHost));
        CRK_HIP(hipMemcpy(b.data(), t->nd_count[cur].p, t->n_leaves * 4,
                          hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < t->n_leaves; ++k) {
            if (leaf_start) leaf_start[k] = a[k];
            if (leaf_count) leaf_count[k] = b[k];
        }
    }
    return CRK_OK;
}

int crk_graph_begin(crk_ctx *ctx) {
    CRK_TRY(check_ctx(ctx));
    if (!ctx->stream)
        return set_error(CRK_EINVAL, "graph capture needs a non-default stream");
    if (ctx->capturing) return set_error(CRK_ESTATE, "capture already active");
    CRK_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    return CRK_OK;
}

int crk_graph_end(crk_ctx *ctx) {
    CRK_TRY(check_ctx(ctx));
    if (!ctx->capturing) return set_error(CRK_ESTATE, "no capture active");
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    CRK_HIP(hipStreamEndCapture(ctx->stream, &g));
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph = g;
    ctx->graph_exec = nullptr;
    CRK_HIP(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
    ctx->graph_gen = alloc_generation();
    return CRK_OK;
}

int crk_graph_reset(crk_ctx *ctx) {
    CRK_TRY(check_ctx(ctx));
    if (ctx->capturing) return set_error(CRK_ESTATE, "graph reset during capture");
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    return CRK_OK;
}

int crk_graph_launch(crk_ctx *ctx) {
    CRK_TRY(check_ctx(ctx));
    if (!ctx->graph_exec) return set_error(CRK_ESTATE, "no graph captured");
    // the graph's kernels hold raw pointers: a buffer grown, moved or freed
    // since the capture (an eager build at a larger size, crk_tree_free)
    // would be a use after free, so such a graph is never launched
    if (ctx->graph_gen != alloc_generation())
        return set_error(CRK_ESTATE,
                         "library buffers were reallocated or freed since the "
                         "graph was captured; capture it again");
    CRK_HIP(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    return CRK_OK;
}

int crk_tree_free(crk_tree *t) {
    if (!t) return CRK_OK;
    crk_ctx *c = t->owner;
    if (c) {
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        else (void)hipDeviceSynchronize();
    }
    DevBuf *bufs[] = {&t->d_gas_off, &t->d_dm_off, &t->d_ncm, &t->d_bin_base,
                      &t->d_rc, &t->d_eps, &t->d_hmax, &t->binkey, &t->flag_c,
                      &t->f_pos, &t->f_scan, &t->elem_node, &t->elem_node2,
                      &t->perm, &t->hsm, &t->nd_split, &t->nd_left, &t->nd_axis,
                      &t->nd_child, &t->nd_nchild, &t->counters, &t->leaf_box,
                      &t->leaf_lo, &t->leaf_hi, &t->leaf_hmax, &t->bin_leaf,
                      &t->bin_cnt, &t->g_cnt, &t->h_cnt, &t->g_off, &t->h_off,
                      &t->g_list, &t->h_list};
    for (DevBuf *b : bufs) b->release();
    for (int i = 0; i < 2; ++i) {
        t->keys[i].release();
        t->vals[i].release();
        t->nd_start[i].release();
        t->nd_count[i].release();
        t->nd_key[i].release();
    }
    for (int a = 0; a < 3; ++a) {
        t->S[a].release();
        t->S2[a].release();
        t->pos[a].release();
    }
    for (auto &b : t->pf) b.release();
    t->h_boxinfo.release();
    delete t;
    return CRK_OK;
}

int crk_timing_enable(crk_ctx *ctx, int enable) {
    CRK_TRY(check_ctx(ctx));
    if (ctx->capturing) return set_error(CRK_ESTATE, "timing change during capture");
    ctx->timing = enable != 0;
    return CRK_OK;
}

int crk_pass_times(crk_ctx *ctx, double pass_ms[9], double kernel_ms[9],
                   int64_t launches[9]) {
    CRK_TRY(check_ctx(ctx));
    if (ctx->capturing) return set_error(CRK_ESTATE, "query during capture");
    CRK_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < P_COUNT; ++k) {
        if (pass_ms) pass_ms[k] = 0.0;
        if (kernel_ms) kernel_ms[k] = 0.0;
        if (launches) launches[k] = 0;
    }
    for (auto &s : ctx->spans) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, s.a, s.b);
        if (s.kernel) {
            if (kernel_ms) kernel_ms[s.pass] += ms;
            if (launches) launches[s.pass] += 1;
        } else if (pass_ms) {
            pass_ms[s.pass] += ms;
        }
        (void)hipEventDestroy(s.a);
        (void)hipEventDestroy(s.b);
    }
    ctx->spans.clear();
    return CRK_OK;
}

}  // extern "C"
