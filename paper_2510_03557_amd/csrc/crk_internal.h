// Internal declarations of the MI355X short-range step library.
// Everything here is private to the library; the public ABI is crk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/crk.h"

namespace crk {

// --------------------------------------------------------------------------
// error handling
// --------------------------------------------------------------------------

// Sets the thread-local last-error message and returns the status.
int set_error(int status, const std::string &msg);

#define CRK_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            return ::crk::set_error(CRK_EDEVICE,                             \
                                    std::string(#call ": ") +                \
                                        hipGetErrorString(e_));              \
    } while (0)

#define CRK_TRY(call)                                                        \
    do {                                                                     \
        int s_ = (call);                                                     \
        if (s_ != CRK_OK) return s_;                                         \
    } while (0)

// Bits of the device-side error word.
enum : int {
    DEV_ERR_INPUT = 1,     // non-finite / out-of-range position or h
    DEV_ERR_HMAX = 2,      // h above the declared per-box bound
    DEV_ERR_CAPACITY = 4,  // list or k-d capacity fixed at capture exceeded
};

// --------------------------------------------------------------------------
// device buffers
// --------------------------------------------------------------------------

// Every release of library memory (device or pinned host), including the
// old block of a buffer that grows, advances a process-wide generation.  A
// captured graph holds raw pointers, so it may be replayed only while the
// generation it was captured at is current (checked by crk_graph_launch).
uint64_t alloc_generation();
void alloc_generation_bump();

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    // Grows to at least n bytes (contents are not preserved).  Fails when
    // growth is needed during graph capture.
    int ensure(size_t n, bool capturing);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    int ensure(size_t n);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// --------------------------------------------------------------------------
// context and tree
// --------------------------------------------------------------------------

enum PassId {
    P_TREE = 0, P_LISTS, P_DENSITY, P_COEFF, P_HYDRO, P_GRAV, P_INTEG, P_VGRAD,
    P_ENERGY, P_COUNT
};

// long-range mesh workspace (pm.hip): double deposit mesh, real mesh and
// two half-spectra of the context precision, and the FFT plans of one size
struct crk_pm {
    DevBuf rho, real, rhok, tmpk;
    int n = 0, elem = 0;
    bool plans = false;
    hipfftHandle fwd = nullptr, inv = nullptr;
};
void pm_release(crk_pm &pm);

struct TimedSpan {
    int pass;
    bool kernel;  // true: the pass's main kernel only
    hipEvent_t a, b;
};

}  // namespace crk

struct crk_ctx {
    int precision = CRK_FP32;
    hipStream_t stream = nullptr;
    crk_params params{};
    crk_tuning tuning{};
    int device = 0;
    int n_cu = 256;
    bool capturing = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_gen = 0;   // allocation generation at the last capture
    void *noalloc_scratch = nullptr;  // this device's static scratch array
    std::string noalloc_error;        // why it is missing, if it is
    crk::DevBuf err;          // int error word + int64 required capacity
    crk::HostBuf err_host;
    crk::DevBuf scratch;      // primitives' temporary storage
    bool timing = false;
    crk::crk_pm pm;
    std::vector<crk::TimedSpan> spans;
    std::vector<hipEvent_t> event_pool;
    size_t elem() const { return precision == CRK_FP64 ? 8 : 4; }
};

struct crk_tree {
    crk_ctx *owner = nullptr;
    // sizes
    int64_t n_gas = 0, n_dm = 0, n = 0;
    int32_t n_boxes = 0;
    int64_t total_bins = 0;
    int32_t bin_bits = 0;
    int32_t leaf_max = 64;
    int64_t leaf_cap = 0;       // upper bound of the leaf count
    int64_t n_leaves = 0;       // last eager value (host)
    int64_t n_gas_leaves = 0;   // last eager value (host)
    // launch bounds of leaf-indexed kernels: the eager counts, or under
    // capture the graph bounds (eager count + 25 % + 1024, at most leaf_cap)
    int64_t nb_launch = 0, ngb_launch = 0;
    int64_t graph_nb = 0, graph_ngb = 0;
    int32_t kd_levels = 0;      // levels run by the last eager build
    int64_t grav_cap = 0, hydro_cap = 0;        // list capacities (entries)
    int64_t grav_entries = 0, hydro_entries = 0;  // last eager values
    bool lists_built = false;

    // host copies of the box description (pinned, read by captured copies)
    crk::HostBuf h_boxinfo;
    std::vector<int64_t> cur_gas_off, cur_dm_off;
    std::vector<double> cur_rc, cur_eps, cur_hmax;

    // device: per box
    crk::DevBuf d_gas_off, d_dm_off;   // int64 [n_boxes+1]
    crk::DevBuf d_ncm;                 // int32 [n_boxes]
    crk::DevBuf d_bin_base;            // int64 [n_boxes+1]
    crk::DevBuf d_rc, d_eps, d_hmax;   // double [n_boxes]

    // device: per particle (tree order unless noted)
    crk::DevBuf keys[2], vals[2];      // radix-sort double buffers
    crk::DevBuf S[3], S2[3];           // axis-sorted caller indices (int32)
    crk::DevBuf binkey;                // int32 bin key per sorted slot
    crk::DevBuf flag_c;                // int32 per caller index
    crk::DevBuf f_pos, f_scan;         // int32 per slot
    crk::DevBuf elem_node, elem_node2; // int32 per slot
    crk::DevBuf perm;                  // int32 caller index per slot
    crk::DevBuf iperm;                 // int32 slot per caller index
    crk::DevBuf pos[3];                // T, tree-order positions
    crk::DevBuf hsm;                   // T, tree-order smoothing lengths (gas slots)

    // device: k-d nodes / leaves
    crk::DevBuf nd_start[2], nd_count[2], nd_key[2];  // int32
    crk::DevBuf nd_split, nd_left, nd_axis, nd_child, nd_nchild; // int32
    int32_t *S_final[3] = {nullptr, nullptr, nullptr};  // axis-sorted, final
    std::vector<int32_t> h_ncm;        // host copy of bins per side per box
    std::vector<double> h_rc;          // host copy of r_c per box
    crk::DevBuf counters;              // int64 scalars (see tree.hip)
    crk::DevBuf leaf_box;              // int32
    crk::DevBuf leaf_lo, leaf_hi;      // T [3][leaf_cap]
    crk::DevBuf leaf_hmax;             // T
    crk::DevBuf bin_leaf;              // int32 [2*total_bins + 1]
    crk::DevBuf bin_cnt;               // int32 [2*total_bins + 1]
    // sub-leaves: every leaf of <= 64 particles is split by up to two more
    // k-d levels into <= 4 sub-leaves of <= 16 (slots 4*leaf + k)
    bool has_sub = false;
    crk::DevBuf sub_nsub;              // int32 per leaf
    crk::DevBuf sub_start, sub_count;  // int32 per slot
    crk::DevBuf sub_lo, sub_hi;        // T [3][4*leaf_cap]
    crk::DevBuf sub_hmax;              // T per slot
    int cur_nodes = 0;                 // which node buffer holds the leaves
    bool lds_tree = false;             // last eager build used the per-bin
                                       // LDS build (captures follow it)
    int32_t seg_size = 64;             // padded segment size of that build

    // device: interaction lists
    crk::DevBuf g_cnt, h_cnt;          // int32 per leaf
    crk::DevBuf g_off, h_off;          // int64 per leaf + 1
    crk::DevBuf g_list, h_list;        // uint32 entries: leaf | shift << 27
    // work queue: per-leaf cost (candidate pairs) and cost-descending order
    crk::DevBuf g_cost, h_cost;        // int32 per leaf
    crk::DevBuf ord_k[2], ord_v[2];    // radix-sort buffers
    crk::DevBuf g_order, h_order;      // int32 leaf index per queue slot
    crk::DevBuf q_counter;             // int32 queue heads (one per launch)
    bool orders_built = false;

    // device: per-pass scratch (tree order)
    crk::DevBuf pf[32];                // pass fields, reused between passes

    // active subset of a hierarchical time step (crk_tree_set_active):
    // per-slot flags, active leaves in leaf order (gas leaves first), device
    // counts {all, gas} and their host copies
    bool act_on = false;
    int64_t act_substep = -1;          // the selection's substep and levels
    int act_level = 0;
    crk::DevBuf act_flags;             // uint8 per slot
    crk::DevBuf act_leaf;              // int32 per leaf (flag, then scan)
    crk::DevBuf act_items;             // int32 per active leaf
    // int32 {active leaves, active gas leaves, scan total, active slots,
    //        sub-leaf entries, gas sub-leaf entries}
    crk::DevBuf act_count;
    int64_t act_nall = 0, act_ngas = 0, act_npart = 0;
    // the sub-leaves of the active leaves that hold an active particle (or,
    // with groups, their groups), one entry 4 leaf + g each, in leaf order
    // (gas leaves' entries first): the split sweeps launch one wavefront per
    // entry.  Valid while slist_on (set with the subset, dropped by refit)
    bool slist_on = false;
    crk::DevBuf act_sub;               // int32 [3][leaf_cap + 1]: mask, count, offset
    crk::DevBuf act_slist;             // int32 [4 * leaf_cap]
    // dense groups of the active particles of every active leaf (tuning
    // act_groups, trees with sub-leaves): the sub-leaf tables of the
    // subset, group g of leaf I in slot 4 I + g
    bool grp_on = false;
    crk::DevBuf grp_nsub;              // int32 per leaf
    crk::DevBuf grp_cnt;               // int32 per slot
    crk::DevBuf grp_idx;               // int32 [16] per slot: tree slots
    crk::DevBuf grp_lo, grp_hi;        // T [3][4*leaf_cap]
    crk::DevBuf grp_hmax;              // T per slot
    crk::DevBuf overhang;              // int flag: a leaf left the stencil (refit)
};

namespace crk {

// --------------------------------------------------------------------------
// primitives (primitives.hip)
// --------------------------------------------------------------------------

// Exclusive prefix sum of n values; optional device pointer receiving the
// total.  tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n,
                              int32_t *d_total, void *tmp, hipStream_t s);
hipError_t exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out,
                                     int64_t n, int64_t *d_total, void *tmp,
                                     hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys.  keys[0]/vals[0] hold the input; returns the index (0 or 1) of the
// buffer pair holding the sorted result.  tmp: radix_tmp_bytes(n).
size_t radix_tmp_bytes(int64_t n);
int radix_sort_u64_i32(uint64_t *keys[2], int32_t *vals[2], int64_t n,
                       int bits, void *tmp, hipStream_t s, hipError_t *err);

// fill kernel (graph-safe replacement of memset)
hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

// --------------------------------------------------------------------------
// stages (tree.hip, lists.hip, passes.hip, integrate.hip)
// --------------------------------------------------------------------------

int tree_build(crk_ctx *ctx, crk_tree *t, const crk_boxes *boxes,
               const void *gx, const void *gy, const void *gz,
               const void *gh, const void *dx, const void *dy,
               const void *dz);
int lists_build(crk_ctx *ctx, crk_tree *t);
int pass_density(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                 void *rho_tilde);
// crk_density with the tree-order masses in caller-provided scratch (at
// least n_gas values of the context precision); allocates nothing
int pass_density_scratch(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                         void *rho_tilde, void *scratch);
int pass_coefficients(crk_ctx *ctx, crk_tree *t, const void *m,
                      const void *V, const void *u, void *A, void *B,
                      void *gradA, void *gradB, void *rho, void *P,
                      void *cs);
int pass_hydro(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
               const void *vy, const void *vz, const void *V,
               const void *rho, const void *P, const void *cs, const void *A,
               const void *B, const void *gradA, const void *gradB,
               const void *dv, double eta_crit, double eta_fold, void *ax,
               void *ay, void *az, void *dudt);
int pass_energy_compatible(crk_ctx *ctx, crk_tree *t, const void *m,
                           const void *vx, const void *vy, const void *vz,
                           const void *V, const void *rho, const void *P,
                           const void *cs, const void *A, const void *B,
                           const void *gradA, const void *gradB, const void *dv,
                           double eta_crit, double eta_fold, double dt,
                           const int32_t *bins, int max_level, int64_t substep,
                           const void *const a_grav[3],
                           const void *const a_hydro[3], void *dudt);
int pass_velocity_gradient(crk_ctx *ctx, crk_tree *t, const void *vx,
                           const void *vy, const void *vz, const void *V,
                           const void *A, const void *B, const void *gradA,
                           const void *gradB, void *dv);
int pass_gravity(crk_ctx *ctx, crk_tree *t, const void *m_gas,
                 const void *m_dm, void *ax_gas, void *ay_gas, void *az_gas,
                 void *ax_dm, void *ay_dm, void *az_dm);
int count_pairs(crk_ctx *ctx, crk_tree *t, int64_t totals[6]);
int integrate(crk_ctx *ctx, int64_t n, double dt, double *x64, double *v64,
              double *u64, const void *const a_grav[3],
              const void *const a_hydro[3], const void *dudt,
              void *const x[3], void *const v[3], void *u);
// hierarchical time steps (substep.hip)
int timestep_bins(crk_ctx *ctx, int64_t n, double dt, int max_level,
                  double eps, double c_cfl, double eta,
                  const void *const a_grav[3], const void *const a_hydro[3],
                  const void *h, const void *cs, int32_t *bins);
int tree_set_active(crk_ctx *ctx, crk_tree *t, const int32_t *bins_gas,
                    const int32_t *bins_dm, int max_level, int64_t substep);
int tree_refit(crk_ctx *ctx, crk_tree *t, const void *gx, const void *gy,
               const void *gz, const void *dx, const void *dy,
               const void *dz);
int block_kick(crk_ctx *ctx, int64_t n, double dt, int max_level,
               int64_t substep, int phase, const int32_t *bins, double *v64,
               double *u64, const void *const a_grav[3],
               const void *const a_hydro[3], const void *dudt,
               void *const v[3], void *u);
int drift(crk_ctx *ctx, int64_t n, double delta, int wrap, double *x64,
          const double *v64, void *const x[3]);
// friends-of-friends groups over the gravity lists (passes.hip)
int fof_groups(crk_ctx *ctx, crk_tree *t, double b, int32_t *labels_gas,
               int32_t *labels_dm);
// long-range gravity on a mesh (pm.hip)
int pm_gravity(crk_ctx *ctx, int n_mesh, double r_c, int64_t n_gas,
               const void *gx, const void *gy, const void *gz, const void *m_gas,
               int64_t n_dm, const void *dx, const void *dy, const void *dz,
               const void *m_dm, void *const a_gas[3], void *const a_dm[3]);

// timing helpers (capi.cpp): bracket a span on the context stream
void span_begin(crk_ctx *ctx, int pass, bool kernel, hipEvent_t *ev);
void span_end(crk_ctx *ctx, int pass, bool kernel, hipEvent_t ev);

// device error word access for kernels
inline int *dev_err_word(crk_ctx *ctx) { return ctx->err.as<int>(); }
inline long long *dev_required(crk_ctx *ctx) {
    return reinterpret_cast<long long *>(ctx->err.as<char>() + 8);
}

// int32 counters of the tree build (tree->counters)
enum { C_NN = 0, C_NN_NEXT = 1, C_ANY = 2, C_MAXC = 3 };
// int64 counters of the list build (tree->counters, int64 view from 8)
enum { C64_GTOT = 8, C64_HTOT = 9 };

// list entry encoding: leaf index in the low 27 bits, periodic image code
// (sx+1)*9 + (sy+1)*3 + (sz+1) in the high 5 bits.
constexpr uint32_t LIST_LEAF_BITS = 27;
constexpr uint32_t LIST_LEAF_MASK = (1u << LIST_LEAF_BITS) - 1u;

}  // namespace crk
