// Hierarchical time steps on a tree kept for a whole interval: timestep
// bins, the active subset of a substep, the refit of the leaf boxes to
// drifted positions, and the block kick / drift of the double-precision
// state.  The paper's adaptive integration groups particles into timestep
// bins (Sec. IV-A); only active leaves are updated at a substep, and leaf
// bounding boxes grow instead of the tree being rebuilt (Sec. IV-B.1).
// Elementwise or per-leaf work, HBM/latency-bound.
#include <algorithm>
#include <cmath>
#include <limits>

#include "crk_internal.h"

namespace crk {

namespace {

inline unsigned grid_n(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)std::max<int64_t>(1, g);
}

#define GRID_LOOP(i, n)                                                     \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// Bin of every particle: the smallest b in [0, L] whose step
// tau = dt / 2^b satisfies tau^4 |a|^2 <= rhs_a (rhs_a = (2 eta eps)^2,
// the acceleration criterion tau <= sqrt(2 eta eps / |a|) squared twice)
// and, for gas, tau cs <= c_cfl h; L when none does.  Every product and
// sum is rounded once, in a fixed order (no contraction), so the integer
// decision is reproducible by any implementation of the same steps.
template <typename T>
__global__ void bins_kernel(int64_t n, double dt, int L, double rhs_a,
                            double c_cfl, const T *__restrict__ g0,
                            const T *__restrict__ g1, const T *__restrict__ g2,
                            const T *__restrict__ h0, const T *__restrict__ h1,
                            const T *__restrict__ h2, const T *__restrict__ hs,
                            const T *__restrict__ cs, int32_t *__restrict__ bins) {
#pragma clang fp contract(off)
    GRID_LOOP(i, n) {
        double ax = (double)g0[i], ay = (double)g1[i], az = (double)g2[i];
        if (h0) {
            ax = ax + (double)h0[i];
            ay = ay + (double)h1[i];
            az = az + (double)h2[i];
        }
        const double xx = ax * ax, yy = ay * ay, zz = az * az;
        const double a2 = (xx + yy) + zz;
        const double rc = hs ? c_cfl * (double)hs[i] : 0.0;
        const double c = hs ? (double)cs[i] : 0.0;
        int b = L;
        for (int k = 0; k <= L; ++k) {
            const double tau = ldexp(dt, -k);  // exact
            const double t2 = tau * tau;
            const double t4 = t2 * t2;
            bool ok = t4 * a2 <= rhs_a;
            if (hs) ok = ok && (tau * c <= rc);
            if (ok) {
                b = k;
                break;
            }
        }
        bins[i] = b;
    }
}

// level of slot p's particle (caller bins, clamped to [0, L])
__device__ inline int slot_bin(const int32_t *perm, int64_t n_gas,
                               const int32_t *bg, const int32_t *bd, int L,
                               int64_t p) {
    const int64_t c = perm[p];
    const int b = c < n_gas ? bg[c] : bd[c - n_gas];
    return b < 0 ? 0 : (b > L ? L : b);
}

// s < 0: every slot; else the slots ending a step after substep s.  Adds
// the number of active slots to *count (cleared by the caller).
__global__ void act_flags_kernel(int64_t n, int64_t n_gas,
                                 const int32_t *__restrict__ perm,
                                 const int32_t *__restrict__ bg,
                                 const int32_t *__restrict__ bd, int L, int64_t s,
                                 uint8_t *__restrict__ act,
                                 int32_t *__restrict__ count) {
    int c = 0;
    GRID_LOOP(p, n) {
        bool a = true;
        if (s >= 0) {
            const int64_t per = (int64_t)1 << (L - slot_bin(perm, n_gas, bg, bd, L, p));
            a = ((s + 1) % per) == 0;
        }
        act[p] = a ? 1 : 0;
        c += a ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// per leaf: 1 when any of its slots is active
__global__ void act_leaf_kernel(const int32_t *__restrict__ nn_ptr, int64_t cap,
                                const int32_t *__restrict__ lst,
                                const int32_t *__restrict__ lct,
                                const uint8_t *__restrict__ act,
                                int32_t *__restrict__ flag) {
    const int64_t nn = *nn_ptr;
    GRID_LOOP(I, cap) {
        int f = 0;
        if (I < nn) {
            const int st = lst[I], c = lct[I];
            for (int k = 0; k < c && !f; ++k) f = act[st + k];
        }
        flag[I] = f;
    }
}

__global__ void act_items_kernel(const int32_t *__restrict__ nn_ptr, int64_t cap,
                                 const int32_t *__restrict__ flag,
                                 const int32_t *__restrict__ pos,
                                 int32_t *__restrict__ items) {
    const int64_t nn = *nn_ptr;
    GRID_LOOP(I, cap) {
        if (I < nn && flag[I]) items[pos[I]] = (int32_t)I;
    }
}

// counts {all active leaves, active gas leaves}: gas leaves come first in
// leaf order, so the active gas leaves are the items before position
// pos[number of gas leaves]
__global__ void act_count_kernel(const int32_t *__restrict__ nn_ptr,
                                 const int32_t *__restrict__ ngl_ptr,
                                 const int32_t *__restrict__ pos,
                                 const int32_t *__restrict__ total,
                                 int32_t *__restrict__ out) {
    const int nn = *nn_ptr, ngl = *ngl_ptr;
    out[0] = *total;
    out[1] = ngl < nn ? pos[ngl] : *total;
}

// Sub-leaves of every active leaf holding an active particle: a mask of
// bits q < nsub (sub-leaf q) and its population per item, one wavefront
// per item (lanes = the leaf's slots, <= 64)
__global__ __launch_bounds__(64) void act_submask_kernel(
    const int32_t *__restrict__ items, int64_t n_items,
    const int32_t *__restrict__ lstart, const int32_t *__restrict__ lcount,
    const int32_t *__restrict__ nsub, const int32_t *__restrict__ sst,
    const int32_t *__restrict__ scnt, const uint8_t *__restrict__ act,
    int32_t *__restrict__ mask, int32_t *__restrict__ count) {
    const int64_t k = blockIdx.x;
    if (k >= n_items) return;
    const int I = items[k];
    const int lane = threadIdx.x;
    const int st = lstart[I], cnt = min(lcount[I], 64);
    const uint64_t m = __ballot(lane < cnt && act[st + lane] != 0);
    const int ns = min(nsub[I], 4);
    int bits = 0;
    for (int q = 0; q < ns; ++q) {
        const int lo = sst[4 * (int64_t)I + q] - st;
        const int c = scnt[4 * (int64_t)I + q];
        const uint64_t sm = (c >= 64 ? ~0ull : ((1ull << c) - 1)) << lo;
        if (m & sm) bits |= 1 << q;
    }
    if (lane == 0) {
        mask[k] = bits;
        count[k] = __popc(bits);
    }
}

// Entries 4 I + g of item k at off[k]: g = the sub-leaf, or with groups
// (compressed) its rank among the item's sub-leaves holding an active
// particle, which is the group index.  Thread k == n_items also writes the
// entries of the gas items (items [0, n_gas_items)) to cnt[5].
__global__ void act_sublist_kernel(const int32_t *__restrict__ items,
                                   int64_t n_items, int64_t n_gas_items,
                                   const int32_t *__restrict__ mask,
                                   const int32_t *__restrict__ off, int groups,
                                   int32_t *__restrict__ list,
                                   int32_t *__restrict__ cnt) {
    GRID_LOOP(k, n_items + 1) {
        if (k == n_gas_items) cnt[5] = k < n_items ? off[k] : cnt[4];
        if (k < n_items) {
            const int I = items[k], m = mask[k];
            int p = off[k], r = 0;
            for (int q = 0; q < 4; ++q) {
                if ((m >> q) & 1) {
                    list[p++] = 4 * I + (groups ? r : q);
                    ++r;
                }
            }
        }
    }
}

// new positions into tree order
template <typename T>
__global__ void refit_pos_kernel(int64_t n, int64_t n_gas,
                                 const int32_t *__restrict__ perm,
                                 const T *__restrict__ gx, const T *__restrict__ gy,
                                 const T *__restrict__ gz, const T *__restrict__ dx,
                                 const T *__restrict__ dy, const T *__restrict__ dz,
                                 T *__restrict__ p0, T *__restrict__ p1,
                                 T *__restrict__ p2) {
    GRID_LOOP(p, n) {
        const int64_t c = perm[p];
        if (c < n_gas) {
            p0[p] = gx[c];
            p1[p] = gy[c];
            p2[p] = gz[c];
        } else {
            p0[p] = dx[c - n_gas];
            p1[p] = dy[c - n_gas];
            p2[p] = dz[c - n_gas];
        }
    }
}

template <typename T> __device__ inline T wmin(T v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}
template <typename T> __device__ inline T wmax(T v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Groups of the active particles: one wavefront per active leaf (<= 64
// slots, one per lane).  Group g of leaf I holds the active particles of
// one of its sub-leaves, in slot order (sub-leaves without an active
// particle make no group), at grp_idx[16 (4 I + g) ...], with their count,
// the bounding box of their current positions and their largest h: the
// sweeps take only active i-particles, culled against a box no larger
// than their sub-leaf's.  (Merging sibling sub-leaves whose actives fit one
// group of 16 gives fewer, larger groups and measured slower: their boxes
// take in many more candidates.)
template <typename T>
__global__ __launch_bounds__(64) void act_groups_kernel(
    const int32_t *__restrict__ items, int64_t n_items,
    const int32_t *__restrict__ lstart, const int32_t *__restrict__ lcount,
    const int32_t *__restrict__ nsub, const int32_t *__restrict__ sst,
    const int32_t *__restrict__ scnt, const uint8_t *__restrict__ act,
    const T *__restrict__ px, const T *__restrict__ py,
    const T *__restrict__ pz, const T *__restrict__ h, int64_t lcap,
    int32_t *__restrict__ gnsub, int32_t *__restrict__ gcnt,
    int32_t *__restrict__ gidx, T *__restrict__ glo, T *__restrict__ ghi,
    T *__restrict__ ghm) {
    const int64_t k = blockIdx.x;
    if (k >= n_items) return;
    const int I = items[k];
    const int lane = threadIdx.x;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int st = lstart[I], cnt = min(lcount[I], 64);
    const int s = st + lane;
    const bool a = lane < cnt && act[s] != 0;
    const uint64_t m = __ballot(a);
    // lanes of each sub-leaf (contiguous slot ranges) and their actives
    const int ns = min(nsub[I], 4);
    auto lanes_of = [&](int q) -> uint64_t {
        if (q >= ns) return 0ull;
        const int lo = sst[4 * (int64_t)I + q] - st;
        const int c = scnt[4 * (int64_t)I + q];
        return (c >= 64 ? ~0ull : ((1ull << c) - 1)) << lo;
    };
    const uint64_t s0 = lanes_of(0), s1 = lanes_of(1), s2 = lanes_of(2),
                   s3 = lanes_of(3);
    // one group per sub-leaf holding an active particle
    const uint64_t c0 = (m & s0) ? s0 : 0ull, c1 = (m & s1) ? s1 : 0ull,
                   c2 = (m & s2) ? s2 : 0ull, c3 = (m & s3) ? s3 : 0ull;
    const int ng = (c0 != 0) + (c1 != 0) + (c2 != 0) + (c3 != 0);
    // group q is the q-th non-empty candidate
    auto gmask = [&](int q) -> uint64_t {
        int seen = 0;
        if (c0) { if (seen == q) return c0; ++seen; }
        if (c1) { if (seen == q) return c1; ++seen; }
        if (c2) { if (seen == q) return c2; ++seen; }
        if (c3 && seen == q) return c3;
        return 0ull;
    };
    if (lane == 0) gnsub[I] = ng;
    int g = 0;
    for (int q = 1; q < 4; ++q)
        if ((gmask(q) >> lane) & 1ull) g = q;
    if (a) {
        // < 16 by construction (sub-leaves hold <= 16); the bound keeps every
        // write inside the group's 16 entries regardless
        const int rank = __popcll(m & gmask(g) & lt_mask);
        if (rank < 16) gidx[(4 * (int64_t)I + g) * 16 + rank] = s;
    }
    const T big = std::numeric_limits<T>::max();
    const int64_t sl = 4 * lcap;
    for (int q = 0; q < ng; ++q) {
        const uint64_t gq = gmask(q);
        const bool in = a && ((gq >> lane) & 1ull);
        const T x = in ? px[s] : big, y = in ? py[s] : big, z = in ? pz[s] : big;
        const T lx = wmin(x, 64), ly = wmin(y, 64), lz = wmin(z, 64);
        const T hx = wmax(in ? x : -big, 64), hy = wmax(in ? y : -big, 64),
                hz = wmax(in ? z : -big, 64);
        const T hm = wmax(in ? h[s] : T(0), 64);
        if (lane == 0) {
            const int64_t slot = 4 * (int64_t)I + q;
            gcnt[slot] = __popcll(m & gq);
            glo[slot] = lx;
            glo[sl + slot] = ly;
            glo[2 * sl + slot] = lz;
            ghi[slot] = hx;
            ghi[sl + slot] = hy;
            ghi[2 * sl + slot] = hz;
            ghm[slot] = hm;
        }
    }
}

// One wavefront per leaf (four per workgroup): grow the leaf box and its
// sub-leaf boxes to the current positions (boxes never shrink; sub-leaf g
// on lanes 16g..16g+15).  Every pair the lists could miss has a particle
// that left its bin: while each leaf box reaches at most d out of its bin
// with 2 d + range <= bin width, the 27-bin stencil still holds every
// partner; a leaf breaking that sets *stale.
template <typename T>
__global__ __launch_bounds__(256) void refit_box_kernel(
    const int32_t *__restrict__ nn_ptr, int64_t lcap,
    const int32_t *__restrict__ lst, const int32_t *__restrict__ lct,
    const int32_t *__restrict__ lkey, const int32_t *__restrict__ lbox,
    const T *__restrict__ p0, const T *__restrict__ p1, const T *__restrict__ p2,
    T *__restrict__ lo, T *__restrict__ hi, int has_sub,
    const int32_t *__restrict__ nsub, const int32_t *__restrict__ sst,
    const int32_t *__restrict__ scnt, T *__restrict__ slo, T *__restrict__ shi,
    int64_t total_bins, const int *__restrict__ ncm,
    const int64_t *__restrict__ bin_base, const double *__restrict__ rc,
    const double *__restrict__ hmax, int *__restrict__ stale) {
    const int64_t nn = *nn_ptr;
    const int lane = threadIdx.x & 63;
    const int64_t I = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (I >= nn) return;  // the whole wavefront leaves together
    const int st = lst[I], c = lct[I];
    T l0 = lo[I], l1 = lo[lcap + I], l2 = lo[2 * lcap + I];
    T u0 = hi[I], u1 = hi[lcap + I], u2 = hi[2 * lcap + I];
    for (int q = st + lane; q < st + c; q += 64) {
        l0 = fmin(l0, p0[q]);
        u0 = fmax(u0, p0[q]);
        l1 = fmin(l1, p1[q]);
        u1 = fmax(u1, p1[q]);
        l2 = fmin(l2, p2[q]);
        u2 = fmax(u2, p2[q]);
    }
    l0 = wmin(l0, 64);
    l1 = wmin(l1, 64);
    l2 = wmin(l2, 64);
    u0 = wmax(u0, 64);
    u1 = wmax(u1, 64);
    u2 = wmax(u2, 64);
    if (lane == 0) {
        lo[I] = l0;
        lo[lcap + I] = l1;
        lo[2 * lcap + I] = l2;
        hi[I] = u0;
        hi[lcap + I] = u1;
        hi[2 * lcap + I] = u2;
        const int key = lkey[I];
        const int64_t gbin = key < total_bins ? key : key - total_bins;
        const int b = lbox[I];
        const int nc = ncm[b];
        const int64_t lb = gbin - bin_base[b];
        const int64_t cc[3] = {lb / ((int64_t)nc * nc), (lb / nc) % nc, lb % nc};
        const double L[3] = {(double)l0, (double)l1, (double)l2};
        const double U[3] = {(double)u0, (double)u1, (double)u2};
        double ov = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double cl = 1.0 + (double)cc[a] / nc;
            const double ch = 1.0 + (double)(cc[a] + 1) / nc;
            ov = fmax(ov, fmax(cl - L[a], U[a] - ch));
        }
        const double R = fmax(rc[b], 2.0 * hmax[b]) * (1.0 + 1e-5);
        if (2.0 * ov * (1.0 + 1e-6) + R > 1.0 / nc) atomicOr(stale, 1);
    }
    if (has_sub) {
        const int g = lane >> 4, u = lane & 15;
        const int ns = nsub[I];
        const int64_t sl = 4 * I + (g < ns ? g : 0);
        const bool v = g < ns && u < scnt[sl];
        const int q = v ? sst[sl] + u : st;
        T a0 = slo[sl], a1 = slo[4 * lcap + sl], a2 = slo[8 * lcap + sl];
        T b0 = shi[sl], b1 = shi[4 * lcap + sl], b2 = shi[8 * lcap + sl];
        if (v) {
            a0 = fmin(a0, p0[q]);
            b0 = fmax(b0, p0[q]);
            a1 = fmin(a1, p1[q]);
            b1 = fmax(b1, p1[q]);
            a2 = fmin(a2, p2[q]);
            b2 = fmax(b2, p2[q]);
        }
        a0 = wmin(a0, 16);
        a1 = wmin(a1, 16);
        a2 = wmin(a2, 16);
        b0 = wmax(b0, 16);
        b1 = wmax(b1, 16);
        b2 = wmax(b2, 16);
        if (u == 0 && g < ns) {
            slo[sl] = a0;
            slo[4 * lcap + sl] = a1;
            slo[8 * lcap + sl] = a2;
            shi[sl] = b0;
            shi[4 * lcap + sl] = b1;
            shi[8 * lcap + sl] = b2;
        }
    }
}

// Block kick: the particles starting (phase 0: s % 2^(L-b) == 0) or ending
// (phase 1: (s + 1) % 2^(L-b) == 0) a step of tau_b = dt / 2^b at substep
// s get v += (a_grav + a_hydro) tau_b / 2 and u += du/dt tau_b / 2; the
// context-precision copies follow.
template <typename T>
__global__ void kick_kernel(int64_t n, double dt, int L, int64_t s, int phase,
                            const int32_t *__restrict__ bins,
                            double *__restrict__ v64, double *__restrict__ u64,
                            const T *__restrict__ g0, const T *__restrict__ g1,
                            const T *__restrict__ g2, const T *__restrict__ h0,
                            const T *__restrict__ h1, const T *__restrict__ h2,
                            const T *__restrict__ dudt, T *__restrict__ v0,
                            T *__restrict__ v1, T *__restrict__ v2,
                            T *__restrict__ u) {
    const T *g[3] = {g0, g1, g2};
    const T *h[3] = {h0, h1, h2};
    T *vo[3] = {v0, v1, v2};
    GRID_LOOP(i, n) {
        int b = bins[i];
        b = b < 0 ? 0 : (b > L ? L : b);
        const int64_t per = (int64_t)1 << (L - b);
        const bool sel = phase == 0 ? (s % per) == 0 : ((s + 1) % per) == 0;
        if (!sel) continue;
        const double half = ldexp(dt, -b) * 0.5;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double acc = (double)g[a][i];
            if (h0) acc += (double)h[a][i];
            const double v = v64[a * n + i] + acc * half;
            v64[a * n + i] = v;
            vo[a][i] = (T)v;
        }
        if (u64) {
            const double uu = u64[i] + (double)dudt[i] * half;
            u64[i] = uu;
            u[i] = (T)uu;
        }
    }
}

// Drift of every particle, x += v delta; wrapped into [1, 2) only when
// wrap is set (inside an interval the tree keeps unwrapped positions).
template <typename T>
__global__ void drift_kernel(int64_t n, double delta, int wrap,
                             double *__restrict__ x64, const double *__restrict__ v64,
                             T *__restrict__ x0, T *__restrict__ x1,
                             T *__restrict__ x2) {
    T *xo[3] = {x0, x1, x2};
    GRID_LOOP(i, n) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double x = x64[a * n + i] + v64[a * n + i] * delta;
            if (wrap) {
                x = x - floor(x - 1.0);
                if (x >= 2.0) x -= 1.0;
            }
            x64[a * n + i] = x;
            T xs = (T)x;
            if (wrap && xs >= T(2)) xs = T(1);  // rounding up to 2 wraps to 1
            xo[a][i] = xs;
        }
    }
}

template <typename T> const T *cp(const void *p) { return static_cast<const T *>(p); }
template <typename T> T *mp(void *p) { return static_cast<T *>(p); }

template <typename T>
int bins_impl(crk_ctx *ctx, int64_t n, double dt, int L, double eps,
              double c_cfl, double eta, const void *const ag[3],
              const void *const ah[3], const void *h, const void *cs,
              int32_t *bins) {
    double r = 2.0 * eta * eps;
    r = r * r;
    hipLaunchKernelGGL((bins_kernel<T>), dim3(grid_n(n)), dim3(256), 0,
                       ctx->stream, n, dt, L, r, c_cfl, cp<T>(ag[0]),
                       cp<T>(ag[1]), cp<T>(ag[2]), ah ? cp<T>(ah[0]) : nullptr,
                       ah ? cp<T>(ah[1]) : nullptr, ah ? cp<T>(ah[2]) : nullptr,
                       cp<T>(h), cp<T>(cs), bins);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

template <typename T>
int refit_impl(crk_ctx *ctx, crk_tree *t, const void *gx, const void *gy,
               const void *gz, const void *dx, const void *dy, const void *dz) {
    hipStream_t s = ctx->stream;
    const int64_t n = t->n;
    // grown leaf boxes need new lists, moved particles new active groups
    // (and the sub-leaf entries, which name groups when those are on)
    t->lists_built = false;
    t->grp_on = false;
    t->slist_on = false;
    hipLaunchKernelGGL((refit_pos_kernel<T>), dim3(grid_n(n)), dim3(256), 0, s,
                       n, t->n_gas, t->perm.as<int32_t>(), cp<T>(gx), cp<T>(gy),
                       cp<T>(gz), cp<T>(dx), cp<T>(dy), cp<T>(dz),
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>());
    CRK_HIP(hipGetLastError());
    CRK_TRY(t->overhang.ensure(4, false));
    CRK_HIP(fill_i32(t->overhang.as<int32_t>(), 0, 1, s));
    const int cur = t->cur_nodes;
    const unsigned nwg = (unsigned)std::max<int64_t>(1, (t->n_leaves + 3) / 4);
    hipLaunchKernelGGL((refit_box_kernel<T>), dim3(nwg), dim3(256),
                       0, s, t->counters.as<int32_t>() + C_NN, t->leaf_cap,
                       t->nd_start[cur].as<int32_t>(), t->nd_count[cur].as<int32_t>(),
                       t->nd_key[cur].as<int32_t>(), t->leaf_box.as<int32_t>(),
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                       t->leaf_lo.as<T>(), t->leaf_hi.as<T>(), t->has_sub ? 1 : 0,
                       t->sub_nsub.as<int32_t>(), t->sub_start.as<int32_t>(),
                       t->sub_count.as<int32_t>(), t->sub_lo.as<T>(),
                       t->sub_hi.as<T>(), t->total_bins, t->d_ncm.as<int>(),
                       t->d_bin_base.as<int64_t>(), t->d_rc.as<double>(),
                       t->d_hmax.as<double>(), t->overhang.as<int>());
    CRK_HIP(hipGetLastError());
    int32_t *hb = ctx->err_host.as<int32_t>() + 12;
    CRK_HIP(hipMemcpyAsync(hb, t->overhang.p, 4, hipMemcpyDeviceToHost, s));
    CRK_HIP(hipStreamSynchronize(s));
    if (*hb)
        return set_error(CRK_ESTALE,
                         "tree_refit: particles moved too far out of their "
                         "chaining-mesh bins for the interaction stencil; "
                         "rebuild the tree");
    return CRK_OK;
}

template <typename T>
int kick_impl(crk_ctx *ctx, int64_t n, double dt, int L, int64_t s, int phase,
              const int32_t *bins, double *v64, double *u64,
              const void *const ag[3], const void *const ah[3], const void *dudt,
              void *const v[3], void *u) {
    hipLaunchKernelGGL((kick_kernel<T>), dim3(grid_n(n)), dim3(256), 0,
                       ctx->stream, n, dt, L, s, phase, bins, v64, u64,
                       cp<T>(ag[0]), cp<T>(ag[1]), cp<T>(ag[2]),
                       ah ? cp<T>(ah[0]) : nullptr, ah ? cp<T>(ah[1]) : nullptr,
                       ah ? cp<T>(ah[2]) : nullptr, cp<T>(dudt), mp<T>(v[0]),
                       mp<T>(v[1]), mp<T>(v[2]), mp<T>(u));
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

template <typename T>
int drift_impl(crk_ctx *ctx, int64_t n, double delta, int wrap, double *x64,
               const double *v64, void *const x[3]) {
    hipLaunchKernelGGL((drift_kernel<T>), dim3(grid_n(n)), dim3(256), 0,
                       ctx->stream, n, delta, wrap, x64, v64, mp<T>(x[0]),
                       mp<T>(x[1]), mp<T>(x[2]));
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

}  // namespace

int timestep_bins(crk_ctx *ctx, int64_t n, double dt, int max_level, double eps,
                  double c_cfl, double eta, const void *const a_grav[3],
                  const void *const a_hydro[3], const void *h, const void *cs,
                  int32_t *bins) {
    if (n == 0) return CRK_OK;
    if (ctx->precision == CRK_FP64)
        return bins_impl<double>(ctx, n, dt, max_level, eps, c_cfl, eta, a_grav,
                                 a_hydro, h, cs, bins);
    return bins_impl<float>(ctx, n, dt, max_level, eps, c_cfl, eta, a_grav,
                            a_hydro, h, cs, bins);
}

template <typename T> int act_groups(crk_ctx *ctx, crk_tree *t) {
    const int64_t lcap = t->leaf_cap, sl = 4 * lcap;
    CRK_TRY(t->grp_nsub.ensure((size_t)(lcap + 1) * 4, false));
    CRK_TRY(t->grp_cnt.ensure((size_t)sl * 4, false));
    CRK_TRY(t->grp_idx.ensure((size_t)sl * 16 * 4, false));
    CRK_TRY(t->grp_lo.ensure((size_t)3 * sl * sizeof(T), false));
    CRK_TRY(t->grp_hi.ensure((size_t)3 * sl * sizeof(T), false));
    CRK_TRY(t->grp_hmax.ensure((size_t)sl * sizeof(T), false));
    const int cur = t->cur_nodes;
    hipLaunchKernelGGL((act_groups_kernel<T>), dim3((unsigned)t->act_nall),
                       dim3(64), 0, ctx->stream, t->act_items.as<int32_t>(),
                       t->act_nall, t->nd_start[cur].as<int32_t>(),
                       t->nd_count[cur].as<int32_t>(), t->sub_nsub.as<int32_t>(),
                       t->sub_start.as<int32_t>(), t->sub_count.as<int32_t>(),
                       t->act_flags.as<uint8_t>(),
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                       t->hsm.as<T>(), lcap, t->grp_nsub.as<int32_t>(),
                       t->grp_cnt.as<int32_t>(), t->grp_idx.as<int32_t>(),
                       t->grp_lo.as<T>(), t->grp_hi.as<T>(), t->grp_hmax.as<T>());
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

// the sub-leaf entries of the active subset (act_count[4], [5]: their
// counts, all and gas; left at 0 by the caller for an empty subset)
int act_sublist(crk_ctx *ctx, crk_tree *t) {
    const int64_t lcap = t->leaf_cap, na = t->act_nall;
    hipStream_t s = ctx->stream;
    CRK_TRY(t->act_sub.ensure((size_t)3 * (lcap + 1) * 4, false));
    CRK_TRY(t->act_slist.ensure((size_t)4 * lcap * 4, false));
    int32_t *mask = t->act_sub.as<int32_t>();
    int32_t *count = mask + (lcap + 1);
    int32_t *off = count + (lcap + 1);
    int32_t *cnt = t->act_count.as<int32_t>();
    const int cur = t->cur_nodes;
    hipLaunchKernelGGL(act_submask_kernel, dim3((unsigned)na), dim3(64), 0, s,
                       t->act_items.as<int32_t>(), na,
                       t->nd_start[cur].as<int32_t>(), t->nd_count[cur].as<int32_t>(),
                       t->sub_nsub.as<int32_t>(), t->sub_start.as<int32_t>(),
                       t->sub_count.as<int32_t>(), t->act_flags.as<uint8_t>(),
                       mask, count);
    CRK_HIP(hipGetLastError());
    CRK_HIP(exclusive_scan_i32(count, off, na, cnt + 4, ctx->scratch.p, s));
    hipLaunchKernelGGL(act_sublist_kernel, dim3(grid_n(na + 1)), dim3(256), 0, s,
                       t->act_items.as<int32_t>(), na, t->act_ngas, mask, off,
                       t->grp_on ? 1 : 0, t->act_slist.as<int32_t>(), cnt);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

int tree_set_active(crk_ctx *ctx, crk_tree *t, const int32_t *bins_gas,
                    const int32_t *bins_dm, int max_level, int64_t substep) {
    hipStream_t s = ctx->stream;
    // lists belong to one subset: the next passes need a list build
    t->lists_built = false;
    t->act_substep = substep < 0 ? -1 : substep;
    t->act_level = max_level;
    t->grp_on = false;
    t->slist_on = false;
    if (substep < 0) {
        t->act_on = false;
        return CRK_OK;
    }
    const int64_t n = t->n, lcap = t->leaf_cap;
    CRK_TRY(t->act_flags.ensure((size_t)std::max<int64_t>(n, 1), false));
    CRK_TRY(t->act_leaf.ensure((size_t)(lcap + 1) * 2 * 4, false));
    CRK_TRY(t->act_items.ensure((size_t)(lcap + 1) * 4, false));
    CRK_TRY(t->act_count.ensure(8 * 4, false));
    CRK_TRY(ctx->scratch.ensure(scan_tmp_bytes(lcap + 1), false));
    // cnt: {active leaves, active gas leaves, scan total, active slots}
    int32_t *cnt = t->act_count.as<int32_t>();
    CRK_HIP(hipMemsetAsync(cnt + 3, 0, 3 * 4, s));
    hipLaunchKernelGGL(act_flags_kernel, dim3(grid_n(n)), dim3(256), 0, s, n,
                       t->n_gas, t->perm.as<int32_t>(), bins_gas, bins_dm,
                       max_level, substep, t->act_flags.as<uint8_t>(), cnt + 3);
    CRK_HIP(hipGetLastError());
    const int cur = t->cur_nodes;
    int32_t *flag = t->act_leaf.as<int32_t>();
    int32_t *pos = flag + (lcap + 1);
    hipLaunchKernelGGL(act_leaf_kernel, dim3(grid_n(lcap)), dim3(256), 0, s,
                       t->counters.as<int32_t>() + C_NN, lcap,
                       t->nd_start[cur].as<int32_t>(), t->nd_count[cur].as<int32_t>(),
                       t->act_flags.as<uint8_t>(), flag);
    CRK_HIP(hipGetLastError());
    CRK_HIP(exclusive_scan_i32(flag, pos, lcap, cnt + 2, ctx->scratch.p, s));
    hipLaunchKernelGGL(act_items_kernel, dim3(grid_n(lcap)), dim3(256), 0, s,
                       t->counters.as<int32_t>() + C_NN, lcap, flag, pos,
                       t->act_items.as<int32_t>());
    CRK_HIP(hipGetLastError());
    hipLaunchKernelGGL(act_count_kernel, dim3(1), dim3(1), 0, s,
                       t->counters.as<int32_t>() + C_NN,
                       t->bin_leaf.as<int32_t>() + t->total_bins, pos, cnt + 2, cnt);
    CRK_HIP(hipGetLastError());
    int32_t hc[4];
    CRK_HIP(hipMemcpyAsync(hc, cnt, 16, hipMemcpyDeviceToHost, s));
    CRK_HIP(hipStreamSynchronize(s));
    t->act_nall = hc[0];
    t->act_ngas = hc[1];
    t->act_npart = hc[3];
    t->act_on = true;
    t->grp_on = false;
    // groups when the active leaves hold at least k active particles each
    // on average (k = 1: always; 0: never)
    const int64_t k = ctx->tuning.act_groups;
    if (t->has_sub && k > 0 && t->act_nall > 0 && t->act_npart >= k * t->act_nall) {
        if (ctx->precision == CRK_FP64) CRK_TRY(act_groups<double>(ctx, t));
        else CRK_TRY(act_groups<float>(ctx, t));
        t->grp_on = true;
    }
    if (t->has_sub && t->act_nall > 0) CRK_TRY(act_sublist(ctx, t));
    t->slist_on = t->has_sub;
    return CRK_OK;
}

int tree_refit(crk_ctx *ctx, crk_tree *t, const void *gx, const void *gy,
               const void *gz, const void *dx, const void *dy, const void *dz) {
    if (ctx->precision == CRK_FP64)
        return refit_impl<double>(ctx, t, gx, gy, gz, dx, dy, dz);
    return refit_impl<float>(ctx, t, gx, gy, gz, dx, dy, dz);
}

int block_kick(crk_ctx *ctx, int64_t n, double dt, int max_level, int64_t substep,
               int phase, const int32_t *bins, double *v64, double *u64,
               const void *const a_grav[3], const void *const a_hydro[3],
               const void *dudt, void *const v[3], void *u) {
    if (n == 0) return CRK_OK;
    if (ctx->precision == CRK_FP64)
        return kick_impl<double>(ctx, n, dt, max_level, substep, phase, bins, v64,
                                 u64, a_grav, a_hydro, dudt, v, u);
    return kick_impl<float>(ctx, n, dt, max_level, substep, phase, bins, v64, u64,
                            a_grav, a_hydro, dudt, v, u);
}

int drift(crk_ctx *ctx, int64_t n, double delta, int wrap, double *x64,
          const double *v64, void *const x[3]) {
    if (n == 0) return CRK_OK;
    if (ctx->precision == CRK_FP64)
        return drift_impl<double>(ctx, n, delta, wrap, x64, v64, x);
    return drift_impl<float>(ctx, n, delta, wrap, x64, v64, x);
}

}  // namespace crk
