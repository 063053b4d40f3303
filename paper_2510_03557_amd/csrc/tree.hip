// build_tree: chaining-mesh bins and per-bin k-d base leaves (Sec. IV-B.1).
//
// Device-side algorithm (all boxes and both species at once):
//  1. key per particle = (species, box, bin) and its coordinate along one
//     axis; three stable radix sorts give, for each axis a, the particles
//     ordered by (bin, coordinate_a, caller index) -- the arrays S_a.
//  2. every non-empty (species, bin) segment is a k-d node.  A level splits
//     each node holding more than leaf_max particles along its widest
//     extent, at the quantile that gives the left side ceil(k/2) of the k
//     leaves the node needs (the median when k is even), so leaves end up
//     nearly full.  The extent is O(1) from the axis-sorted arrays (first
//     and last element); the left half is the first ceil(c/2) elements of
//     S_axis, and all three arrays are partitioned stably with one prefix
//     sum each, so every array stays sorted inside every node.  A level
//     always rewrites its outputs (identity where nothing splits), so the
//     same launch sequence is valid inside a captured graph.
//  3. the final nodes are the leaves (only base leaves are kept); their
//     bounding boxes come from the sorted arrays, h_max from a reduction,
//     and a (species, bin) -> first-leaf table from a count + prefix sum.
// Positions and h are copied to tree order; S_0 gives the tree permutation.
#include <algorithm>
#include <cmath>

#include "crk_internal.h"

namespace crk {

namespace {

constexpr int TB = 256;

inline unsigned grid_for(int64_t n, int per = TB) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 1048576) g = 1048576;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n)                                                     \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// Order-preserving 23-bit coordinate key of a value in [1, 2).
__device__ inline uint32_t coord_bits(float x) {
    return __float_as_uint(x) & 0x7FFFFFu;
}
__device__ inline uint32_t coord_bits(double x) {
    return (uint32_t)((__double_as_longlong(x) >> 29) & 0x7FFFFFll);
}

// largest b with off[b] <= i (so empty boxes are skipped)
__device__ inline int find_box(const int64_t *off, int nb, int64_t i) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Combined caller index c: gas particles 0..n_gas-1, then dm particles.
template <typename T>
__global__ void keys_kernel(const T *__restrict__ gx, const T *__restrict__ gy,
                            const T *__restrict__ gz, const T *__restrict__ gh,
                            const T *__restrict__ dx, const T *__restrict__ dy,
                            const T *__restrict__ dz, int64_t n_gas, int64_t n,
                            int nb, const int64_t *__restrict__ gas_off,
                            const int64_t *__restrict__ dm_off,
                            const int *__restrict__ ncm,
                            const int64_t *__restrict__ bin_base,
                            const double *__restrict__ hmax,
                            int64_t total_bins, int axis, int first,
                            T *__restrict__ px, T *__restrict__ py,
                            T *__restrict__ pz, T *__restrict__ ph,
                            uint64_t *__restrict__ kout,
                            int32_t *__restrict__ vout, int *__restrict__ err) {
    GRID_STRIDE(c, n) {
        const bool gas = c < n_gas;
        const int64_t li = gas ? c : c - n_gas;
        T x = gas ? gx[li] : dx[li];
        T y = gas ? gy[li] : dy[li];
        T z = gas ? gz[li] : dz[li];
        const int b = find_box(gas ? gas_off : dm_off, nb, li);
        const int nc = ncm[b];
        bool bad = !(x >= T(1) && x < T(2)) || !(y >= T(1) && y < T(2)) ||
                   !(z >= T(1) && z < T(2));
        T h = T(0);
        if (gas) {
            h = gh[li];
            if (!(h > T(0)) || !(h < T(1))) bad = true;
            else if (first && (double)h > hmax[b]) atomicOr(err, DEV_ERR_HMAX);
        }
        if (bad) {
            if (first) atomicOr(err, DEV_ERR_INPUT);
            x = T(1);
            y = T(1);
            z = T(1);
            h = T(0);
        }
        int cx = min(max((int)((x - T(1)) * T(nc)), 0), nc - 1);
        int cy = min(max((int)((y - T(1)) * T(nc)), 0), nc - 1);
        int cz = min(max((int)((z - T(1)) * T(nc)), 0), nc - 1);
        int64_t gbin = bin_base[b] + ((int64_t)cx * nc + cy) * nc + cz;
        uint64_t bk = (uint64_t)((gas ? 0 : total_bins) + gbin);
        if (first) {
            px[c] = x;
            py[c] = y;
            pz[c] = z;
            ph[c] = h;
        }
        T v = axis == 0 ? x : (axis == 1 ? y : z);
        kout[c] = (bk << 23) | coord_bits(v);
        vout[c] = (int32_t)c;
    }
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ a,
                                int32_t *__restrict__ b, int64_t n) {
    GRID_STRIDE(i, n) b[i] = a[i];
}

__global__ void seg_flags_kernel(const uint64_t *__restrict__ k, int64_t n,
                                 int32_t *__restrict__ flags,
                                 int32_t *__restrict__ binkey) {
    GRID_STRIDE(p, n) {
        uint32_t bk = (uint32_t)(k[p] >> 23);
        binkey[p] = (int32_t)bk;
        flags[p] = (p == 0 || (uint32_t)(k[p - 1] >> 23) != bk) ? 1 : 0;
    }
}

__global__ void seg_nodes_kernel(const int32_t *__restrict__ flags,
                                 const int32_t *__restrict__ sf,
                                 const int32_t *__restrict__ binkey, int64_t n,
                                 int32_t *__restrict__ nd_start,
                                 int32_t *__restrict__ nd_key,
                                 int32_t *__restrict__ elem_node) {
    GRID_STRIDE(p, n) {
        int node = sf[p] + flags[p] - 1;
        elem_node[p] = node;
        if (flags[p]) {
            nd_start[node] = (int32_t)p;
            nd_key[node] = binkey[p];
        }
    }
}

__global__ void node_counts_kernel(const int32_t *__restrict__ nd_start,
                                   const int32_t *__restrict__ nn_ptr,
                                   int64_t cap, int64_t n,
                                   int32_t *__restrict__ nd_count) {
    const int64_t nn = *nn_ptr;
    GRID_STRIDE(k, cap) {
        if (k >= nn) break;
        int64_t end = (k + 1 < nn) ? nd_start[k + 1] : n;
        nd_count[k] = (int32_t)(end - nd_start[k]);
    }
}

// Decide the split of every node: axis of widest extent (ties: lowest
// axis); the left part takes ceil(k/2) of the node's k leaves.  On the last
// level of a captured
// sequence a node that still needs a split raises the capacity error.
template <typename T>
__global__ void kd_plan_kernel(
    const int32_t *__restrict__ nd_start, const int32_t *__restrict__ nd_count,
    const int32_t *__restrict__ nn_ptr, int64_t cap, int L, int last,
    const int32_t *__restrict__ S0, const int32_t *__restrict__ S1,
    const int32_t *__restrict__ S2, const T *__restrict__ px,
    const T *__restrict__ py, const T *__restrict__ pz,
    int32_t *__restrict__ split, int32_t *__restrict__ left,
    int32_t *__restrict__ axis, int32_t *__restrict__ nchild,
    int32_t *__restrict__ any_split, int *__restrict__ err) {
    const int64_t nn = *nn_ptr;
    GRID_STRIDE(k, cap) {
        if (k >= nn) {
            nchild[k] = 0;
            continue;
        }
        const int st = nd_start[k];
        const int cnt = nd_count[k];
        int s = 0;
        if (cnt > L) {
            if (last) {
                atomicOr(err, DEV_ERR_CAPACITY);
            } else {
                const int e = st + cnt - 1;
                T ex = px[S0[e]] - px[S0[st]];
                T ey = py[S1[e]] - py[S1[st]];
                T ez = pz[S2[e]] - pz[S2[st]];
                int a = 0;
                T best = ex;
                if (ey > best) {
                    a = 1;
                    best = ey;
                }
                if (ez > best) a = 2;
                axis[k] = a;
                // the node needs nl = ceil(cnt / L) leaves; the left part
                // takes ceil(nl / 2) of them, in proportion (the median when
                // nl is even), so that leaves come out nearly full
                const int nl = (cnt + L - 1) / L;
                const int nleft = (nl + 1) / 2;
                left[k] = (int)(((long long)cnt * nleft + nl / 2) / nl);
                s = 1;
                *any_split = 1;
            }
        }
        split[k] = s;
        nchild[k] = s ? 2 : 1;
    }
}

__global__ void kd_flag_kernel(const int32_t *__restrict__ elem_node,
                               const int32_t *__restrict__ nd_start,
                               const int32_t *__restrict__ split,
                               const int32_t *__restrict__ left,
                               const int32_t *__restrict__ axis,
                               const int32_t *__restrict__ S0,
                               const int32_t *__restrict__ S1,
                               const int32_t *__restrict__ S2, int64_t n,
                               const int32_t *__restrict__ nn_next, int64_t cap,
                               int32_t *__restrict__ flag_c) {
    if (*nn_next > cap) return;  // overflowing level: nothing splits
    GRID_STRIDE(p, n) {
        int k = elem_node[p];
        if (split[k]) {
            int a = axis[k];
            const int32_t *S = a == 0 ? S0 : (a == 1 ? S1 : S2);
            flag_c[S[p]] = (p - nd_start[k] < left[k]) ? 1 : 0;
        }
    }
}

__global__ void kd_part_flags_kernel(const int32_t *__restrict__ elem_node,
                                     const int32_t *__restrict__ split,
                                     const int32_t *__restrict__ S,
                                     const int32_t *__restrict__ flag_c,
                                     int64_t n,
                                     const int32_t *__restrict__ nn_next,
                                     int64_t cap, int32_t *__restrict__ f) {
    const bool ovf = *nn_next > cap;
    GRID_STRIDE(p, n) f[p] = (split[elem_node[p]] && !ovf) ? flag_c[S[p]] : 1;
}

__global__ void kd_part_scatter_kernel(
    const int32_t *__restrict__ elem_node, const int32_t *__restrict__ nd_start,
    const int32_t *__restrict__ nd_count, const int32_t *__restrict__ split,
    const int32_t *__restrict__ left, const int32_t *__restrict__ f,
    const int32_t *__restrict__ sf, const int32_t *__restrict__ S, int64_t n,
    const int32_t *__restrict__ nn_next, int64_t cap,
    int32_t *__restrict__ Snew) {
    const bool ovf = *nn_next > cap;
    GRID_STRIDE(p, n) {
        int k = elem_node[p];
        int st = nd_start[k];
        int lc = (split[k] && !ovf) ? left[k] : nd_count[k];
        int rl = sf[p] - sf[st];
        int np = f[p] ? st + rl : st + lc + ((int)p - st - rl);
        Snew[np] = S[p];
    }
}

__global__ void kd_children_kernel(
    const int32_t *__restrict__ nd_start, const int32_t *__restrict__ nd_count,
    const int32_t *__restrict__ nd_key, const int32_t *__restrict__ split,
    const int32_t *__restrict__ left, const int32_t *__restrict__ child,
    const int32_t *__restrict__ nn_ptr, const int32_t *__restrict__ nn_next,
    int64_t cap, int32_t *__restrict__ ns, int32_t *__restrict__ nc,
    int32_t *__restrict__ nkey) {
    const int64_t nn = *nn_ptr;
    const bool ovf = *nn_next > cap;
    GRID_STRIDE(k, cap) {
        if (k >= nn) break;
        int cb = ovf ? (int)k : child[k];
        int st = nd_start[k], cnt = nd_count[k], key = nd_key[k];
        if (split[k] && !ovf) {
            int l = left[k];
            ns[cb] = st;
            nc[cb] = l;
            nkey[cb] = key;
            ns[cb + 1] = st + l;
            nc[cb + 1] = cnt - l;
            nkey[cb + 1] = key;
        } else {
            ns[cb] = st;
            nc[cb] = cnt;
            nkey[cb] = key;
        }
    }
}

__global__ void kd_elem_node_kernel(const int32_t *__restrict__ elem_node,
                                    const int32_t *__restrict__ nd_start,
                                    const int32_t *__restrict__ split,
                                    const int32_t *__restrict__ left,
                                    const int32_t *__restrict__ child,
                                    int64_t n,
                                    const int32_t *__restrict__ nn_next,
                                    int64_t cap, int32_t *__restrict__ out) {
    const bool ovf = *nn_next > cap;
    GRID_STRIDE(p, n) {
        int k = elem_node[p];
        if (ovf) {
            out[p] = k;
            continue;
        }
        int cb = child[k];
        out[p] = cb + ((split[k] && (int)p - nd_start[k] >= left[k]) ? 1 : 0);
    }
}

// node count of the next level; a level that would exceed the node
// capacity was run as an identity level and raises the capacity error
__global__ void next_count_kernel(const int32_t *__restrict__ nn_next,
                                  int64_t cap, int32_t *__restrict__ nn,
                                  int *__restrict__ err) {
    if (*nn_next > cap) atomicOr(err, DEV_ERR_CAPACITY);
    else *nn = *nn_next;
}

template <typename T>
__global__ void gather_tree_kernel(const int32_t *__restrict__ S0,
                                   const T *__restrict__ px,
                                   const T *__restrict__ py,
                                   const T *__restrict__ pz,
                                   const T *__restrict__ ph, int64_t n,
                                   int32_t *__restrict__ perm,
                                   T *__restrict__ tx, T *__restrict__ ty,
                                   T *__restrict__ tz, T *__restrict__ th) {
    GRID_STRIDE(p, n) {
        int c = S0[p];
        perm[p] = c;
        tx[p] = px[c];
        ty[p] = py[c];
        tz[p] = pz[c];
        th[p] = ph[c];
    }
}

template <typename T>
__global__ void leaves_kernel(
    const int32_t *__restrict__ nd_start, const int32_t *__restrict__ nd_count,
    const int32_t *__restrict__ nd_key, const int32_t *__restrict__ nn_ptr,
    int64_t cap, const int32_t *__restrict__ S0, const int32_t *__restrict__ S1,
    const int32_t *__restrict__ S2, const T *__restrict__ px,
    const T *__restrict__ py, const T *__restrict__ pz,
    const T *__restrict__ th, int64_t total_bins, int nb,
    const int64_t *__restrict__ bin_base, int32_t *__restrict__ leaf_box,
    T *__restrict__ lo, T *__restrict__ hi, T *__restrict__ lhmax,
    int32_t *__restrict__ bin_cnt) {
    const int64_t nn = *nn_ptr;
    GRID_STRIDE(k, cap) {
        if (k >= nn) break;
        int st = nd_start[k], cnt = nd_count[k], key = nd_key[k];
        int e = st + cnt - 1;
        int64_t gbin = key >= total_bins ? key - total_bins : key;
        leaf_box[k] = find_box(bin_base, nb, gbin);
        lo[k] = px[S0[st]];
        hi[k] = px[S0[e]];
        lo[cap + k] = py[S1[st]];
        hi[cap + k] = py[S1[e]];
        lo[2 * cap + k] = pz[S2[st]];
        hi[2 * cap + k] = pz[S2[e]];
        T hm = T(0);
        for (int p = st; p <= e; ++p) hm = th[p] > hm ? th[p] : hm;
        lhmax[k] = hm;
        atomicAdd(&bin_cnt[key], 1);
    }
}

int ensure_all(crk_tree *t, int64_t n, int64_t leaf_cap, size_t elem,
               int64_t total_bins, bool cap) {
    size_t n1 = (size_t)std::max<int64_t>(n, 1);
    size_t l1 = (size_t)std::max<int64_t>(leaf_cap, 1) + 1;
    for (int i = 0; i < 2; ++i) {
        CRK_TRY(t->keys[i].ensure(n1 * 8, cap));
        CRK_TRY(t->vals[i].ensure(n1 * 4, cap));
    }
    for (int a = 0; a < 3; ++a) {
        CRK_TRY(t->S[a].ensure(n1 * 4, cap));
        CRK_TRY(t->S2[a].ensure(n1 * 4, cap));
        CRK_TRY(t->pos[a].ensure(n1 * elem, cap));
    }
    CRK_TRY(t->hsm.ensure(n1 * elem, cap));
    CRK_TRY(t->binkey.ensure(n1 * 4, cap));
    CRK_TRY(t->flag_c.ensure(n1 * 4, cap));
    CRK_TRY(t->f_pos.ensure(n1 * 4, cap));
    CRK_TRY(t->f_scan.ensure(n1 * 4, cap));
    CRK_TRY(t->elem_node.ensure(n1 * 4, cap));
    CRK_TRY(t->elem_node2.ensure(n1 * 4, cap));
    CRK_TRY(t->perm.ensure(n1 * 4, cap));
    // caller-order combined positions and h live in pass-field slots 0..3
    for (int a = 0; a < 4; ++a) CRK_TRY(t->pf[a].ensure(n1 * elem, cap));
    for (int i = 0; i < 2; ++i) {
        CRK_TRY(t->nd_start[i].ensure(l1 * 4, cap));
        CRK_TRY(t->nd_count[i].ensure(l1 * 4, cap));
        CRK_TRY(t->nd_key[i].ensure(l1 * 4, cap));
    }
    CRK_TRY(t->nd_split.ensure(l1 * 4, cap));
    CRK_TRY(t->nd_left.ensure(l1 * 4, cap));
    CRK_TRY(t->nd_axis.ensure(l1 * 4, cap));
    CRK_TRY(t->nd_child.ensure(l1 * 4, cap));
    CRK_TRY(t->nd_nchild.ensure(l1 * 4, cap));
    CRK_TRY(t->counters.ensure(64 * 8, cap));
    CRK_TRY(t->leaf_box.ensure(l1 * 4, cap));
    CRK_TRY(t->leaf_lo.ensure(3 * l1 * elem, cap));
    CRK_TRY(t->leaf_hi.ensure(3 * l1 * elem, cap));
    CRK_TRY(t->leaf_hmax.ensure(l1 * elem, cap));
    CRK_TRY(t->bin_leaf.ensure((size_t)(2 * total_bins + 2) * 4, cap));
    CRK_TRY(t->bin_cnt.ensure((size_t)(2 * total_bins + 2) * 4, cap));
    return CRK_OK;
}

template <typename T>
int build_impl(crk_ctx *ctx, crk_tree *t, const void *gx_, const void *gy_,
               const void *gz_, const void *gh_, const void *dx_,
               const void *dy_, const void *dz_) {
    const T *gx = static_cast<const T *>(gx_), *gy = static_cast<const T *>(gy_),
            *gz = static_cast<const T *>(gz_), *gh = static_cast<const T *>(gh_);
    const T *dx = static_cast<const T *>(dx_), *dy = static_cast<const T *>(dy_),
            *dz = static_cast<const T *>(dz_);
    hipStream_t s = ctx->stream;
    const bool cap = ctx->capturing;
    const int64_t n = t->n;
    const int64_t lcap = t->leaf_cap;
    int *err = dev_err_word(ctx);
    int32_t *cnt = t->counters.as<int32_t>();
    T *px = t->pf[0].as<T>(), *py = t->pf[1].as<T>(), *pz = t->pf[2].as<T>(),
      *ph = t->pf[3].as<T>();
    uint64_t *K[2] = {t->keys[0].as<uint64_t>(), t->keys[1].as<uint64_t>()};
    int32_t *Vv[2] = {t->vals[0].as<int32_t>(), t->vals[1].as<int32_t>()};
    int32_t *S[3] = {t->S[0].as<int32_t>(), t->S[1].as<int32_t>(),
                     t->S[2].as<int32_t>()};
    int32_t *Sn[3] = {t->S2[0].as<int32_t>(), t->S2[1].as<int32_t>(),
                      t->S2[2].as<int32_t>()};
    int32_t *flags = t->f_pos.as<int32_t>();
    int32_t *sf = t->f_scan.as<int32_t>();
    const int key_bits = 23 + t->bin_bits;

    // 1. one stable sort per axis by (bin key, coordinate), caller index as
    //    the tie-break (input order)
    for (int a = 0; a < 3; ++a) {
        hipLaunchKernelGGL((keys_kernel<T>), dim3(grid_for(n)), dim3(TB), 0, s,
                           gx, gy, gz, gh, dx, dy, dz, t->n_gas, n, t->n_boxes,
                           t->d_gas_off.as<int64_t>(), t->d_dm_off.as<int64_t>(),
                           t->d_ncm.as<int>(), t->d_bin_base.as<int64_t>(),
                           t->d_hmax.as<double>(), t->total_bins, a,
                           a == 0 ? 1 : 0, px, py, pz, ph, K[0], Vv[0], err);
        CRK_HIP(hipGetLastError());
        hipError_t he;
        int r = radix_sort_u64_i32(K, Vv, n, key_bits, ctx->scratch.p, s, &he);
        CRK_HIP(he);
        hipLaunchKernelGGL(copy_i32_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                           Vv[r], S[a], n);
        CRK_HIP(hipGetLastError());
        if (a == 0) {
            // 2. segments of equal (species, bin) are the initial k-d nodes
            hipLaunchKernelGGL(seg_flags_kernel, dim3(grid_for(n)), dim3(TB), 0,
                               s, K[r], n, flags, t->binkey.as<int32_t>());
            CRK_HIP(hipGetLastError());
        }
    }
    CRK_HIP(exclusive_scan_i32(flags, sf, n, cnt + C_NN, ctx->scratch.p, s));
    int cur = 0;
    int32_t *en = t->elem_node.as<int32_t>();
    int32_t *en2 = t->elem_node2.as<int32_t>();
    hipLaunchKernelGGL(seg_nodes_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                       flags, sf, t->binkey.as<int32_t>(), n,
                       t->nd_start[cur].as<int32_t>(),
                       t->nd_key[cur].as<int32_t>(), en);
    CRK_HIP(hipGetLastError());
    hipLaunchKernelGGL(node_counts_kernel, dim3(grid_for(lcap)), dim3(TB), 0, s,
                       t->nd_start[cur].as<int32_t>(), cnt + C_NN, lcap, n,
                       t->nd_count[cur].as<int32_t>());
    CRK_HIP(hipGetLastError());

    // 3. k-d levels
    const int max_levels = cap ? t->kd_levels + 2 : 64;
    int levels_run = 0;
    for (int lev = 0; lev < max_levels; ++lev) {
        const int last = (cap && lev == max_levels - 1) ? 1 : 0;
        int32_t *ns = t->nd_start[cur].as<int32_t>();
        int32_t *nc = t->nd_count[cur].as<int32_t>();
        int32_t *nk = t->nd_key[cur].as<int32_t>();
        CRK_HIP(fill_i32(cnt + C_ANY, 0, 1, s));
        hipLaunchKernelGGL((kd_plan_kernel<T>), dim3(grid_for(lcap)), dim3(TB), 0,
                           s, ns, nc, cnt + C_NN, lcap, t->leaf_max, last, S[0],
                           S[1], S[2], px, py, pz, t->nd_split.as<int32_t>(),
                           t->nd_left.as<int32_t>(), t->nd_axis.as<int32_t>(),
                           t->nd_nchild.as<int32_t>(), cnt + C_ANY, err);
        CRK_HIP(hipGetLastError());
        if (last) break;
        if (!cap) {
            int32_t *hb = ctx->err_host.as<int32_t>() + 8;
            CRK_HIP(hipMemcpyAsync(hb, cnt + C_ANY, 4, hipMemcpyDeviceToHost, s));
            CRK_HIP(hipStreamSynchronize(s));
            if (*hb == 0) break;
        }
        ++levels_run;
        CRK_HIP(exclusive_scan_i32(t->nd_nchild.as<int32_t>(),
                                   t->nd_child.as<int32_t>(), lcap,
                                   cnt + C_NN_NEXT, ctx->scratch.p, s));
        hipLaunchKernelGGL(kd_flag_kernel, dim3(grid_for(n)), dim3(TB), 0, s, en,
                           ns, t->nd_split.as<int32_t>(),
                           t->nd_left.as<int32_t>(), t->nd_axis.as<int32_t>(),
                           S[0], S[1], S[2], n, cnt + C_NN_NEXT, lcap,
                           t->flag_c.as<int32_t>());
        CRK_HIP(hipGetLastError());
        for (int a = 0; a < 3; ++a) {
            hipLaunchKernelGGL(kd_part_flags_kernel, dim3(grid_for(n)), dim3(TB),
                               0, s, en, t->nd_split.as<int32_t>(), S[a],
                               t->flag_c.as<int32_t>(), n, cnt + C_NN_NEXT,
                               lcap, flags);
            CRK_HIP(hipGetLastError());
            CRK_HIP(exclusive_scan_i32(flags, sf, n, nullptr, ctx->scratch.p, s));
            hipLaunchKernelGGL(kd_part_scatter_kernel, dim3(grid_for(n)),
                               dim3(TB), 0, s, en, ns, nc,
                               t->nd_split.as<int32_t>(),
                               t->nd_left.as<int32_t>(), flags, sf, S[a], n,
                               cnt + C_NN_NEXT, lcap, Sn[a]);
            CRK_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(kd_children_kernel, dim3(grid_for(lcap)), dim3(TB), 0,
                           s, ns, nc, nk, t->nd_split.as<int32_t>(),
                           t->nd_left.as<int32_t>(), t->nd_child.as<int32_t>(),
                           cnt + C_NN, cnt + C_NN_NEXT, lcap,
                           t->nd_start[cur ^ 1].as<int32_t>(),
                           t->nd_count[cur ^ 1].as<int32_t>(),
                           t->nd_key[cur ^ 1].as<int32_t>());
        CRK_HIP(hipGetLastError());
        hipLaunchKernelGGL(kd_elem_node_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                           en, ns, t->nd_split.as<int32_t>(),
                           t->nd_left.as<int32_t>(), t->nd_child.as<int32_t>(),
                           n, cnt + C_NN_NEXT, lcap, en2);
        CRK_HIP(hipGetLastError());
        hipLaunchKernelGGL(next_count_kernel, dim3(1), dim3(1), 0, s,
                           cnt + C_NN_NEXT, lcap, cnt + C_NN, err);
        CRK_HIP(hipGetLastError());
        for (int a = 0; a < 3; ++a) std::swap(S[a], Sn[a]);
        std::swap(en, en2);
        cur ^= 1;
    }
    if (!cap) t->kd_levels = levels_run;
    // remember which buffers hold the final state
    t->cur_nodes = cur;
    for (int a = 0; a < 3; ++a) t->S_final[a] = S[a];

    // 4. tree order, leaves, bin -> leaf table
    const int64_t nbin2 = 2 * t->total_bins;
    hipLaunchKernelGGL((gather_tree_kernel<T>), dim3(grid_for(n)), dim3(TB), 0, s,
                       S[0], px, py, pz, ph, n, t->perm.as<int32_t>(),
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                       t->hsm.as<T>());
    CRK_HIP(hipGetLastError());
    CRK_HIP(fill_i32(t->bin_cnt.as<int32_t>(), 0, nbin2 + 1, s));
    hipLaunchKernelGGL((leaves_kernel<T>), dim3(grid_for(lcap)), dim3(TB), 0, s,
                       t->nd_start[cur].as<int32_t>(),
                       t->nd_count[cur].as<int32_t>(),
                       t->nd_key[cur].as<int32_t>(), cnt + C_NN, lcap, S[0], S[1],
                       S[2], px, py, pz, t->hsm.as<T>(), t->total_bins,
                       t->n_boxes, t->d_bin_base.as<int64_t>(),
                       t->leaf_box.as<int32_t>(), t->leaf_lo.as<T>(),
                       t->leaf_hi.as<T>(), t->leaf_hmax.as<T>(),
                       t->bin_cnt.as<int32_t>());
    CRK_HIP(hipGetLastError());
    CRK_HIP(exclusive_scan_i32(t->bin_cnt.as<int32_t>(),
                               t->bin_leaf.as<int32_t>(), nbin2 + 1, nullptr,
                               ctx->scratch.p, s));
    if (!cap) {
        // sizes for the host: leaves, gas leaves
        int32_t *hb = ctx->err_host.as<int32_t>() + 8;
        CRK_HIP(hipMemcpyAsync(hb, cnt + C_NN, 4, hipMemcpyDeviceToHost, s));
        CRK_HIP(hipMemcpyAsync(hb + 1, t->bin_leaf.as<int32_t>() + t->total_bins,
                               4, hipMemcpyDeviceToHost, s));
        CRK_HIP(hipStreamSynchronize(s));
        t->n_leaves = hb[0];
        t->n_gas_leaves = hb[1];
    }
    return CRK_OK;
}

int bits_for(int64_t v) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) <= v) ++b;
    return b;
}

}  // namespace

int tree_build(crk_ctx *ctx, crk_tree *t, const crk_boxes *bx, const void *gx,
               const void *gy, const void *gz, const void *gh, const void *dx,
               const void *dy, const void *dz) {
    const int nb = bx->n_boxes;
    const bool cap = ctx->capturing;
    const int64_t n_gas = bx->gas_off[nb], n_dm = bx->dm_off[nb];
    const int64_t n = n_gas + n_dm;
    if (n >= (int64_t)1 << 31)
        return set_error(CRK_EINVAL, "build_tree: more than 2^31 particles");
    const int L = ctx->tuning.leaf_max;
    // chaining-mesh geometry per box
    std::vector<int32_t> ncm(nb);
    std::vector<int64_t> base(nb + 1);
    base[0] = 0;
    for (int b = 0; b < nb; ++b) {
        // a bin at least as wide as every interaction range, so the 27-bin
        // stencil holds all partners; with cm_factor = 0 the bins are
        // widened until they hold ~4 leaves of the denser species
        const double w_min = std::max(bx->r_c[b], 2.0 * bx->h_max[b]);
        double w = w_min;
        if (ctx->tuning.cm_factor > 0.0) {
            w = w_min * ctx->tuning.cm_factor;
        } else {
            const double nsp = (double)std::max(bx->gas_off[b + 1] - bx->gas_off[b],
                                                bx->dm_off[b + 1] - bx->dm_off[b]);
            if (nsp > 0) w = std::max(w_min, std::cbrt(4.0 * L / nsp));
        }
        int64_t c = (int64_t)std::floor(1.0 / w);
        if (c < 1) c = 1;
        if (c > 1024) c = 1024;
        ncm[b] = (int32_t)c;
        base[b + 1] = base[b] + c * c * c;
    }
    const int64_t total_bins = base[nb];
    if (2 * total_bins + 2 >= ((int64_t)1 << 31) / 2 ||
        2 * total_bins >= ((int64_t)1 << 27))
        return set_error(CRK_EINVAL,
                         "build_tree: too many chaining-mesh bins (raise "
                         "cm_factor or r_c)");
    bool same = !t->cur_gas_off.empty() && t->n_boxes == nb &&
                std::equal(bx->gas_off, bx->gas_off + nb + 1, t->cur_gas_off.begin()) &&
                std::equal(bx->dm_off, bx->dm_off + nb + 1, t->cur_dm_off.begin()) &&
                std::equal(bx->r_c, bx->r_c + nb, t->cur_rc.begin()) &&
                std::equal(bx->eps, bx->eps + nb, t->cur_eps.begin()) &&
                std::equal(bx->h_max, bx->h_max + nb, t->cur_hmax.begin()) &&
                t->leaf_max == L;
    if (cap && !same)
        return set_error(CRK_ESTATE,
                         "build_tree: boxes or tuning changed during capture");
    // leaf upper bound: unsplit segments + split leaves, which hold about
    // L/2 particles or more (a quarter of L keeps a wide margin; a level
    // that would still overflow is run as an identity level and reported)
    int64_t seg_bound = std::min<int64_t>(n, 2 * total_bins);
    int64_t leaf_cap = seg_bound + n / std::max(1, L / 4) + 1;
    if (leaf_cap > n + 1) leaf_cap = n + 1;
    if (leaf_cap >= (int64_t)crk::LIST_LEAF_MASK)
        return set_error(CRK_EINVAL, "build_tree: too many leaves");
    t->n_gas = n_gas;
    t->n_dm = n_dm;
    t->n = n;
    t->n_boxes = nb;
    t->total_bins = total_bins;
    t->bin_bits = bits_for(2 * total_bins);
    t->leaf_max = L;
    t->leaf_cap = leaf_cap;
    CRK_TRY(ensure_all(t, n, leaf_cap, ctx->elem(), total_bins, cap));
    size_t need = std::max(radix_tmp_bytes(n), scan_tmp_bytes(n));
    need = std::max(need, scan_tmp_bytes(2 * total_bins + 2));
    need = std::max(need, scan_tmp_bytes(leaf_cap + 1));
    CRK_TRY(ctx->scratch.ensure(need, cap));
    if (!same) {
        // per-box metadata: pinned staging, then device
        size_t bytes = (size_t)(nb + 1) * 8 * 3 + (size_t)nb * (4 + 8 * 3) + 64;
        CRK_TRY(t->h_boxinfo.ensure(bytes));
        char *hp = t->h_boxinfo.as<char>();
        int64_t *hgo = reinterpret_cast<int64_t *>(hp);
        int64_t *hdo = hgo + (nb + 1);
        int64_t *hbb = hdo + (nb + 1);
        double *hrc = reinterpret_cast<double *>(hbb + (nb + 1));
        double *heps = hrc + nb;
        double *hhm = heps + nb;
        int32_t *hnc = reinterpret_cast<int32_t *>(hhm + nb);
        for (int b = 0; b <= nb; ++b) {
            hgo[b] = bx->gas_off[b];
            hdo[b] = bx->dm_off[b];
            hbb[b] = base[b];
        }
        for (int b = 0; b < nb; ++b) {
            hrc[b] = bx->r_c[b];
            heps[b] = bx->eps[b];
            hhm[b] = bx->h_max[b];
            hnc[b] = ncm[b];
        }
        CRK_TRY(t->d_gas_off.ensure((nb + 1) * 8, cap));
        CRK_TRY(t->d_dm_off.ensure((nb + 1) * 8, cap));
        CRK_TRY(t->d_bin_base.ensure((nb + 1) * 8, cap));
        CRK_TRY(t->d_rc.ensure(nb * 8, cap));
        CRK_TRY(t->d_eps.ensure(nb * 8, cap));
        CRK_TRY(t->d_hmax.ensure(nb * 8, cap));
        CRK_TRY(t->d_ncm.ensure(nb * 4, cap));
        hipStream_t s = ctx->stream;
        CRK_HIP(hipMemcpyAsync(t->d_gas_off.p, hgo, (nb + 1) * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_dm_off.p, hdo, (nb + 1) * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_bin_base.p, hbb, (nb + 1) * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_rc.p, hrc, nb * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_eps.p, heps, nb * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_hmax.p, hhm, nb * 8, hipMemcpyHostToDevice, s));
        CRK_HIP(hipMemcpyAsync(t->d_ncm.p, hnc, nb * 4, hipMemcpyHostToDevice, s));
        t->cur_gas_off.assign(bx->gas_off, bx->gas_off + nb + 1);
        t->cur_dm_off.assign(bx->dm_off, bx->dm_off + nb + 1);
        t->cur_rc.assign(bx->r_c, bx->r_c + nb);
        t->cur_eps.assign(bx->eps, bx->eps + nb);
        t->cur_hmax.assign(bx->h_max, bx->h_max + nb);
        t->h_ncm = ncm;
        t->h_rc = t->cur_rc;
    }
    t->lists_built = false;
    if (ctx->precision == CRK_FP64)
        return build_impl<double>(ctx, t, gx, gy, gz, gh, dx, dy, dz);
    return build_impl<float>(ctx, t, gx, gy, gz, gh, dx, dy, dz);
}

}  // namespace crk
