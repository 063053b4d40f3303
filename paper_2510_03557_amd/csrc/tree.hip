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
#include <limits>

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
        kout[c] = axis < 3 ? ((bk << 23) | coord_bits(v)) : bk;
        vout[c] = (int32_t)c;
    }
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ a,
                                int32_t *__restrict__ b, int64_t n) {
    GRID_STRIDE(i, n) b[i] = a[i];
}

__global__ void seg_flags_kernel(const uint64_t *__restrict__ k, int64_t n,
                                 int shift, int32_t *__restrict__ flags,
                                 int32_t *__restrict__ binkey) {
    GRID_STRIDE(p, n) {
        uint32_t bk = (uint32_t)(k[p] >> shift);
        binkey[p] = (int32_t)bk;
        flags[p] = (p == 0 || (uint32_t)(k[p - 1] >> shift) != bk) ? 1 : 0;
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

// a leaf count above the launch bound fixed at capture: error, and clamp
// (the clamped leaves are all written, so later kernels stay in bounds)
__global__ void bound_clamp_kernel(int32_t *__restrict__ nn, int64_t bound,
                                   int *__restrict__ err) {
    if (*nn > bound) {
        atomicOr(err, DEV_ERR_CAPACITY);
        *nn = (int32_t)bound;
    }
}

__global__ void bound_check_kernel(const int32_t *__restrict__ nn,
                                   int64_t bound, int *__restrict__ err) {
    if (*nn > bound) atomicOr(err, DEV_ERR_CAPACITY);
}

// slot of every caller index (the inverse of perm)
__global__ void iperm_kernel(const int32_t *__restrict__ perm, int64_t n,
                             int32_t *__restrict__ iperm) {
    GRID_STRIDE(p, n) iperm[perm[p]] = (int32_t)p;
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

// wave-wide reductions (all 64 lanes converged)
template <typename T> __device__ inline T wave_min(T v) {
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}
template <typename T> __device__ inline T wave_max(T v) {
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// ascending bitonic sort of one value per lane across the wavefront: lane r
// ends with the r-th smallest (all 64 lanes converged)
__device__ inline uint32_t wave_sort_u32(uint32_t v) {
    const int lane = threadIdx.x & 63;
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t o = __shfl_xor(v, j);
            const bool up = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            v = (lower == up) ? min(v, o) : max(v, o);
        }
    }
    return v;
}

// Leaf boxes (exact min / max of the members), h_max, box id and the count
// of leaves per (species, bin).  One wavefront per leaf.
template <typename T>
__global__ __launch_bounds__(256) void leaves_kernel(
    const int32_t *__restrict__ nd_start, const int32_t *__restrict__ nd_count,
    const int32_t *__restrict__ nd_key, const int32_t *__restrict__ nn_ptr,
    int64_t cap, const T *__restrict__ tx, const T *__restrict__ ty,
    const T *__restrict__ tz, const T *__restrict__ th, int64_t total_bins,
    int nb, const int64_t *__restrict__ bin_base,
    int32_t *__restrict__ leaf_box, T *__restrict__ lo, T *__restrict__ hi,
    T *__restrict__ lhmax, int32_t *__restrict__ bin_cnt, int sub,
    const int32_t *__restrict__ sub_n, const int32_t *__restrict__ sub_st,
    const int32_t *__restrict__ sub_c, T *__restrict__ slo,
    T *__restrict__ shi, T *__restrict__ shm) {
    const int64_t nn = *nn_ptr;
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nn) return;  // the whole wavefront leaves together
    const int st = nd_start[k], cnt = nd_count[k], key = nd_key[k];
    const T BIG = T(4), SMALL = T(0);
    T lx = BIG, ly = BIG, lz = BIG, hx = SMALL, hy = SMALL, hz = SMALL;
    T hm = SMALL;
    for (int p = st + lane; p < st + cnt; p += 64) {
        const T x = tx[p], y = ty[p], z = tz[p], h = th[p];
        lx = x < lx ? x : lx;
        hx = x > hx ? x : hx;
        ly = y < ly ? y : ly;
        hy = y > hy ? y : hy;
        lz = z < lz ? z : lz;
        hz = z > hz ? z : hz;
        hm = h > hm ? h : hm;
    }
    lx = wave_min(lx);
    ly = wave_min(ly);
    lz = wave_min(lz);
    hx = wave_max(hx);
    hy = wave_max(hy);
    hz = wave_max(hz);
    hm = wave_max(hm);
    if (lane == 0) {
        const int64_t gbin = key >= total_bins ? key - total_bins : key;
        leaf_box[k] = find_box(bin_base, nb, gbin);
        lo[k] = lx;
        hi[k] = hx;
        lo[cap + k] = ly;
        hi[cap + k] = hy;
        lo[2 * cap + k] = lz;
        hi[2 * cap + k] = hz;
        lhmax[k] = hm;
        atomicAdd(&bin_cnt[key], 1);
    }
    if (sub) {
        // sub-leaf g (<= 16 slots) on lanes 16g..16g+15, reduced per group
        const int g = lane >> 4, u = lane & 15;
        const int64_t sl = 4 * k + g;
        const bool v = g < sub_n[k] && u < sub_c[sl];
        const int q = v ? sub_st[sl] + u : st;
        const T x = tx[q], y = ty[q], z = tz[q], h = th[q];
        T ax = v ? x : BIG, bx = v ? x : SMALL, ay = v ? y : BIG,
          by = v ? y : SMALL, az = v ? z : BIG, bz = v ? z : SMALL,
          bh = v ? h : SMALL;
        for (int off = 8; off > 0; off >>= 1) {
            T w;
            w = __shfl_xor(ax, off); ax = w < ax ? w : ax;
            w = __shfl_xor(bx, off); bx = w > bx ? w : bx;
            w = __shfl_xor(ay, off); ay = w < ay ? w : ay;
            w = __shfl_xor(by, off); by = w > by ? w : by;
            w = __shfl_xor(az, off); az = w < az ? w : az;
            w = __shfl_xor(bz, off); bz = w > bz ? w : bz;
            w = __shfl_xor(bh, off); bh = w > bh ? w : bh;
        }
        if (u == 0 && g < sub_n[k]) {
            slo[sl] = ax;
            shi[sl] = bx;
            slo[4 * cap + sl] = ay;
            shi[4 * cap + sl] = by;
            slo[8 * cap + sl] = az;
            shi[8 * cap + sl] = bz;
            shm[sl] = bh;
        }
    }
}

// Splits every leaf of <= 64 particles by up to two more k-d levels (widest
// extent of the node, left side taking ceil(k/2) of the k sub-leaves of
// <= 16 it needs, ties by position in the leaf) and reorders the leaf's
// slots sub-leaf by sub-leaf (keeping the previous relative order inside
// each).  Writes per leaf the number of sub-leaves and per slot 4*leaf + k
// the sub-leaf's start, count, bounding box and h_max.  One wavefront per
// leaf, one particle per lane.
template <typename T>
__global__ __launch_bounds__(64) void subleaf_kernel(
    const int32_t *__restrict__ nn_ptr, const int32_t *__restrict__ leaf_start,
    const int32_t *__restrict__ leaf_count, int64_t cap, T *__restrict__ px,
    T *__restrict__ py, T *__restrict__ pz, T *__restrict__ ph,
    int32_t *__restrict__ perm, int32_t *__restrict__ nsub,
    int32_t *__restrict__ sst, int32_t *__restrict__ scnt,
    T *__restrict__ slo, T *__restrict__ shi, T *__restrict__ shm) {
    const int I = (int)blockIdx.x;
    if (I >= *nn_ptr) return;
    const int t = threadIdx.x;
    const int st = leaf_start[I];
    const int c = min(leaf_count[I], 64);
    const bool act = t < c;
    const int p = st + (act ? t : 0);
    const T x = px[p], y = py[p], z = pz[p], h = ph[p];
    const int pm = perm[p];
    const T BIG = T(4), SMALL = T(0);
    int node = 0;
    for (int lev = 0; lev < 2; ++lev) {
        int side = 0;
        const int nodes = 1 << lev;
        for (int n = 0; n < nodes; ++n) {
            const bool in = act && node == n;
            const int cn = __popcll(__ballot(in));
            if (cn <= 16) continue;
            const T ex = wave_max(in ? x : SMALL) - wave_min(in ? x : BIG);
            const T ey = wave_max(in ? y : SMALL) - wave_min(in ? y : BIG);
            const T ez = wave_max(in ? z : SMALL) - wave_min(in ? z : BIG);
            int a = 0;
            T best = ex;
            if (ey > best) {
                a = 1;
                best = ey;
            }
            if (ez > best) a = 2;
            // order key: coordinate bits along the axis, then the slot
            const T key = a == 0 ? x : (a == 1 ? y : z);
            const uint32_t k32 =
                in ? ((coord_bits(key) << 6) | (uint32_t)t) : 0xFFFFFFFFu;
            const uint32_t sorted = wave_sort_u32(k32);
            const int nl = (cn + 15) / 16;
            const int nleft = (nl + 1) / 2;
            const int left = (cn * nleft + nl / 2) / nl;
            // the right part starts at the left-th smallest key of the node
            const uint32_t thr = __shfl(sorted, left);
            if (in) side = k32 >= thr ? 1 : 0;
        }
        node = 2 * node + side;
    }
    // final order: sub-leaf by sub-leaf, previous order inside each
    int cnt4[4];
    uint64_t msk[4];
    for (int m = 0; m < 4; ++m) {
        msk[m] = __ballot(act && node == m);
        cnt4[m] = __popcll(msk[m]);
    }
    const uint64_t lt = (t == 0) ? 0ull : (~0ull >> (64 - t));
    const uint64_t mine = node == 0 ? msk[0]
                        : (node == 1 ? msk[1] : (node == 2 ? msk[2] : msk[3]));
    const int within = __popcll(mine & lt);
    int off = 0;
    for (int m = 0; m < node; ++m) off += cnt4[m];
    // every lane holds its particle in registers: safe to overwrite
    __syncthreads();
    if (act) {
        const int q = st + off + within;
        px[q] = x;
        py[q] = y;
        pz[q] = z;
        ph[q] = h;
        perm[q] = pm;
    }
    // boxes of the sub-leaves: stage the new leaf order in LDS, then lanes
    // 16k..16k+15 hold non-empty sub-leaf k and reduce within their group
    __shared__ T sx[64], sy[64], sz[64], sh[64];
    if (act) {
        sx[off + within] = x;
        sy[off + within] = y;
        sz[off + within] = z;
        sh[off + within] = h;
    }
    int kst[4] = {0, 0, 0, 0}, kcn[4] = {0, 0, 0, 0};
    int nk = 0, o = 0;
    for (int m = 0; m < 4; ++m) {
        if (cnt4[m] == 0) continue;
        kst[nk] = o;
        kcn[nk] = cnt4[m];
        o += cnt4[m];
        ++nk;
    }
    __syncthreads();
    const int g = t >> 4, u = t & 15;
    const int gst = g == 0 ? kst[0] : (g == 1 ? kst[1] : (g == 2 ? kst[2] : kst[3]));
    const int gcn = g == 0 ? kcn[0] : (g == 1 ? kcn[1] : (g == 2 ? kcn[2] : kcn[3]));
    const bool v = g < nk && u < gcn;
    T lx = v ? sx[gst + u] : BIG, hx = v ? sx[gst + u] : SMALL;
    T ly = v ? sy[gst + u] : BIG, hy = v ? sy[gst + u] : SMALL;
    T lz = v ? sz[gst + u] : BIG, hz = v ? sz[gst + u] : SMALL;
    T hm = v ? sh[gst + u] : SMALL;
    for (int off2 = 8; off2 > 0; off2 >>= 1) {
        T w;
        w = __shfl_xor(lx, off2); lx = w < lx ? w : lx;
        w = __shfl_xor(hx, off2); hx = w > hx ? w : hx;
        w = __shfl_xor(ly, off2); ly = w < ly ? w : ly;
        w = __shfl_xor(hy, off2); hy = w > hy ? w : hy;
        w = __shfl_xor(lz, off2); lz = w < lz ? w : lz;
        w = __shfl_xor(hz, off2); hz = w > hz ? w : hz;
        w = __shfl_xor(hm, off2); hm = w > hm ? w : hm;
    }
    if (u == 0 && g < nk) {
        const int64_t sl = 4 * (int64_t)I + g;
        sst[sl] = st + gst;
        scnt[sl] = gcn;
        slo[sl] = lx;
        shi[sl] = hx;
        slo[4 * cap + sl] = ly;
        shi[4 * cap + sl] = hy;
        slo[8 * cap + sl] = lz;
        shi[8 * cap + sl] = hz;
        shm[sl] = hm;
    }
    if (t == 0) nsub[I] = nk;
}

// ---------------------------------------------------------------------------
// Per-bin build in LDS.  After one stable sort by (species, bin) key alone,
// every segment holds its particles in caller order; one workgroup per
// segment then (a) sorts the segment along each axis by (coordinate key,
// position in the segment) -- the same order the per-axis global sorts give,
// since position in the segment is caller order -- and (b) runs every k-d
// level of that segment on the three sorted arrays in LDS with the same
// split rule and the same stable partitions as the global levels.  The
// leaves come out identical, in the same order, at the leaf offsets given by
// a prefix sum of ceil(count / leaf_max) per segment (the exact leaf count of
// the balanced split).

constexpr int SEG_TB = 256;      // threads per segment workgroup
constexpr int SEG_MAX = 2048;    // largest segment sorted in LDS
constexpr int SEG_RANK = 512;    // up to here: rank sort (else bitonic)

// Bytes before the sorted position arrays.  Rank sort (SEG <= 512): u32
// keys (coordinate bits << 9 | position) of all three axes, which stay
// valid through the k-d levels, then the level scratch (9 B per slot);
// bitonic sort: u64 keys of one axis at a time, aliased by the level
// scratch afterwards.
__device__ __host__ inline size_t seg_key_bytes(int SEG) {
    return (size_t)(SEG <= SEG_RANK ? 12 + 9 : 9) * SEG;
}

// leaves the balanced split makes of a node of c particles
__device__ __host__ inline int seg_leaves(int c, int L) {
    return c <= 0 ? 0 : (c + L - 1) / L;
}

__global__ void seg_leafcount_kernel(const int32_t *__restrict__ nd_count,
                                     const int32_t *__restrict__ nn_ptr,
                                     int64_t cap, int L,
                                     int32_t *__restrict__ nl,
                                     int32_t *__restrict__ maxc) {
    const int64_t nn = *nn_ptr;
    GRID_STRIDE(k, cap) {
        if (k >= nn) {
            nl[k] = 0;
            continue;
        }
        const int c = nd_count[k];
        nl[k] = seg_leaves(c, L);
        atomicMax(maxc, c);
    }
}

template <typename T>
__device__ inline T seg_coord(const T *px, const T *py, const T *pz, int a,
                              int32_t c) {
    return a == 0 ? px[c] : (a == 1 ? py[c] : pz[c]);
}

// One workgroup per segment; SEG (a power of two >= 64, <= SEG_MAX) is the
// padded segment size the dynamic LDS is laid out for:
//   SEG <= SEG_RANK: keys u32[3][SEG], then the level scratch
//   larger SEG:      keys u64[SEG] (one axis at a time), aliased by the
//                    level scratch
//   level scratch:   spare u16[3][SEG], en u16[SEG], flag u8[SEG]
//   S0, S1, S2 u16[SEG] (axis-sorted positions in the segment)
//   node arrays (MAXN = SEG/8 + 2 each): start, count (two generations),
//   left, axis, child, three partition bases, saved leaf start and count
// With sub = 1 (leaf_max <= 64), every leaf is then split by further levels
// at 16 into <= 4 sub-leaves (same rule), written per leaf slot 4*leaf + k.
// A segment larger than SEG raises the capacity error and is cut into
// consecutive chunks of leaf_max (and 16) (bounds-safe, not a k-d split).
template <typename T>
__global__ __launch_bounds__(SEG_TB) void seg_build_kernel(
    const int32_t *__restrict__ nn_ptr, const int32_t *__restrict__ seg_start,
    const int32_t *__restrict__ seg_count, const int32_t *__restrict__ seg_key,
    const int32_t *__restrict__ leaf_off, const int32_t *__restrict__ V,
    const T *__restrict__ px, const T *__restrict__ py,
    const T *__restrict__ pz, int L, int SEG, int cmin, int cmax,
    int64_t lcap, int sub, int32_t *__restrict__ S0g,
    int32_t *__restrict__ lf_start,
    int32_t *__restrict__ lf_count, int32_t *__restrict__ lf_key,
    int32_t *__restrict__ sub_n, int32_t *__restrict__ sub_st,
    int32_t *__restrict__ sub_c, int *__restrict__ err) {
    extern __shared__ __align__(16) unsigned char seg_lds[];
    const int sg = (int)blockIdx.x;
    if (sg >= *nn_ptr) return;
    const int t = threadIdx.x;
    const int s0 = seg_start[sg], cnt = seg_count[sg], key = seg_key[sg];
    // this launch builds the segments of one size class, cmin < cnt <= cmax
    if (cnt <= cmin || cnt > cmax) return;
    const int loff = leaf_off[sg];
    const int nlv = seg_leaves(cnt, L);
    if ((int64_t)loff + nlv > lcap || cnt > SEG) {
        // a leaf count beyond the capacity is reported by the count kernel
        // and cannot happen (the capacity bounds the sum of ceil(c / L));
        // a segment beyond SEG is cut in chunks: every slot stays valid
        if (t == 0) atomicOr(err, DEV_ERR_CAPACITY);
        for (int p = t; p < cnt; p += SEG_TB) S0g[s0 + p] = V[s0 + p];
        if ((int64_t)loff + nlv > lcap) return;
        for (int k = t; k < nlv; k += SEG_TB) {
            const int c = min(L, cnt - k * L);
            lf_start[loff + k] = s0 + k * L;
            lf_count[loff + k] = c;
            lf_key[loff + k] = key;
            if (sub) {
                const int ns = min(4, (c + 15) / 16);
                sub_n[loff + k] = ns;
                for (int g = 0; g < ns; ++g) {
                    sub_st[4 * (int64_t)(loff + k) + g] = s0 + k * L + 16 * g;
                    sub_c[4 * (int64_t)(loff + k) + g] = min(16, c - 16 * g);
                }
            }
        }
        return;
    }
    const int MAXN = SEG / 8 + 2;
    const bool rank = SEG <= SEG_RANK;
    uint64_t *keys = reinterpret_cast<uint64_t *>(seg_lds);
    uint32_t *CK = reinterpret_cast<uint32_t *>(seg_lds);  // rank: [3][SEG]
    uint16_t *spare0 = reinterpret_cast<uint16_t *>(
        seg_lds + (rank ? (size_t)12 * SEG : 0));
    uint16_t *spare[3] = {spare0, spare0 + SEG, spare0 + 2 * SEG};
    uint16_t *en = spare0 + 3 * SEG;
    uint8_t *flag = reinterpret_cast<uint8_t *>(en + SEG);
    uint16_t *Sa[3];
    Sa[0] = reinterpret_cast<uint16_t *>(seg_lds + seg_key_bytes(SEG));
    Sa[1] = Sa[0] + SEG;
    Sa[2] = Sa[1] + SEG;
    int32_t *nst[2], *ncnt[2];
    nst[0] = reinterpret_cast<int32_t *>(Sa[2] + SEG);
    nst[1] = nst[0] + MAXN;
    ncnt[0] = nst[1] + MAXN;
    ncnt[1] = ncnt[0] + MAXN;
    int32_t *nleft = ncnt[1] + MAXN;
    int32_t *naxis = nleft + MAXN;
    int32_t *nchild = naxis + MAXN;
    int32_t *nbase = nchild + MAXN;  // [3][MAXN]
    int32_t *lst = nbase + 3 * MAXN;
    int32_t *lct = lst + MAXN;
    __shared__ long long wsum64[SEG_TB / 64];
    __shared__ int s_nn;

    // (a) three sorts by (coordinate key, position)
    if (rank) {
        // bucketed rank sort: keys are distinct (coordinate bits, then the
        // position in the segment); per axis the positions are grouped into
        // 64 buckets of equal coordinate width (counting sort in LDS), and
        // the rank of an element is its bucket's start plus the number of
        // smaller keys inside its bucket
        uint32_t *K[3] = {CK, CK + SEG, CK + 2 * SEG};
        __shared__ int hist[3][64], bst[3][64], bcur[3][64];
        __shared__ uint32_t wmn[SEG_TB / 64][3], wmx[SEG_TB / 64][3];
        uint32_t lmn[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        uint32_t lmx[3] = {0u, 0u, 0u};
        for (int p = t; p < cnt; p += SEG_TB) {
            const int32_t c = V[s0 + p];
            const uint32_t kx = coord_bits(px[c]), ky = coord_bits(py[c]),
                           kz = coord_bits(pz[c]);
            K[0][p] = (kx << 9) | (uint32_t)p;
            K[1][p] = (ky << 9) | (uint32_t)p;
            K[2][p] = (kz << 9) | (uint32_t)p;
            lmn[0] = min(lmn[0], kx);
            lmx[0] = max(lmx[0], kx);
            lmn[1] = min(lmn[1], ky);
            lmx[1] = max(lmx[1], ky);
            lmn[2] = min(lmn[2], kz);
            lmx[2] = max(lmx[2], kz);
        }
        for (int k = t; k < 3 * 64; k += SEG_TB) (&hist[0][0])[k] = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            for (int off = 32; off > 0; off >>= 1) {
                lmn[a] = min(lmn[a], (uint32_t)__shfl_xor((int)lmn[a], off));
                lmx[a] = max(lmx[a], (uint32_t)__shfl_xor((int)lmx[a], off));
            }
            if ((t & 63) == 0) {
                wmn[t >> 6][a] = lmn[a];
                wmx[t >> 6][a] = lmx[a];
            }
        }
        __syncthreads();
        uint32_t mn[3], wd[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint32_t m0 = 0xFFFFFFFFu, m1 = 0u;
            for (int w = 0; w < SEG_TB / 64; ++w) {
                m0 = min(m0, wmn[w][a]);
                m1 = max(m1, wmx[w][a]);
            }
            mn[a] = m0;
            wd[a] = m1 >= m0 ? m1 - m0 + 1 : 1;
        }
        auto bucket = [&](int a, uint32_t k) {
            return (int)((uint64_t)((k >> 9) - mn[a]) * 64u / wd[a]);
        };
        for (int p = t; p < cnt; p += SEG_TB) {
#pragma unroll
            for (int a = 0; a < 3; ++a) atomicAdd(&hist[a][bucket(a, K[a][p])], 1);
        }
        __syncthreads();
        if (t < 3) {
            int acc = 0;
            for (int q = 0; q < 64; ++q) {
                bst[t][q] = acc;
                bcur[t][q] = acc;
                acc += hist[t][q];
            }
        }
        __syncthreads();
        // bucket members (any order inside a bucket) in the level scratch
        for (int p = t; p < cnt; p += SEG_TB) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int bk = bucket(a, K[a][p]);
                spare[a][atomicAdd(&bcur[a][bk], 1)] = (uint16_t)p;
            }
        }
        __syncthreads();
        for (int p = t; p < cnt; p += SEG_TB) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uint32_t kp = K[a][p];
                const int bk = bucket(a, kp);
                const int b0 = bst[a][bk], b1 = b0 + hist[a][bk];
                int r = b0;
                for (int q = b0; q < b1; ++q) r += K[a][spare[a][q]] < kp ? 1 : 0;
                Sa[a][r] = (uint16_t)p;
            }
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            for (int p = t; p < SEG; p += SEG_TB) {
                uint64_t kk = ~0ull;
                if (p < cnt)
                    kk = ((uint64_t)coord_bits(seg_coord(px, py, pz, a, V[s0 + p]))
                          << 16) | (uint64_t)p;
                keys[p] = kk;
            }
            __syncthreads();
            for (int k = 2; k <= SEG; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = t; i < SEG; i += SEG_TB) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const uint64_t x = keys[i], y = keys[ixj];
                            const bool up = (i & k) == 0;
                            if ((x > y) == up) {
                                keys[i] = y;
                                keys[ixj] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (int p = t; p < cnt; p += SEG_TB)
                Sa[a][p] = (uint16_t)(keys[p] & 0xFFFFu);
            __syncthreads();
        }
    }

    // (b) k-d levels: first at L, then (sub) at 16 inside the leaves
    int cur = 0;
    int nn = 1;
    if (t == 0) {
        nst[0][0] = 0;
        ncnt[0][0] = cnt;
    }
    for (int p = t; p < cnt; p += SEG_TB) en[p] = 0;
    __syncthreads();
    // positions per thread in the partition: a contiguous run of PER
    const int PER = SEG / SEG_TB > 0 ? SEG / SEG_TB : 1;
    const int p0 = t * PER;
    auto level = [&](const int Lc) -> bool {
        int any = 0;
        for (int k = t; k < nn; k += SEG_TB) {
            const int st = nst[cur][k], c = ncnt[cur][k];
            int lf = 0, ax = 0;
            if (c > Lc) {
                const int e = st + c - 1;
                if (sizeof(T) == 4 && rank) {
                    // float coordinates in [1, 2) share one exponent: the
                    // difference of their bits orders the extents exactly
                    const int ex = (int)(CK[Sa[0][e]] >> 9) - (int)(CK[Sa[0][st]] >> 9);
                    const int ey = (int)(CK[SEG + Sa[1][e]] >> 9) -
                                   (int)(CK[SEG + Sa[1][st]] >> 9);
                    const int ez = (int)(CK[2 * SEG + Sa[2][e]] >> 9) -
                                   (int)(CK[2 * SEG + Sa[2][st]] >> 9);
                    int best = ex;
                    if (ey > best) {
                        ax = 1;
                        best = ey;
                    }
                    if (ez > best) ax = 2;
                } else {
                    const T ex = px[V[s0 + Sa[0][e]]] - px[V[s0 + Sa[0][st]]];
                    const T ey = py[V[s0 + Sa[1][e]]] - py[V[s0 + Sa[1][st]]];
                    const T ez = pz[V[s0 + Sa[2][e]]] - pz[V[s0 + Sa[2][st]]];
                    T best = ex;
                    if (ey > best) {
                        ax = 1;
                        best = ey;
                    }
                    if (ez > best) ax = 2;
                }
                const int nl = (c + Lc - 1) / Lc;
                const int nlft = (nl + 1) / 2;
                lf = (int)(((long long)c * nlft + nl / 2) / nl);
                any = 1;
            }
            nleft[k] = lf;
            naxis[k] = ax;
        }
        if (!__syncthreads_or(any)) return false;
        if (t == 0) {
            int acc = 0;
            for (int k = 0; k < nn; ++k) {
                nchild[k] = acc;
                acc += nleft[k] ? 2 : 1;
            }
            s_nn = acc;
        }
        // left-side flag per position in the segment (indexed by position
        // in the unsorted segment, which every sorted array refers to)
        for (int p = t; p < cnt; p += SEG_TB) {
            const int k = en[p];
            const int lf = nleft[k];
            if (lf) {
                const int ax = naxis[k];
                const uint16_t *Sx = ax == 0 ? Sa[0] : (ax == 1 ? Sa[1] : Sa[2]);
                flag[Sx[p]] = (p - nst[cur][k] < lf) ? 1 : 0;
            }
        }
        __syncthreads();
        // stable partition of every splitting node of all three arrays at
        // once: one prefix sum of the three left-flags packed in 21-bit
        // fields (counts <= SEG_MAX), node bases from the node starts
        int fb[16];
        long long sum = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (u >= PER) break;
            const int p = p0 + u;
            int f = 0;
            if (p < cnt) {
                const int k = en[p];
                if (nleft[k])
                    f = flag[Sa[0][p]] | (flag[Sa[1][p]] << 1) | (flag[Sa[2][p]] << 2);
                else
                    f = 7;
            }
            fb[u] = f;
            sum += (long long)(f & 1) | ((long long)((f >> 1) & 1) << 21) |
                   ((long long)(f >> 2) << 42);
        }
        long long run;
        {
            const int lane = t & 63, w = t >> 6;
            long long incl = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const long long o = __shfl_up(incl, off);
                if (lane >= off) incl += o;
            }
            if (lane == 63) wsum64[w] = incl;
            __syncthreads();
            long long base = 0;
            for (int q = 0; q < SEG_TB / 64; ++q) base += q < w ? wsum64[q] : 0;
            run = base + incl - sum;
        }
        {
            long long r = run;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (u >= PER) break;
                const int p = p0 + u;
                if (p < cnt) {
                    const int k = en[p];
                    if (nst[cur][k] == p) {
                        nbase[k] = (int)(r & 0x1FFFFF);
                        nbase[MAXN + k] = (int)((r >> 21) & 0x1FFFFF);
                        nbase[2 * MAXN + k] = (int)(r >> 42);
                    }
                }
                const int f = fb[u];
                r += (long long)(f & 1) | ((long long)((f >> 1) & 1) << 21) |
                     ((long long)(f >> 2) << 42);
            }
        }
        __syncthreads();
        {
            long long r = run;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                if (u >= PER) break;
                const int p = p0 + u;
                if (p < cnt) {
                    const int k = en[p];
                    const int st = nst[cur][k];
                    const int lf = nleft[k];
                    const int lc = lf ? lf : ncnt[cur][k];
                    const int f = fb[u];
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int rb = (int)((r >> (21 * b)) & 0x1FFFFF);
                        const int rl = rb - nbase[b * MAXN + k];
                        const int np = ((f >> b) & 1) ? st + rl
                                                      : st + lc + (p - st - rl);
                        spare[b][np] = Sa[b][p];
                    }
                }
                const int f = fb[u];
                r += (long long)(f & 1) | ((long long)((f >> 1) & 1) << 21) |
                     ((long long)(f >> 2) << 42);
            }
        }
        // children and the position -> node map of the next level
        const int nxt = cur ^ 1;
        for (int k = t; k < nn; k += SEG_TB) {
            const int cb = nchild[k], st = nst[cur][k], c = ncnt[cur][k];
            const int lf = nleft[k];
            if (lf) {
                nst[nxt][cb] = st;
                ncnt[nxt][cb] = lf;
                nst[nxt][cb + 1] = st + lf;
                ncnt[nxt][cb + 1] = c - lf;
            } else {
                nst[nxt][cb] = st;
                ncnt[nxt][cb] = c;
            }
        }
        // (the positions this thread scattered from: no other thread reads
        // their en in this level)
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (u >= PER) break;
            const int p = p0 + u;
            if (p < cnt) {
                const int k = en[p];
                const int lf = nleft[k];
                en[p] = (uint16_t)(nchild[k] +
                                   ((lf && p - nst[cur][k] >= lf) ? 1 : 0));
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint16_t *tmp = Sa[b];
            Sa[b] = spare[b];
            spare[b] = tmp;
        }
        nn = s_nn;
        cur = nxt;
        return true;
    };
    while (level(L)) {
    }
    // the leaves
    const int nleaves = nn;
    for (int k = t; k < nn; k += SEG_TB) {
        lst[k] = nst[cur][k];
        lct[k] = ncnt[cur][k];
        lf_start[loff + k] = s0 + nst[cur][k];
        lf_count[loff + k] = ncnt[cur][k];
        lf_key[loff + k] = key;
    }
    if (sub) {
        __syncthreads();
        while (level(16)) {
        }
        // final node m lies in leaf k: its slot is 4 (loff + k) + (m - first
        // node of leaf k); nodes and leaves are both in position order
        for (int k = t; k < nleaves; k += SEG_TB) {
            int lo = 0, hi = nn;  // first node with start >= lst[k]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (nst[cur][mid] < lst[k]) lo = mid + 1;
                else hi = mid;
            }
            int m = lo, g = 0;
            while (m < nn && nst[cur][m] < lst[k] + lct[k] && g < 4) {
                sub_st[4 * (int64_t)(loff + k) + g] = s0 + nst[cur][m];
                sub_c[4 * (int64_t)(loff + k) + g] = ncnt[cur][m];
                ++m;
                ++g;
            }
            sub_n[loff + k] = g;
        }
    }

    // (c) the tree order of the segment
    for (int p = t; p < cnt; p += SEG_TB) S0g[s0 + p] = V[s0 + Sa[0][p]];
}

size_t seg_lds_bytes(int SEG) {
    const int MAXN = SEG / 8 + 2;
    return seg_key_bytes(SEG) + (size_t)SEG * 6 + (size_t)MAXN * 12 * 4;
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
    CRK_TRY(t->iperm.ensure(n1 * 4, cap));
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
    const int L = t->leaf_max;
    // sub-leaves (leaves of <= 64 particles, for the sub-leaf sweeps)
    t->has_sub = L <= 64 && ctx->tuning.sub_sweep != 0;
    bool sub_done = false;  // split by the per-bin build
    if (t->has_sub) {
        const int64_t sl = 4 * (lcap + 1);
        CRK_TRY(t->sub_nsub.ensure((lcap + 1) * 4, cap));
        CRK_TRY(t->sub_start.ensure(sl * 4, cap));
        CRK_TRY(t->sub_count.ensure(sl * 4, cap));
        CRK_TRY(t->sub_lo.ensure(3 * sl * sizeof(T), cap));
        CRK_TRY(t->sub_hi.ensure(3 * sl * sizeof(T), cap));
        CRK_TRY(t->sub_hmax.ensure(sl * sizeof(T), cap));
    }
    // segments: one per non-empty (species, bin)
    const int64_t seg_cap = std::min<int64_t>(n, 2 * t->total_bins);
    int cur = 0;
    bool use_lds = cap ? t->lds_tree : ctx->tuning.tree_lds != 0;
    if (use_lds) {
        // 1. one stable sort by (species, bin): caller order inside a bin
        hipLaunchKernelGGL((keys_kernel<T>), dim3(grid_for(n)), dim3(TB), 0, s,
                           gx, gy, gz, gh, dx, dy, dz, t->n_gas, n, t->n_boxes,
                           t->d_gas_off.as<int64_t>(), t->d_dm_off.as<int64_t>(),
                           t->d_ncm.as<int>(), t->d_bin_base.as<int64_t>(),
                           t->d_hmax.as<double>(), t->total_bins, 3, 1, px, py,
                           pz, ph, K[0], Vv[0], err);
        CRK_HIP(hipGetLastError());
        hipError_t he;
        const int r = radix_sort_u64_i32(K, Vv, n, t->bin_bits, ctx->scratch.p,
                                         s, &he);
        CRK_HIP(he);
        hipLaunchKernelGGL(seg_flags_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                           K[r], n, 0, flags, t->binkey.as<int32_t>());
        CRK_HIP(hipGetLastError());
        CRK_HIP(exclusive_scan_i32(flags, sf, n, cnt + C_NN, ctx->scratch.p, s));
        hipLaunchKernelGGL(seg_nodes_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                           flags, sf, t->binkey.as<int32_t>(), n,
                           t->nd_start[0].as<int32_t>(),
                           t->nd_key[0].as<int32_t>(),
                           t->elem_node.as<int32_t>());
        CRK_HIP(hipGetLastError());
        hipLaunchKernelGGL(node_counts_kernel, dim3(grid_for(seg_cap)), dim3(TB),
                           0, s, t->nd_start[0].as<int32_t>(), cnt + C_NN,
                           seg_cap, n, t->nd_count[0].as<int32_t>());
        CRK_HIP(hipGetLastError());
        // 2. leaves per segment and their offsets; the largest segment
        CRK_HIP(fill_i32(cnt + C_MAXC, 0, 1, s));
        hipLaunchKernelGGL(seg_leafcount_kernel, dim3(grid_for(seg_cap)),
                           dim3(TB), 0, s, t->nd_count[0].as<int32_t>(),
                           cnt + C_NN, seg_cap, L,
                           t->nd_nchild.as<int32_t>(), cnt + C_MAXC);
        CRK_HIP(hipGetLastError());
        CRK_HIP(exclusive_scan_i32(t->nd_nchild.as<int32_t>(),
                                   t->nd_child.as<int32_t>(), seg_cap,
                                   cnt + C_NN_NEXT, ctx->scratch.p, s));
        if (!cap) {
            int32_t *hb = ctx->err_host.as<int32_t>() + 8;
            CRK_HIP(hipMemcpyAsync(hb, cnt + C_MAXC, 4, hipMemcpyDeviceToHost, s));
            CRK_HIP(hipStreamSynchronize(s));
            const int maxc = hb[0];
            if (maxc > SEG_MAX) {
                use_lds = false;
            } else {
                // room for growth of the largest bin before a captured
                // replay reports capacity
                int seg = 64;
                while (seg < maxc + maxc / 4 + 16 && seg < SEG_MAX) seg <<= 1;
                t->seg_size = seg;
                int lev = 0;
                while ((1 << lev) < seg_leaves(maxc, L)) ++lev;
                t->kd_levels = lev;
            }
            t->lds_tree = use_lds;
        }
        if (use_lds) {
            // 3. sorts and k-d levels of every segment in LDS, one launch per
            //    size class (padded sizes 128, 256, ... up to the largest):
            //    a segment is sorted at the padded size of its class, with
            //    that class's LDS, instead of at the size of the largest
            //    segment (the same leaves either way: the keys are distinct)
            const int SEG = t->seg_size;
            int cmin = 0;
            for (int c = 128;; c <<= 1) {
                const bool last = c >= SEG;
                const int seg_c = last ? SEG : c;
                hipLaunchKernelGGL((seg_build_kernel<T>),
                                   dim3((unsigned)std::max<int64_t>(1, seg_cap)),
                                   dim3(SEG_TB), seg_lds_bytes(seg_c), s,
                                   cnt + C_NN, t->nd_start[0].as<int32_t>(),
                                   t->nd_count[0].as<int32_t>(),
                                   t->nd_key[0].as<int32_t>(),
                                   t->nd_child.as<int32_t>(), Vv[r], px, py, pz,
                                   L, seg_c, cmin,
                                   last ? std::numeric_limits<int>::max() : c,
                                   lcap, t->has_sub ? 1 : 0, S[0],
                                   t->nd_start[1].as<int32_t>(),
                                   t->nd_count[1].as<int32_t>(),
                                   t->nd_key[1].as<int32_t>(),
                                   t->sub_nsub.as<int32_t>(),
                                   t->sub_start.as<int32_t>(),
                                   t->sub_count.as<int32_t>(), err);
                CRK_HIP(hipGetLastError());
                if (last) break;
                cmin = c;
            }
            sub_done = t->has_sub;
            hipLaunchKernelGGL(next_count_kernel, dim3(1), dim3(1), 0, s,
                               cnt + C_NN_NEXT, lcap, cnt + C_NN, err);
            CRK_HIP(hipGetLastError());
            cur = 1;
        }
    }
    if (!use_lds) {
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
                                   s, K[r], n, 23, flags, t->binkey.as<int32_t>());
                CRK_HIP(hipGetLastError());
            }
        }
        CRK_HIP(exclusive_scan_i32(flags, sf, n, cnt + C_NN, ctx->scratch.p, s));
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
    }
    // remember which buffers hold the final state
    t->cur_nodes = cur;
    for (int a = 0; a < 3; ++a) t->S_final[a] = S[a];

    // 4. launch bound of the leaf-indexed kernels: the exact leaf count
    //    (eager; read back here), or under capture the bound set by the last
    //    eager build -- a larger device count raises the capacity error and
    //    is clamped, so every later kernel stays inside written leaves
    if (!cap) {
        int32_t *hb = ctx->err_host.as<int32_t>() + 8;
        CRK_HIP(hipMemcpyAsync(hb, cnt + C_NN, 4, hipMemcpyDeviceToHost, s));
        CRK_HIP(hipStreamSynchronize(s));
        t->n_leaves = hb[0];
        t->graph_nb = std::min<int64_t>(lcap, t->n_leaves + t->n_leaves / 4 + 1024);
        t->nb_launch = t->n_leaves;
    } else {
        t->nb_launch = t->graph_nb;
        hipLaunchKernelGGL(bound_clamp_kernel, dim3(1), dim3(1), 0, s,
                           cnt + C_NN, t->graph_nb, err);
        CRK_HIP(hipGetLastError());
    }
    const int64_t nbl = std::max<int64_t>(1, t->nb_launch);

    // 5. tree order, leaves, bin -> leaf table
    const int64_t nbin2 = 2 * t->total_bins;
    hipLaunchKernelGGL((gather_tree_kernel<T>), dim3(grid_for(n)), dim3(TB), 0, s,
                       S[0], px, py, pz, ph, n, t->perm.as<int32_t>(),
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                       t->hsm.as<T>());
    CRK_HIP(hipGetLastError());
    CRK_HIP(fill_i32(t->bin_cnt.as<int32_t>(), 0, nbin2 + 1, s));
    hipLaunchKernelGGL((leaves_kernel<T>),
                       dim3((unsigned)((nbl + 3) / 4)), dim3(256), 0, s,
                       t->nd_start[cur].as<int32_t>(),
                       t->nd_count[cur].as<int32_t>(),
                       t->nd_key[cur].as<int32_t>(), cnt + C_NN, lcap,
                       t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                       t->hsm.as<T>(), t->total_bins, t->n_boxes,
                       t->d_bin_base.as<int64_t>(), t->leaf_box.as<int32_t>(),
                       t->leaf_lo.as<T>(), t->leaf_hi.as<T>(),
                       t->leaf_hmax.as<T>(), t->bin_cnt.as<int32_t>(),
                       sub_done ? 1 : 0, t->sub_nsub.as<int32_t>(),
                       t->sub_start.as<int32_t>(), t->sub_count.as<int32_t>(),
                       t->sub_lo.as<T>(), t->sub_hi.as<T>(),
                       t->sub_hmax.as<T>());
    CRK_HIP(hipGetLastError());
    CRK_HIP(exclusive_scan_i32(t->bin_cnt.as<int32_t>(),
                               t->bin_leaf.as<int32_t>(), nbin2 + 1, nullptr,
                               ctx->scratch.p, s));
    // 6. sub-leaves of the general path: one wavefront per leaf
    if (t->has_sub && !sub_done) {
        hipLaunchKernelGGL((subleaf_kernel<T>), dim3((unsigned)nbl),
                           dim3(64), 0, s, cnt + C_NN,
                           t->nd_start[cur].as<int32_t>(),
                           t->nd_count[cur].as<int32_t>(), lcap,
                           t->pos[0].as<T>(), t->pos[1].as<T>(), t->pos[2].as<T>(),
                           t->hsm.as<T>(), t->perm.as<int32_t>(),
                           t->sub_nsub.as<int32_t>(), t->sub_start.as<int32_t>(),
                           t->sub_count.as<int32_t>(), t->sub_lo.as<T>(),
                           t->sub_hi.as<T>(), t->sub_hmax.as<T>());
        CRK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(iperm_kernel, dim3(grid_for(n)), dim3(TB), 0, s,
                       t->perm.as<int32_t>(), n, t->iperm.as<int32_t>());
    CRK_HIP(hipGetLastError());
    int32_t *gas_nl = t->bin_leaf.as<int32_t>() + t->total_bins;
    if (!cap) {
        // gas leaves for the host
        int32_t *hb = ctx->err_host.as<int32_t>() + 8;
        CRK_HIP(hipMemcpyAsync(hb + 1, gas_nl, 4, hipMemcpyDeviceToHost, s));
        CRK_HIP(hipStreamSynchronize(s));
        t->n_gas_leaves = hb[1];
        t->graph_ngb = std::min<int64_t>(
            lcap, t->n_gas_leaves + t->n_gas_leaves / 4 + 1024);
        t->ngb_launch = t->n_gas_leaves;
    } else {
        t->ngb_launch = t->graph_ngb;
        hipLaunchKernelGGL(bound_check_kernel, dim3(1), dim3(1), 0, s, gas_nl,
                           t->graph_ngb, err);
        CRK_HIP(hipGetLastError());
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
