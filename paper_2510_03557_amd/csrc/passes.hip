// The four pair passes of the short-range step: CRKSPH volume/density,
// correction coefficients, hydro forces, and short-range gravity.  Each is a
// per-particle sum phi_i = sum_j phi_ij over the leaf-leaf lists (Eq. (1)).
//
// Kernel shapes (MI355X, wave64).  Default (split): one wavefront owns one
// sub-leaf of <= 16 i-particles with four lanes per particle; it walks the
// parent leaf's list, stages the j particles that survive a cull against
// the sub-leaf box in LDS (coalesced global reads, ballot compaction), and
// lane q of each quad sweeps candidates q, q + 4, ...  Whole-leaf forms:
// one workgroup of BLOCK >= leaf_max threads owns one i-leaf, one particle
// per lane, every lane sweeping every candidate by LDS broadcast.  Either
// way per-particle sums stay in registers and each output is written once
// (no atomics), which keeps results independent of scheduling.
//
// Precision.  Positions are float32 in [1, 2): they are recentred on the
// i-leaf's first particle, e_i = x_i - x_ref and f_j = (x_j - x_ref) + S
// (S the periodic image of the j-leaf), which are exact; so is every
// in-range separation e_i - f_j.  The float32 path sums each tile in plain
// float and folds the tile sum into a compensated (hi, lo) pair with
// TwoSum; the moment-matrix solve runs in double.  The float64 path is
// plain double throughout.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "crk_internal.h"

namespace crk {

namespace {

// --------------------------------------------------------------------------
// arithmetic helpers
// --------------------------------------------------------------------------

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return 1.0 / sqrt(x); }
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp(double x) { return 1.0 / x; }
__device__ inline float fexp(float x) { return __expf(x); }
__device__ inline double fexp(double x) { return exp(x); }

// compensated running sum (float) / plain sum (double)
template <typename T> struct Comp;
template <> struct Comp<float> {
    float hi, lo;
    __device__ void zero() { hi = 0.f; lo = 0.f; }
    __device__ void add(float t) {
        float s = hi + t;
        float bp = s - hi;
        lo += (hi - (s - bp)) + (t - bp);
        hi = s;
    }
    __device__ double value() const { return (double)hi + (double)lo; }
    // adds the running sum of lane (this lane ^ m)
    __device__ void add_lane(int m) {
        const float oh = __shfl_xor(hi, m), ol = __shfl_xor(lo, m);
        add(oh);
        lo += ol;
    }
};
template <> struct Comp<double> {
    double hi;
    __device__ void zero() { hi = 0.0; }
    __device__ void add(double t) { hi += t; }
    __device__ double value() const { return hi; }
    __device__ void add_lane(int m) { hi += __shfl_xor(hi, m); }
};

template <typename T, int N> struct CompArr {
    Comp<T> c[N];
    __device__ void zero() {
#pragma unroll
        for (int k = 0; k < N; ++k) c[k].zero();
    }
    __device__ void fold(T (&t)[N]) {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            c[k].add(t[k]);
            t[k] = T(0);
        }
    }
    // sum over the 4 lanes of each quad (every lane of the quad converged)
    __device__ void quad_reduce() {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            c[k].add_lane(1);
            c[k].add_lane(2);
        }
    }
};

// Cubic spline in units of q = r/h: w(q) (times 1/(pi h^3) gives W) and
// wq(q) = (dw/dq)/q; both vanish for q >= 2.  invq = 1/q (unused for q < 1).
template <typename T>
__device__ inline void spline(T q, T invq, T &w, T &wq) {
    const T t = T(2) - q;
    const T t2 = t * t;
    const bool in = q < T(1);
    const bool on = q < T(2);
    const T w_in = fma(q * q, fma(T(0.75), q, T(-1.5)), T(1));
    const T w_out = T(0.25) * t2 * t;
    const T wq_in = fma(T(2.25), q, T(-3));
    const T wq_out = T(-0.75) * t2 * invq;
    w = in ? w_in : (on ? w_out : T(0));
    wq = in ? wq_in : (on ? wq_out : T(0));
}

constexpr double PI_D = 3.14159265358979323846;

// --------------------------------------------------------------------------
// tree view shared by all passes
// --------------------------------------------------------------------------

template <typename T> struct TreeView {
    const int32_t *leaf_start, *leaf_count, *leaf_box;
    const int64_t *list_off;
    const uint32_t *list;
    const int32_t *n_items;  // device count of work items
    const int32_t *n_leaves; // device count of all leaves
    int64_t list_cap;        // allocated list entries
    const int32_t *perm;
    const T *px, *py, *pz, *h;
    const T *lo, *hi, *hmax;  // leaf boxes (3 planes of lcap) and h_max
    int64_t lcap;
    int xcd_remap;            // map blocks to contiguous leaf ranges per XCD
    int tile;                 // split forms: candidate buffer of tile x 64
                              // (0: the pass's own CAPF)
    int walk_mask;            // passes (bit P::ID) that use the hit walk
    int groups;               // sub-leaf sweep: 1 lane groups, 2 split
    const int32_t *nsub, *sst, *scnt;  // sub-leaves (slots 4*leaf + k)
    const T *slo, *shi, *shm;          // their boxes (3 planes of 4*lcap), h_max
    // dense active groups in place of the sub-leaves: particle k of slot
    // 4*leaf + g is tree slot sidx[16 (4*leaf + g) + k] (NULL: sst + k)
    const int32_t *sidx;
    // the tree's sub-leaves as j-sets (the tables above may hold groups)
    const int32_t *jns, *jst, *jcn;
    const T *jlo, *jhi, *jhm;
    const double *rc, *eps;
    int64_t n_gas;
    // active subset (hierarchical time steps): work item k is leaf items[k]
    // and only slots with act[i] != 0 write outputs; both NULL: all leaves
    const int32_t *items;
    const uint8_t *act;
    // with an active subset and sub-leaves: the sub-leaves (or groups)
    // holding an active particle, entries 4*leaf + g, and their device
    // count for the pass's items (NULL: every sub-leaf of every item)
    const int32_t *slist, *n_slist;
};

// leaf of work item k, and whether slot i writes its outputs
template <typename T> __device__ inline int item_leaf(const TreeView<T> &tv, int k) {
    return tv.items ? tv.items[k] : k;
}
template <typename T> __device__ inline bool slot_active(const TreeView<T> &tv, int i) {
    return !tv.act || tv.act[i] != 0;
}
// tree slot of particle k of sub-leaf (or active group) `slot`
template <typename T>
__device__ inline int sub_slot(const TreeView<T> &tv, int64_t slot, int k) {
    return tv.sidx ? tv.sidx[16 * slot + k] : tv.sst[slot] + k;
}

// a wave-uniform value moved to a scalar register
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline double uni(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// lane k's value (k wave-uniform, in a scalar register): one readlane, no
// LDS round trip as a shuffle would take
__device__ inline int lane_val(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ inline float lane_val(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ inline double lane_val(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sweep forms of the pair kernels
enum { SWEEP_BROADCAST = 0, SWEEP_WALK = 1, SWEEP_GROUPED = 2, SWEEP_SPLIT = 3,
       SWEEP_LEAF = 4 };

__device__ inline void decode_shift(uint32_t code, int &sx, int &sy, int &sz) {
    sx = (int)(code / 9u) - 1;
    sy = (int)((code / 3u) % 3u) - 1;
    sz = (int)(code % 3u) - 1;
}

// Position and the P::NP prefetched fields of slot j: one 16-byte load from
// the pass's packed (x, y, z, field) records where it has them (P::PK),
// else the position planes and P::fetch_j.
template <typename T, typename P>
__device__ __forceinline__ void load_j(T &x, T &y, T &z, T *f,
                                       const typename P::Args &pa,
                                       const TreeView<T> &tv, int j) {
    if constexpr (P::PK) {
        const float4 r = P::packed(pa)[j];
        x = r.x;
        y = r.y;
        z = r.z;
        f[0] = r.w;
    } else {
        x = tv.px[j];
        y = tv.py[j];
        z = tv.pz[j];
        P::fetch_j(f, pa, tv, j);
    }
}

// Walks the list entries [e0, e1) of one leaf.  Each wavefront loads the
// leaf data of 64 entries at once (one entry per lane) and prefetches the
// position and the P::NP prefetched fields of slot js + t of entry k + 1
// while entry k is processed, so the dependent global loads of the walk
// overlap.  visit(js, jc, code, hJ, x, y, z, f) gets the j-leaf's first
// slot, size (clamped to CLAMP), periodic image code, h_max, and the raw
// position and fields of slot js + t for t < jc.  Entries that were never
// written (after a capacity error), and entries for which keep(J, code, hJ)
// is false, are skipped.  Every thread of the workgroup calls visit for
// every entry kept.
template <typename T, typename P, int CLAMP, typename K, typename F>
__device__ __forceinline__ void walk_list(const TreeView<T> &tv,
                                          const typename P::Args &pa,
                                          int64_t e0, int64_t e1, int t,
                                          K &&keep, F &&visit) {
    const int lane = t & 63;
    const int nl = *tv.n_leaves;
    for (int64_t eb = e0; eb < e1; eb += 64) {
        const int nb = (int)min((int64_t)64, e1 - eb);
        int bjs = 0, bjc = 0, bcode = 0;
        T bh = T(0);
        if (lane < nb) {
            const uint32_t ent = tv.list[eb + lane];
            const int J = (int)(ent & LIST_LEAF_MASK);
            if (J < nl) {
                bh = tv.hmax[J];
                bcode = (int)(ent >> LIST_LEAF_BITS);
                if (keep(J, (uint32_t)bcode, bh)) {
                    bjs = tv.leaf_start[J];
                    bjc = min(tv.leaf_count[J], CLAMP);
                }
            }
        }
        // entry values are wave-uniform: read into scalar registers
        int js = lane_val(bjs, 0), jc = lane_val(bjc, 0);
        T nx = T(0), ny = T(0), nz = T(0);
        T nf[P::NP];
#pragma unroll
        for (int u = 0; u < P::NP; ++u) nf[u] = T(0);
        if (t < jc) load_j<T, P>(nx, ny, nz, nf, pa, tv, js + t);
        for (int k = 0; k < nb; ++k) {
            const int cjs = js, cjc = jc;
            const T cx = nx, cy = ny, cz = nz;
            T cf[P::NP];
#pragma unroll
            for (int u = 0; u < P::NP; ++u) cf[u] = nf[u];
            const int code = lane_val(bcode, k);
            const T hJ = lane_val(bh, k);
            if (k + 1 < nb) {
                js = lane_val(bjs, k + 1);
                jc = lane_val(bjc, k + 1);
                if (t < jc) load_j<T, P>(nx, ny, nz, nf, pa, tv, js + t);
            }
            if (cjc == 0) continue;
            visit(cjs, cjc, (uint32_t)code, hJ, cx, cy, cz, cf);
        }
    }
}

// The common driver: P supplies the per-pass state and arithmetic.
//   P::NJ        number of T fields staged per j particle
//   P::I         per-lane i-state
//   P::load_i(I&, args, tv, i, ex, ey, ez, box)
//   P::NP, P::fetch_j(T f[NP], args, tv, j)  fields loaded with the position
//   P::store_j(T* dst, f, args, tv, j, fx, fy, fz)  stage a culling survivor
//   P::range(args, tv, box, hmax_I, hmax_J)  interaction range of a leaf pair
//   P::Tile / P::Acc  per-sweep sums and compensated totals
//   P::pair(Tile&, const I&, const T* jd, bool self)
//   P::finish(const Acc&, const I&, args, tv, i)
//
// Every j particle of a listed j-leaf is first tested against the i-set's
// bounding box widened by the pair range; survivors are compacted (ballot +
// prefix) into an LDS buffer of CAPF*BLOCK candidates that spans several
// j-leaves.  A full buffer is swept and its partial sums are folded into
// the compensated totals.  Culled particles are out of range of every i,
// so the sums do not change beyond rounding order.
template <typename T, typename P, int BLOCK, int MODE>
__device__ __forceinline__ void process_leaf(const TreeView<T> &tv,
                                             const typename P::Args &pa,
                                             const int I, T *sj, int *sjid,
                                             int *wcnt, uint32_t *smask,
                                             short *glist) {
    constexpr int CAP = P::CAPF * BLOCK;
    constexpr int NW = BLOCK / 64;
    const int st = tv.leaf_start[I];
    // a leaf above BLOCK exists only after a capacity error (already
    // latched); clamping keeps every access inside the LDS buffer
    const int cnt = min(tv.leaf_count[I], BLOCK);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // lane groups: with sub-leaves, lanes 16g..16g+15 hold sub-leaf g
    const bool grouped = MODE == SWEEP_GROUPED;
    const int ns = grouped ? tv.nsub[I] : 1;
    const int g = grouped ? (t >> 4) : 0;
    const int64_t slot = 4 * (int64_t)I + g;
    const bool act = grouped ? (g < ns && (t & 15) < tv.scnt[g < ns ? slot : 4 * (int64_t)I])
                             : (t < cnt);
    const int i = act ? (grouped ? sub_slot(tv, slot, t & 15) : st + t) : st;
    const T rx = tv.px[st], ry = tv.py[st], rz = tv.pz[st];
    const int box = tv.leaf_box[I];
    // i-leaf box relative to the reference particle (exact in float32)
    const T blx = tv.lo[I] - rx, bly = tv.lo[tv.lcap + I] - ry,
            blz = tv.lo[2 * tv.lcap + I] - rz;
    const T bhx = tv.hi[I] - rx, bhy = tv.hi[tv.lcap + I] - ry,
            bhz = tv.hi[2 * tv.lcap + I] - rz;
    const T hmI = tv.hmax[I];
    typename P::I is;
    P::load_i(is, pa, tv, i, tv.px[i] - rx, tv.py[i] - ry, tv.pz[i] - rz, box);
    typename P::Tile tile;
    tile.zero();
    typename P::Acc acc;
    acc.zero();
    // after a capacity error (latched by the list builder) offsets may run
    // past the allocation: clamp, and skip entries that were never written
    const int64_t e0 = min(tv.list_off[I], tv.list_cap);
    const int64_t e1 = min(tv.list_off[I + 1], tv.list_cap);
    int nbuf = 0;
    // Sweep of a full buffer.  Broadcast form: every lane evaluates every
    // candidate (LDS broadcast reads); the pair function applies the exact
    // range test and the wave skips the arithmetic when no lane is in range.
    // Walk form (MODE SWEEP_WALK): every lane first tests all
    // candidates against its own particle and stores a hit bitmask in LDS,
    // then walks its own hits in candidate order with per-lane reads, so the
    // pair arithmetic runs only for in-range pairs; the wave loops while any
    // lane has hits left.  Buffers where hits are dense (at least a quarter
    // of lane x candidate pairs) use the broadcast form.  Every lane meets
    // its hits in candidate order either way, so the sums are the same.
    const int lanes = __popcll(__ballot(act));  // active lanes of this wave
    constexpr bool walk = MODE == SWEEP_WALK;
    auto sweep = [&](int n) {
        __syncthreads();
        bool broadcast = true;
        if (walk && n > 0) {
            const int nw = (n + 31) / 32;
            int hits = 0;
            for (int w = 0; w < nw; ++w) {
                uint32_t bits = 0;
                for (int b = 0; b < 32; ++b) {
                    const int k = w * 32 + b;
                    if (k >= n) break;
                    const bool hit =
                        act && P::test(is, &sj[k * P::NJ], sjid[k] == i);
                    bits |= (uint32_t)hit << b;
                }
                smask[w * BLOCK + t] = bits;
                hits += __popc(bits);
            }
            int tot = hits;  // wave total (all lanes converged here)
            for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
            broadcast = 4 * tot >= lanes * n;
            if (!broadcast) {
                int w = 0;
                uint32_t mm = smask[t];
                while (true) {
                    while (mm == 0u && w + 1 < nw) {
                        ++w;
                        mm = smask[w * BLOCK + t];
                    }
                    const bool has = mm != 0u;
                    if (!__any(has)) break;
                    if (has) {
                        const int k = w * 32 + __ffs(mm) - 1;
                        mm &= mm - 1u;
                        P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                    }
                }
            }
        }
        if (MODE == SWEEP_GROUPED && broadcast && n > 0) {
            // per sub-leaf candidate lists (ballot compaction, in order)
            int len[4] = {0, 0, 0, 0};
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                if (gg >= ns) break;
                const int64_t sg = 4 * (int64_t)I + gg;
                const T gl0 = tv.slo[sg] - rx, gl1 = tv.slo[4 * tv.lcap + sg] - ry,
                        gl2 = tv.slo[8 * tv.lcap + sg] - rz;
                const T gh0 = tv.shi[sg] - rx, gh1 = tv.shi[4 * tv.lcap + sg] - ry,
                        gh2 = tv.shi[8 * tv.lcap + sg] - rz;
                const T hg = tv.shm[sg];
                int l = 0;
                for (int base = 0; base < n; base += 64) {
                    const int k = base + lane;
                    bool hit = false;
                    if (k < n) {
                        const T *jd = &sj[k * P::NJ];
                        const T R = P::sub_range(pa, tv, box, hg, jd);
                        const T dx = fmax(fmax(gl0 - jd[0], jd[0] - gh0), T(0));
                        const T dy = fmax(fmax(gl1 - jd[1], jd[1] - gh1), T(0));
                        const T dz = fmax(fmax(gl2 - jd[2], jd[2] - gh2), T(0));
                        hit = dx * dx + dy * dy + dz * dz < R * R;
                    }
                    const uint64_t mk = __ballot(hit);
                    if (hit) glist[gg * CAP + l + __popcll(mk & lt_mask)] = (short)k;
                    l += __popcll(mk);
                }
                len[gg] = l;
            }
            __syncthreads();
            const int maxlen = max(max(len[0], len[1]), max(len[2], len[3]));
            const int mylen = g == 0 ? len[0] : (g == 1 ? len[1] : (g == 2 ? len[2] : len[3]));
            for (int it = 0; it < maxlen; ++it) {
                if (act && it < mylen) {
                    const int k = glist[g * CAP + it];
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            }
        } else if (broadcast) {
            // every lane runs the loop (an inactive lane holds a valid
            // particle and its sums are never written), so the loop is
            // uniform; unrolled by 4 so that the LDS reads of several
            // candidates are in flight together
            int k = 0;
            for (; k + 4 <= n; k += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    P::pair(tile, is, &sj[(k + u) * P::NJ], sjid[k + u] == i);
            }
            for (; k < n; ++k)
                P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
        }
        acc.fold(tile);
        __syncthreads();
    };
    // the leaf's list holds exactly the j-leaves in range of its box
    auto keep_all = [](int, uint32_t, T) { return true; };
    walk_list<T, P, BLOCK>(tv, pa, e0, e1, t, keep_all,
                           [&](int js, int jc, uint32_t code, T hJ, T x, T y,
                               T z, const T *f) {
        int sx, sy, sz;
        decode_shift(code, sx, sy, sz);
        if (nbuf + jc > CAP) {
            sweep(nbuf);
            nbuf = 0;
        }
        const T R = P::range(pa, tv, box, hmI, hJ);
        const T R2 = R * R;
        bool keep = false;
        T fx = T(0), fy = T(0), fz = T(0);
        const int j = js + t;
        if (t < jc) {
            fx = (x - rx) + T(sx);
            fy = (y - ry) + T(sy);
            fz = (z - rz) + T(sz);
            const T dx = fmax(fmax(blx - fx, fx - bhx), T(0));
            const T dy = fmax(fmax(bly - fy, fy - bhy), T(0));
            const T dz = fmax(fmax(blz - fz, fz - bhz), T(0));
            keep = dx * dx + dy * dy + dz * dz < R2;
        }
        const uint64_t m = __ballot(keep);
        int off = __popcll(m & lt_mask);
        int tot = __popcll(m);
        if (NW > 1) {
            if (lane == 0) wcnt[wave] = tot;
            __syncthreads();
            tot = 0;
            for (int w = 0; w < NW; ++w) {
                if (w < wave) off += wcnt[w];
                tot += wcnt[w];
            }
            __syncthreads();
        }
        if (keep) {
            const int pos = nbuf + off;
            P::store_j(&sj[pos * P::NJ], f, pa, tv, j, fx, fy, fz);
            sjid[pos] = j;
        }
        nbuf += tot;
    });
    sweep(nbuf);
    if (act && slot_active(tv, i)) P::finish(acc, is, pa, tv, i);
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2.  Remapping block b (on XCD b % 8) to a contiguous range
// of leaves per XCD keeps spatial neighbours -- which share j-leaves -- in
// the same L2.  A bijection of [0, G) for any G.
__device__ inline int xcd_block(int b, int G) {
    constexpr int NX = 8;
    const int q = G / NX, r = G % NX;
    const int x = b % NX, k = b / NX;
    return x * q + min(x, r) + k;
}

// One workgroup per leaf (leaf order remapped per XCD).  MODE selects the
// sweep form; the walk and group forms exist for BLOCK 64 only.
template <typename T, typename P, int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void pair_kernel(const TreeView<T> tv,
                                                     const typename P::Args pa) {
    static_assert(MODE == SWEEP_BROADCAST || BLOCK == 64, "64-lane forms");
    __shared__ __attribute__((aligned(16))) T sj[P::CAPF * BLOCK * P::NJ];
    __shared__ int sjid[P::CAPF * BLOCK];
    __shared__ int wcnt[BLOCK / 64];
    __shared__ uint32_t smask[MODE == SWEEP_WALK ? P::CAPF * BLOCK / 32 * BLOCK : 1];
    __shared__ short glist[MODE == SWEEP_GROUPED ? 4 * P::CAPF * BLOCK : 1];
    // the grid may exceed the device-side leaf count (graph capture sizes it
    // by capacity): surplus blocks leave first, the remap covers [0, n)
    const int n_items = *tv.n_items;
    if ((int)blockIdx.x >= n_items) return;
    const int I = item_leaf(tv, tv.xcd_remap ? xcd_block(blockIdx.x, n_items)
                                             : (int)blockIdx.x);
    process_leaf<T, P, BLOCK, MODE>(tv, pa, I, sj, sjid, wcnt, smask, glist);
}

// Candidate buffer of the split forms: tile x 64 records (the pass's CAPF
// when no tile is set), capped at 64 KiB of LDS with the record ids.
template <typename T, typename P> __host__ __device__ constexpr int split_cap_of(int tile) {
    const int want = (tile > 0 ? tile : P::CAPF) * 64;
    const int most = 65536 / (P::NJ * (int)sizeof(T) + 4) / 64 * 64;
    return want < most ? want : most;
}
template <typename T, typename P> __device__ inline int split_cap(const TreeView<T> &tv) {
    return split_cap_of<T, P>(tv.tile);
}

// Split forms: one wavefront per sub-leaf (<= 16 particles).  The wave
// walks the parent leaf's list sixteen entries at a time: lane l tests
// sub-leaf l % 4 of the j-leaf of entry l / 4 (the tree's sub-leaves, in
// the entry's periodic image) against this sub-leaf's box widened by the
// pair range, so that only j sub-leaves in range are read.  The survivors
// are then taken four at a time, sixteen lanes each (lane 16 g + p reads
// particle p of the g-th), while the next four are being loaded; every j
// particle is culled against the box and the survivors are staged,
// recentred on the parent leaf's first particle as in the other forms, in
// an LDS buffer of P::CAPF * 64 candidates; sweep(n) consumes a full
// buffer.  Packing sub-leaves of different j-leaves into one round cuts
// the rounds to about two thirds of one per j-leaf.
template <typename T, typename P, typename Sweep>
__device__ __forceinline__ void stage_subleaf(const TreeView<T> &tv,
                                              const typename P::Args &pa,
                                              const int I, const int64_t slot,
                                              T *sj, int *sjid, Sweep &&sweep) {
    const int CAP = split_cap<T, P>(tv);
    const int lane = threadIdx.x;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int st = tv.leaf_start[I];
    const T rx = tv.px[st], ry = tv.py[st], rz = tv.pz[st];
    const int box = tv.leaf_box[I];
    const int64_t sl = 4 * tv.lcap;
    const T hmS = tv.shm[slot];
    const int64_t e0 = min(tv.list_off[I], tv.list_cap);
    const int64_t e1 = min(tv.list_off[I + 1], tv.list_cap);
    const int nl = *tv.n_leaves;
    const T slx = tv.slo[slot], sly = tv.slo[sl + slot], slz = tv.slo[2 * sl + slot];
    const T shx = tv.shi[slot], shy = tv.shi[sl + slot], shz = tv.shi[2 * sl + slot];
    // with P::FARNEAR, candidates at least P::far_range from the box go to
    // the front of the buffer ([0, nbuf)), the others to its back
    // ([CAP - nnear, CAP)), and sweep(nbuf, nnear) takes both ranges
    int nbuf = 0, nnear = 0;
    T Rf2 = T(0);
    if constexpr (P::FARNEAR) {
        const T Rf = P::far_range(tv, box);
        Rf2 = Rf * Rf;
    }
    // the pair range, when it does not depend on the j side
    const T Rc = P::RANGE_HJ ? T(0) : P::range(pa, tv, box, hmS, T(0)) + T(1e-6);
    const int g = lane >> 4, p = lane & 15;

    // the next four surviving sub-leaves of mask `rem` (wave-uniform, lanes
    // of the entry-side values js, jc, code, hJ): group g of the wavefront
    // takes the g-th and loads its particle p
    auto fetch = [&](uint64_t &rem, int js, int jc, int code, T hJ, int &gjs,
                     int &gjc, int &gcode, T &ghJ, T &x, T &y, T &z, T *f) {
        int src[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            src[k] = rem ? __builtin_ctzll(rem) : -1;
            rem &= rem - 1;  // (0 stays 0)
        }
        const int s = g == 0 ? src[0] : g == 1 ? src[1] : g == 2 ? src[2] : src[3];
        const int sr = s < 0 ? 0 : s;
        // every lane takes part in every shuffle (a shuffle under a
        // condition reads nothing from the lanes the condition leaves out)
        const int vjs = __shfl(js, sr);
        const int vjc = __shfl(jc, sr);
        const int vcode = __shfl(code, sr);
        T vhJ = T(0);
        if constexpr (P::RANGE_HJ) vhJ = __shfl(hJ, sr);
        gjs = vjs;
        gjc = s < 0 ? 0 : vjc;
        gcode = vcode;
        ghJ = vhJ;
        x = y = z = T(0);
#pragma unroll
        for (int u = 0; u < P::NP; ++u) f[u] = T(0);
        if (p < gjc) load_j<T, P>(x, y, z, f, pa, tv, gjs + p);
    };
    // cull one round's particles against the box moved to their images
    // (the shifted bounds round by at most a few 1e-7: the range gets an
    // absolute 1e-6 on top of its relative widening) and stage survivors
    auto stage = [&](int cjs, int cjc, int ccode, T chJ, T x, T y, T z,
                     const T *f) {
        int sx, sy, sz;
        decode_shift((uint32_t)ccode, sx, sy, sz);
        const T R = P::RANGE_HJ ? P::range(pa, tv, box, hmS, chJ) + T(1e-6) : Rc;
        const T R2 = R * R;
        // every lane computes the distance (lanes past the sub-leaf's count
        // hold zero coordinates: arithmetic only, no access)
        const T dx = fmax(fmax((slx - T(sx)) - x, x - (shx - T(sx))), T(0));
        const T dy = fmax(fmax((sly - T(sy)) - y, y - (shy - T(sy))), T(0));
        const T dz = fmax(fmax((slz - T(sz)) - z, z - (shz - T(sz))), T(0));
        const T d2 = dx * dx + dy * dy + dz * dz;
        const bool keep = (p < cjc) & (d2 < R2);
        const int j = cjs + p;
        const T fx = (x - rx) + T(sx), fy = (y - ry) + T(sy), fz = (z - rz) + T(sz);
        if constexpr (P::FARNEAR) {
            const bool far = keep & (d2 >= Rf2);
            const uint64_t mf = __ballot(far), mn = __ballot(keep && !far);
            if (nbuf + nnear + __popcll(mf) + __popcll(mn) > CAP) {
                sweep(nbuf, nnear);
                nbuf = 0;
                nnear = 0;
            }
            if (keep) {
                const int pos = far ? nbuf + __popcll(mf & lt_mask)
                                    : CAP - 1 - (nnear + __popcll(mn & lt_mask));
                P::store_j(&sj[pos * P::NJ], f, pa, tv, j, fx, fy, fz);
                sjid[pos] = j;
            }
            nbuf += __popcll(mf);
            nnear += __popcll(mn);
        } else {
            const uint64_t m = __ballot(keep);
            if (nbuf + __popcll(m) > CAP) {
                sweep(nbuf);
                nbuf = 0;
            }
            if (keep) {
                // recentred (exact for every pair in range)
                const int pos = nbuf + __popcll(m & lt_mask);
                P::store_j(&sj[pos * P::NJ], f, pa, tv, j, fx, fy, fz);
                sjid[pos] = j;
            }
            nbuf += __popcll(m);
        }
    };

    for (int64_t eb = e0; eb < e1; eb += 16) {
        // lane l: sub-leaf l % 4 of entry eb + l / 4.  Entries never written
        // (after a capacity error) name no leaf below the leaf count and are
        // skipped.  The box gap is computed in T from coordinates in [1, 2)
        // shifted by at most one box (a few ulp of error at most), against
        // the pair range widened by 1e-4 relative plus 1e-6 absolute, so
        // nothing in range is dropped.
        const int64_t e = eb + (lane >> 2);
        const int s = lane & 3;
        int js = 0, jc = 0, code = 0;
        T hJ = T(0);
        bool in = false;
        if (e < e1) {
            const uint32_t ent = tv.list[e];
            const int J = (int)(ent & LIST_LEAF_MASK);
            if (J < nl && s < tv.jns[J]) {
                code = (int)(ent >> LIST_LEAF_BITS);
                int sx, sy, sz;
                decode_shift((uint32_t)code, sx, sy, sz);
                const int64_t q = 4 * (int64_t)J + s;
                hJ = tv.jhm[q];
                const T gx = fmax(T(0), fmax((tv.jlo[q] + T(sx)) - shx,
                                             slx - (tv.jhi[q] + T(sx))));
                const T gy = fmax(T(0), fmax((tv.jlo[sl + q] + T(sy)) - shy,
                                             sly - (tv.jhi[sl + q] + T(sy))));
                const T gz = fmax(T(0), fmax((tv.jlo[2 * sl + q] + T(sz)) - shz,
                                             slz - (tv.jhi[2 * sl + q] + T(sz))));
                const T R = P::range(pa, tv, box, hmS, hJ) * T(1.0001) + T(1e-6);
                if (gx * gx + gy * gy + gz * gz < R * R) {
                    js = tv.jst[q];
                    jc = min(tv.jcn[q], 16);
                    in = jc > 0;
                }
            }
        }
        uint64_t rem = __ballot(in);
        if (rem == 0) continue;
        int cjs, cjc, ccode;
        T chJ, cx, cy, cz, cf[P::NP];
        fetch(rem, js, jc, code, hJ, cjs, cjc, ccode, chJ, cx, cy, cz, cf);
        while (true) {
            const bool more = rem != 0;
            int njs = 0, njc = 0, ncode = 0;
            T nhJ = T(0), nx = T(0), ny = T(0), nz = T(0), nf[P::NP];
#pragma unroll
            for (int u = 0; u < P::NP; ++u) nf[u] = T(0);
            if (more) fetch(rem, js, jc, code, hJ, njs, njc, ncode, nhJ, nx, ny, nz, nf);
            stage(cjs, cjc, ccode, chJ, cx, cy, cz, cf);
            if (!more) break;
            cjs = njs;
            cjc = njc;
            ccode = ncode;
            chJ = nhJ;
            cx = nx;
            cy = ny;
            cz = nz;
#pragma unroll
            for (int u = 0; u < P::NP; ++u) cf[u] = nf[u];
        }
    }
    if constexpr (P::FARNEAR) sweep(nbuf, nnear);
    else sweep(nbuf);
}

// Quad form: four lanes per particle.  Lane q of a particle's quad takes
// candidates q, q + 4, ... of each buffer; the quad's compensated sums are
// combined at the end and lane 0 of the quad writes the outputs.
template <typename T, typename P>
__device__ __forceinline__ void process_subleaf(const TreeView<T> &tv,
                                                const typename P::Args &pa,
                                                const int I, const int g,
                                                T *sj, int *sjid) {
    const int lane = threadIdx.x;
    const int64_t slot = 4 * (int64_t)I + g;
    const int scnt = min(tv.scnt[slot], 16);
    const int ii = lane >> 2, q = lane & 3;
    const bool act = ii < scnt;
    const int i = sub_slot(tv, slot, act ? ii : 0);
    const int st = tv.leaf_start[I];
    const T rx = tv.px[st], ry = tv.py[st], rz = tv.pz[st];
    const int box = tv.leaf_box[I];
    typename P::I is;
    P::load_i(is, pa, tv, i, tv.px[i] - rx, tv.py[i] - ry, tv.pz[i] - rz, box);
    typename P::Tile tile;
    tile.zero();
    typename P::Acc acc;
    acc.zero();
    auto sweep = [&](int n) {
        __syncthreads();
        // every lane runs the loop (inactive lanes hold a valid particle
        // whose sums are never written)
        if constexpr (P::MASKED) {
            // two phases: the range test of every candidate of the lane
            // (k = 4 t + q) sets bit t of a mask, then the lane evaluates
            // its in-range candidates in ascending t.  The pair body runs
            // on in-range pairs only, and each lane adds its pairs in the
            // same order as a plain sweep that skips the out-of-range ones.
            using M = uint64_t;
            constexpr int MB = 64;
            const int nt = (n + 3) >> 2;  // candidate slots per lane (CAP % 4 == 0)
            for (int t0 = 0; t0 < nt; t0 += MB) {
                const int tn = min(nt - t0, MB);
                M m = 0;
                int t = 0;
                for (; t + 4 <= tn; t += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int k = 4 * (t0 + t + u) + q;
                        const bool c = P::test(is, &sj[k * P::NJ], sjid[k] == i);
                        m |= M((k < n) & c) << (t + u);
                    }
                }
                for (; t < tn; ++t) {
                    const int k = 4 * (t0 + t) + q;
                    const bool c = P::test(is, &sj[k * P::NJ], sjid[k] == i);
                    m |= M((k < n) & c) << t;
                }
                while (m) {
                    const int b = __builtin_ctzll(m);
                    m &= m - 1;
                    const int k = 4 * (t0 + b) + q;
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            }
        } else {
            // blocks of 16 candidates unrolled
            int k0 = 0;
            for (; k0 + 16 <= n; k0 += 16) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = k0 + 4 * u + q;
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            }
            for (int k = k0 + q; k < n; k += 4)
                P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
        }
        acc.fold(tile);
        __syncthreads();
    };
    if constexpr (P::FARNEAR) {
        // far candidates ([0, nf)) with the far pair body, near ones
        // ([CAP - nn, CAP)) with the full one; the same quad sweep on each
        const int CAP = split_cap<T, P>(tv);
        auto sweep2 = [&](int nf, int nn) {
            __syncthreads();
            int k0 = 0;
            for (; k0 + 16 <= nf; k0 += 16) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    P::pair_far(tile, is, &sj[(k0 + 4 * u + q) * P::NJ]);
            }
            for (int k = k0 + q; k < nf; k += 4) P::pair_far(tile, is, &sj[k * P::NJ]);
            const int b0 = CAP - nn;
            k0 = b0;
            for (; k0 + 16 <= CAP; k0 += 16) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = k0 + 4 * u + q;
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            }
            for (int k = k0 + q; k < CAP; k += 4)
                P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
            acc.fold(tile);
            __syncthreads();
        };
        stage_subleaf<T, P>(tv, pa, I, slot, sj, sjid, sweep2);
    } else {
        stage_subleaf<T, P>(tv, pa, I, slot, sj, sjid, sweep);
    }
    acc.quad_reduce();
    if (act && q == 0 && slot_active(tv, i)) P::finish(acc, is, pa, tv, i);
}

// One wavefront per sub-leaf: block b -> leaf b / 4, sub-leaf b % 4.
// (the candidate buffer lives in dynamic LDS, sized at launch for the tile)
// Waves per SIMD a pass asks of its split kernel (P::MINW; default: the
// compiler's choice)
template <typename P, typename = void> struct MinWaves {
    static constexpr int v = 1;
};
template <typename P> struct MinWaves<P, std::void_t<decltype(P::MINW)>> {
    static constexpr int v = P::MINW;
};
template <typename T, typename P>
__global__ __launch_bounds__(64, MinWaves<P>::v) void pair_kernel_split(const TreeView<T> tv,
                                                        const typename P::Args pa) {
    extern __shared__ __attribute__((aligned(16))) unsigned char split_lds[];
    T *sj = reinterpret_cast<T *>(split_lds);
    int *sjid = reinterpret_cast<int *>(sj + split_cap<T, P>(tv) * P::NJ);
    int I, g;
    if (tv.slist) {
        // active subset: one wavefront per listed sub-leaf, every one of
        // which holds an active particle (no idle workgroups in the grid,
        // whose regular pattern would leave CUs without work)
        const int n = *tv.n_slist;
        if ((int)blockIdx.x >= n) return;
        const int e = tv.slist[tv.xcd_remap ? xcd_block(blockIdx.x, n)
                                            : (int)blockIdx.x];
        I = e >> 2;
        g = e & 3;
    } else {
        const int n_items = *tv.n_items;
        if ((int)blockIdx.x >= 4 * n_items) return;
        const int b = tv.xcd_remap ? xcd_block(blockIdx.x, 4 * n_items)
                                   : (int)blockIdx.x;
        I = item_leaf(tv, b >> 2);
        g = b & 3;
        if (g >= tv.nsub[I]) return;
    }
    if (tv.act && !tv.slist) {
        // active subset: a sub-leaf without active particles has nothing
        // to write (the whole wavefront leaves together)
        const int64_t sl = 4 * (int64_t)I + g;
        const int lane = threadIdx.x;
        const bool a = lane < min(tv.scnt[sl], 16) && tv.act[sub_slot(tv, sl, lane)];
        if (__ballot(a) == 0) return;
    }
    process_subleaf<T, P>(tv, pa, I, g, sj, sjid);
}

// Persistent split form: each 64-thread workgroup pops sub-leaf slots from
// an atomic counter (reset to 0 before the launch) until the queue is
// exhausted; slot q is sub-leaf q % 4 of the leaf of rank q / 4 in
// decreasing cost, so the longest items start first and the sub-leaves of
// one leaf run side by side.  Every workgroup leaves the loop once the
// counter passes the slot count.
template <typename T, typename P>
__global__ __launch_bounds__(64) void pair_kernel_split_queue(
    const TreeView<T> tv, const typename P::Args pa,
    const int32_t *__restrict__ order, int *__restrict__ head) {
    extern __shared__ __attribute__((aligned(16))) unsigned char split_lds[];
    T *sj = reinterpret_cast<T *>(split_lds);
    int *sjid = reinterpret_cast<int *>(sj + split_cap<T, P>(tv) * P::NJ);
    const int n_slots = 4 * *tv.n_items;
    while (true) {
        int q = 0;
        if (threadIdx.x == 0) q = atomicAdd(head, 1);
        q = uni(__shfl(q, 0));
        if (q >= n_slots) break;
        const int I = order[q >> 2], g = q & 3;
        if (g >= tv.nsub[I]) continue;
        process_subleaf<T, P>(tv, pa, I, g, sj, sjid);
    }
}

// Leaf form: one workgroup of four wavefronts per leaf, wavefront w owning
// sub-leaf w.  The four wavefronts walk the leaf's list together, four
// entries per round (entry e0 + 4 r + w by wavefront w), cull each j
// particle against the leaf box widened by the pair range and stage the
// survivors once, for all four sub-leaves, in a shared LDS buffer (in
// round order, wavefront by wavefront).  A full buffer is swept: every
// wavefront culls the staged candidates against its own sub-leaf box into an
// index list (far and near lists with P::FARNEAR) and sweeps that list with
// four lanes per particle as the split form does.  Staging once per leaf
// reads each listed j-leaf from memory once per leaf instead of once per
// sub-leaf.  Every wavefront reaches every barrier: the rounds and sweeps
// are uniform over the workgroup.
template <typename P> constexpr int leaf_cap() {
    return (P::CAPF * 128 > 256) ? P::CAPF * 128 : 256;
}

template <typename T, typename P>
__device__ __forceinline__ void process_leaf4(const TreeView<T> &tv,
                                              const typename P::Args &pa,
                                              const int I, T *sj, int *sjid,
                                              unsigned short (*slist)[leaf_cap<P>()],
                                              int *wcnt) {
    constexpr int CAPL = leaf_cap<P>();
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int ns = tv.nsub[I];
    const int64_t slot = 4 * (int64_t)I + (w < ns ? w : 0);
    const int scnt = w < ns ? min(tv.scnt[slot], 16) : 0;
    const int ii = lane >> 2, q = lane & 3;
    const bool act = ii < scnt;
    const int i = sub_slot(tv, slot, act ? ii : 0);
    // a wavefront sweeps when its sub-leaf exists and, with an active
    // subset, holds an active particle
    bool sweeper = w < ns;
    if (sweeper && tv.act) sweeper = __ballot(act && tv.act[i] != 0) != 0;
    const int st = tv.leaf_start[I];
    const T rx = tv.px[st], ry = tv.py[st], rz = tv.pz[st];
    const int box = tv.leaf_box[I];
    const T hmI = tv.hmax[I];
    const int64_t lc = tv.lcap, sl = 4 * tv.lcap;
    const T llx = tv.lo[I], lly = tv.lo[lc + I], llz = tv.lo[2 * lc + I];
    const T lhx = tv.hi[I], lhy = tv.hi[lc + I], lhz = tv.hi[2 * lc + I];
    // the sub-leaf box relative to the reference particle (the frame of the
    // staged candidates; a few ulp of rounding, covered by the ranges'
    // relative widening and an absolute 1e-6)
    const T gl0 = tv.slo[slot] - rx, gl1 = tv.slo[sl + slot] - ry,
            gl2 = tv.slo[2 * sl + slot] - rz;
    const T gh0 = tv.shi[slot] - rx, gh1 = tv.shi[sl + slot] - ry,
            gh2 = tv.shi[2 * sl + slot] - rz;
    const T hg = tv.shm[slot];
    typename P::I is;
    P::load_i(is, pa, tv, i, tv.px[i] - rx, tv.py[i] - ry, tv.pz[i] - rz, box);
    typename P::Tile tile;
    tile.zero();
    typename P::Acc acc;
    acc.zero();
    T Rf2 = T(0);
    if constexpr (P::FARNEAR) {
        const T Rf = P::far_range(tv, box);
        Rf2 = Rf * Rf;
    }
    unsigned short *my = slist[w];
    auto sweep = [&](int n) {
        __syncthreads();  // the staged candidates are complete
        int nf = 0, nn = 0;
        if (sweeper) {
            for (int base = 0; base < n; base += 64) {
                const int k = base + lane;
                bool keep = false, far = false;
                if (k < n) {
                    const T *jd = &sj[k * P::NJ];
                    const T R = P::sub_range(pa, tv, box, hg, jd) + T(1e-6);
                    const T dx = fmax(fmax(gl0 - jd[0], jd[0] - gh0), T(0));
                    const T dy = fmax(fmax(gl1 - jd[1], jd[1] - gh1), T(0));
                    const T dz = fmax(fmax(gl2 - jd[2], jd[2] - gh2), T(0));
                    const T d2 = dx * dx + dy * dy + dz * dz;
                    keep = d2 < R * R;
                    if constexpr (P::FARNEAR) far = keep && d2 >= Rf2;
                }
                if constexpr (P::FARNEAR) {
                    const uint64_t mf = __ballot(far), mn = __ballot(keep && !far);
                    if (far) my[nf + __popcll(mf & lt_mask)] = (unsigned short)k;
                    else if (keep)
                        my[CAPL - 1 - (nn + __popcll(mn & lt_mask))] = (unsigned short)k;
                    nf += __popcll(mf);
                    nn += __popcll(mn);
                } else {
                    const uint64_t m = __ballot(keep);
                    if (keep) my[nf + __popcll(m & lt_mask)] = (unsigned short)k;
                    nf += __popcll(m);
                }
            }
        }
        __syncthreads();  // every list is complete
        if (sweeper) {
            if constexpr (P::FARNEAR) {
                int u0 = 0;
                for (; u0 + 16 <= nf; u0 += 16) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        P::pair_far(tile, is, &sj[my[u0 + 4 * u + q] * P::NJ]);
                }
                for (int u = u0 + q; u < nf; u += 4)
                    P::pair_far(tile, is, &sj[my[u] * P::NJ]);
                u0 = CAPL - nn;
                for (; u0 + 16 <= CAPL; u0 += 16) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int k = my[u0 + 4 * u + q];
                        P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                    }
                }
                for (int u = u0 + q; u < CAPL; u += 4) {
                    const int k = my[u];
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            } else if constexpr (P::MASKED) {
                // test, then pairs (the split form's two phases, over the list)
                const int nt = (nf + 3) >> 2;
                for (int t0 = 0; t0 < nt; t0 += 64) {
                    const int tn = min(nt - t0, 64);
                    uint64_t m = 0;
                    for (int tt = 0; tt < tn; ++tt) {
                        const int u = 4 * (t0 + tt) + q;
                        const int k = my[u < nf ? u : 0];
                        const bool c = P::test(is, &sj[k * P::NJ], sjid[k] == i);
                        m |= uint64_t((u < nf) & c) << tt;
                    }
                    while (m) {
                        const int b = __builtin_ctzll(m);
                        m &= m - 1;
                        const int k = my[4 * (t0 + b) + q];
                        P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                    }
                }
            } else {
                int u0 = 0;
                for (; u0 + 16 <= nf; u0 += 16) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int k = my[u0 + 4 * u + q];
                        P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                    }
                }
                for (int u = u0 + q; u < nf; u += 4) {
                    const int k = my[u];
                    P::pair(tile, is, &sj[k * P::NJ], sjid[k] == i);
                }
            }
        }
        acc.fold(tile);
        __syncthreads();  // the buffer may be refilled
    };
    // after a capacity error (latched by the list builder) offsets may run
    // past the allocation: clamp, and skip entries that were never written
    const int64_t e0 = min(tv.list_off[I], tv.list_cap);
    const int64_t e1 = min(tv.list_off[I + 1], tv.list_cap);
    const int nl = *tv.n_leaves;
    int nbuf = 0;
    for (int64_t eb = e0; eb < e1; eb += 4) {
        const int64_t e = eb + w;
        int js = 0, jc = 0, sx = 0, sy = 0, sz = 0;
        T hJ = T(0);
        if (e < e1) {
            const uint32_t ent = tv.list[e];
            const int J = (int)(ent & LIST_LEAF_MASK);
            if (J < nl) {
                hJ = tv.hmax[J];
                decode_shift(ent >> LIST_LEAF_BITS, sx, sy, sz);
                js = tv.leaf_start[J];
                jc = min(tv.leaf_count[J], 64);
            }
        }
        js = uni(js);
        jc = uni(jc);
        bool keep = false;
        T x = T(0), y = T(0), z = T(0);
        T f[P::NP];
#pragma unroll
        for (int u = 0; u < P::NP; ++u) f[u] = T(0);
        if (lane < jc) {
            x = tv.px[js + lane];
            y = tv.py[js + lane];
            z = tv.pz[js + lane];
            P::fetch_j(f, pa, tv, js + lane);
            // cull in raw coordinates against the leaf box moved to this
            // image (absolute 1e-6 for the rounding of its shifted bounds)
            const T R = P::range(pa, tv, box, hmI, hJ) + T(1e-6);
            const T dx = fmax(fmax((llx - T(sx)) - x, x - (lhx - T(sx))), T(0));
            const T dy = fmax(fmax((lly - T(sy)) - y, y - (lhy - T(sy))), T(0));
            const T dz = fmax(fmax((llz - T(sz)) - z, z - (lhz - T(sz))), T(0));
            keep = dx * dx + dy * dy + dz * dz < R * R;
        }
        const uint64_t m = __ballot(keep);
        if (lane == 0) wcnt[w] = __popcll(m);
        __syncthreads();
        const int c0 = wcnt[0], c1 = wcnt[1], c2 = wcnt[2], c3 = wcnt[3];
        const int tot = c0 + c1 + c2 + c3;
        if (nbuf + tot > CAPL) {
            sweep(nbuf);
            nbuf = 0;
        }
        if (keep) {
            const int pos = nbuf + (w > 0 ? c0 : 0) + (w > 1 ? c1 : 0) +
                            (w > 2 ? c2 : 0) + __popcll(m & lt_mask);
            const T fx = (x - rx) + T(sx), fy = (y - ry) + T(sy),
                    fz = (z - rz) + T(sz);
            P::store_j(&sj[pos * P::NJ], f, pa, tv, js + lane, fx, fy, fz);
            sjid[pos] = js + lane;
        }
        nbuf += tot;
        __syncthreads();  // wcnt is rewritten by the next round
    }
    sweep(nbuf);
    acc.quad_reduce();
    if (sweeper && act && q == 0 && slot_active(tv, i)) P::finish(acc, is, pa, tv, i);
}

template <typename T, typename P>
__global__ __launch_bounds__(256) void pair_kernel_leaf(const TreeView<T> tv,
                                                       const typename P::Args pa) {
    constexpr int CAPL = leaf_cap<P>();
    __shared__ __attribute__((aligned(16))) T sj[CAPL * P::NJ];
    __shared__ int sjid[CAPL];
    __shared__ unsigned short slist[4][CAPL];
    __shared__ int wcnt[4];
    const int n_items = *tv.n_items;
    if ((int)blockIdx.x >= n_items) return;
    const int bi = tv.xcd_remap ? xcd_block(blockIdx.x, n_items) : (int)blockIdx.x;
    process_leaf4<T, P>(tv, pa, item_leaf(tv, bi), sj, sjid, slist, wcnt);
}

// Persistent leaf form: each four-wavefront workgroup pops leaves in
// decreasing cost from an atomic counter until the queue is exhausted.
template <typename T, typename P>
__global__ __launch_bounds__(256) void pair_kernel_leaf_queue(
    const TreeView<T> tv, const typename P::Args pa,
    const int32_t *__restrict__ order, int *__restrict__ head) {
    constexpr int CAPL = leaf_cap<P>();
    __shared__ __attribute__((aligned(16))) T sj[CAPL * P::NJ];
    __shared__ int sjid[CAPL];
    __shared__ unsigned short slist[4][CAPL];
    __shared__ int wcnt[4];
    __shared__ int slot;
    const int n_items = *tv.n_items;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) slot = atomicAdd(head, 1);
        __syncthreads();
        const int q = slot;
        if (q >= n_items) break;
        process_leaf4<T, P>(tv, pa, order[q], sj, sjid, slist, wcnt);
    }
}

// Persistent grid: each workgroup pops queue slots from an atomic counter
// (reset to 0 before the launch) until the queue is exhausted; the queue
// lists the leaves by decreasing cost, so the longest items start first.
// Every workgroup leaves the loop once the counter passes the item count.
template <typename T, typename P, int BLOCK>
__global__ __launch_bounds__(BLOCK) void pair_kernel_queue(
    const TreeView<T> tv, const typename P::Args pa,
    const int32_t *__restrict__ order, int *__restrict__ head) {
    __shared__ __attribute__((aligned(16))) T sj[P::CAPF * BLOCK * P::NJ];
    __shared__ int sjid[P::CAPF * BLOCK];
    __shared__ int wcnt[BLOCK / 64];
    __shared__ uint32_t smask[1];
    __shared__ short glist[1];
    __shared__ int slot;
    const int n_items = *tv.n_items;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) slot = atomicAdd(head, 1);
        __syncthreads();
        const int q = slot;
        if (q >= n_items) break;
        process_leaf<T, P, BLOCK, SWEEP_BROADCAST>(tv, pa, order[q], sj, sjid,
                                                   wcnt, smask, glist);
    }
}

// widened pair ranges (relative 1e-5 above the exact test, so that every
// pair a float32 test accepts survives the culling)
template <typename T> __device__ inline T widen(double r) {
    return (T)(r * (1.0 + 1e-5));
}

// --------------------------------------------------------------------------
// density / volume:  V_i = 1 / sum_j W_ij,  rho~_i = sum_j m_j W_ij
// --------------------------------------------------------------------------

template <typename T> struct DensityPass {
    struct Args {
        const T *m;       // tree order
        T *V, *rho_t;     // caller order
    };
    static constexpr int NJ = 4;  // fx, fy, fz, m
    static constexpr int CAPF = 4;  // candidate buffer = CAPF * BLOCK
    static constexpr int ID = 0;    // bit in the walk mask
    // split sweep: one phase (the pair body is about as cheap as its test)
    static constexpr bool MASKED = false;
    // float: eight waves per SIMD (64 VGPRs, one spilled) against seven:
    // 20.16 -> 19.87 ms on the 180 M-particle box
    static constexpr int MINW = std::is_same<T, float>::value ? 8 : 1;
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = false;
    __device__ static T range(const Args &, const TreeView<T> &, int, T hI, T) {
        return widen<T>(2.0 * (double)hI);
    }
    __device__ static T sub_range(const Args &, const TreeView<T> &, int, T hg,
                                  const T *) {
        return widen<T>(2.0 * (double)hg);
    }
    struct I {
        T ex, ey, ez, ih2, h;
    };
    struct Tile {
        T s[2];
        __device__ void zero() { s[0] = s[1] = T(0); }
    };
    struct Acc {
        CompArr<T, 2> a;
        __device__ void zero() { a.zero(); }
        __device__ void fold(Tile &t) { a.fold(t.s); }
        __device__ void quad_reduce() { a.quad_reduce(); }
    };
    __device__ static void load_i(I &is, const Args &, const TreeView<T> &tv,
                                  int i, T ex, T ey, T ez, int) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        is.h = tv.h[i];
        is.ih2 = T(1) / (is.h * is.h);
    }
    static constexpr int NP = 1;  // prefetched with the position: m
    __device__ static void fetch_j(T *f, const Args &a, const TreeView<T> &,
                                   int j) {
        f[0] = a.m[j];
    }
    __device__ static void store_j(T *d, const T *f, const Args &,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = f[0];
    }
    __device__ static bool test(const I &is, const T *jd, bool) {
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        return (dx * dx + dy * dy + dz * dz) * is.ih2 < T(4);
    }
    // branch-free: out-of-range pairs add exact zeros, so the sums are
    // bitwise those of the in-range pairs alone
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool) {
        const T mj = jd[3];
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        const T q2 = (dx * dx + dy * dy + dz * dz) * is.ih2;
        const bool in = q2 < T(4);
        const T rq = rsq(q2);
        const T q = q2 > T(0) ? q2 * rq : T(0);
        const T t = T(2) - q;
        const T w = q < T(1) ? fma(q * q, fma(T(0.75), q, T(-1.5)), T(1))
                             : T(0.25) * t * t * t;
        const T wv = in ? w : T(0);
        tl.s[0] += wv;
        tl.s[1] = fma(mj, wv, tl.s[1]);
    }
    __device__ static void finish(const Acc &ac, const I &is, const Args &a,
                                  const TreeView<T> &tv, int i) {
        const double h = (double)is.h;
        const double ph3 = PI_D * h * h * h;
        const int c = tv.perm[i];
        a.V[c] = (T)(ph3 / ac.a.c[0].value());
        a.rho_t[c] = (T)(ac.a.c[1].value() / ph3);
    }
};

// --------------------------------------------------------------------------
// correction coefficients
// --------------------------------------------------------------------------
// Sums, in units u = x_ij / h_i (a = V_j w, b = V_j wq, mw = m_j w):
//   0      m0            sum a
//   1..3   m1            sum a u_a
//   4..9   m2 (ab)       sum a u_a u_b          (00 01 02 11 12 22)
//   10..12 dm0           sum b u_g
//   13..18 sxdw (ga)     sum b u_g u_a          (00 01 02 11 12 22)
//   19..28 sxxdw (gab)   sum b u_g u_a u_b      (000 001 002 011 012 022
//                                                111 112 122 222)
//   29..31 M1            sum mw u_a
//   32     rho~          sum mw
template <typename T> struct CoeffPass {
    struct Args {
        const T *m, *V, *u;  // tree order
        T *A, *B, *gA, *gB, *rho, *P, *cs;  // caller order (planes of n_gas)
        int64_t n_gas;
        double gamma;
    };
    static constexpr int NJ = 8;  // fx fy fz V m + pad
    static constexpr int CAPF = 4;
    static constexpr int ID = 1;
    static constexpr bool MASKED = true;  // split sweep: test, then pairs
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = false;
    static constexpr int NS = 33;
    __device__ static T range(const Args &, const TreeView<T> &, int, T hI, T) {
        return widen<T>(2.0 * (double)hI);
    }
    __device__ static T sub_range(const Args &, const TreeView<T> &, int, T hg,
                                  const T *) {
        return widen<T>(2.0 * (double)hg);
    }
    struct I {
        T ex, ey, ez, ih;
        T h;
    };
    struct Tile {
        T s[NS];
        __device__ void zero() {
#pragma unroll
            for (int k = 0; k < NS; ++k) s[k] = T(0);
        }
    };
    struct Acc {
        CompArr<T, NS> a;
        __device__ void zero() { a.zero(); }
        __device__ void fold(Tile &t) { a.fold(t.s); }
        __device__ void quad_reduce() { a.quad_reduce(); }
    };
    __device__ static void load_i(I &is, const Args &, const TreeView<T> &tv,
                                  int i, T ex, T ey, T ez, int) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        is.h = tv.h[i];
        is.ih = T(1) / is.h;
    }
    static constexpr int NP = 2;  // prefetched with the position: V, m
    __device__ static void fetch_j(T *f, const Args &a, const TreeView<T> &,
                                   int j) {
        f[0] = a.V[j];
        f[1] = a.m[j];
    }
    __device__ static void store_j(T *d, const T *f, const Args &,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = f[0];
        d[4] = f[1];
        d[5] = T(0);
        d[6] = T(0);
        d[7] = T(0);
    }
    __device__ static bool test(const I &is, const T *jd, bool) {
        const T u0 = (is.ex - jd[0]) * is.ih;
        const T u1 = (is.ey - jd[1]) * is.ih;
        const T u2 = (is.ez - jd[2]) * is.ih;
        return u0 * u0 + u1 * u1 + u2 * u2 < T(4);
    }
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool) {
        const T u0 = (is.ex - jd[0]) * is.ih;
        const T u1 = (is.ey - jd[1]) * is.ih;
        const T u2 = (is.ez - jd[2]) * is.ih;
        const T q2 = u0 * u0 + u1 * u1 + u2 * u2;
        if (q2 < T(4)) {
            const T rq = rsq(q2);
            const T q = q2 > T(0) ? q2 * rq : T(0);
            T w, wq;
            spline(q, rq, w, wq);
            T *s = tl.s;
            const T a = jd[3] * w;
            const T b = jd[3] * wq;
            const T mw = jd[4] * w;
            const T au0 = a * u0, au1 = a * u1, au2 = a * u2;
            s[0] += a;
            s[1] += au0;
            s[2] += au1;
            s[3] += au2;
            s[4] = fma(au0, u0, s[4]);
            s[5] = fma(au0, u1, s[5]);
            s[6] = fma(au0, u2, s[6]);
            s[7] = fma(au1, u1, s[7]);
            s[8] = fma(au1, u2, s[8]);
            s[9] = fma(au2, u2, s[9]);
            const T bu0 = b * u0, bu1 = b * u1, bu2 = b * u2;
            s[10] += bu0;
            s[11] += bu1;
            s[12] += bu2;
            const T p00 = bu0 * u0, p01 = bu0 * u1, p02 = bu0 * u2;
            const T p11 = bu1 * u1, p12 = bu1 * u2, p22 = bu2 * u2;
            s[13] += p00;
            s[14] += p01;
            s[15] += p02;
            s[16] += p11;
            s[17] += p12;
            s[18] += p22;
            s[19] = fma(p00, u0, s[19]);
            s[20] = fma(p00, u1, s[20]);
            s[21] = fma(p00, u2, s[21]);
            s[22] = fma(p01, u1, s[22]);
            s[23] = fma(p01, u2, s[23]);
            s[24] = fma(p02, u2, s[24]);
            s[25] = fma(p11, u1, s[25]);
            s[26] = fma(p11, u2, s[26]);
            s[27] = fma(p12, u2, s[27]);
            s[28] = fma(p22, u2, s[28]);
            s[29] = fma(mw, u0, s[29]);
            s[30] = fma(mw, u1, s[30]);
            s[31] = fma(mw, u2, s[31]);
            s[32] += mw;
        }
    }
    __device__ static void finish(const Acc &ac, const I &is, const Args &a,
                                  const TreeView<T> &tv, int i) {
        double S[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) S[k] = ac.a.c[k].value();
        const double h = (double)is.h;
        const double N = 1.0 / (PI_D * h * h * h);
        // symmetric index maps
        const int i2[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
        const int i3[3][3][3] = {{{0, 1, 2}, {1, 3, 4}, {2, 4, 5}},
                                 {{1, 3, 4}, {3, 6, 7}, {4, 7, 8}},
                                 {{2, 4, 5}, {4, 7, 8}, {5, 8, 9}}};
        double m0 = N * S[0];
        double m1[3], m2[3][3], dm0[3], dm1[3][3], dm2[3][3][3], M1[3];
        for (int x = 0; x < 3; ++x) {
            m1[x] = N * h * S[1 + x];
            dm0[x] = N / h * S[10 + x];
            M1[x] = N * h * S[29 + x];
        }
        for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y) m2[x][y] = N * h * h * S[4 + i2[x][y]];
        for (int g = 0; g < 3; ++g)
            for (int x = 0; x < 3; ++x) {
                dm1[g][x] = (x == g ? m0 : 0.0) + N * S[13 + i2[g][x]];
                for (int y = 0; y < 3; ++y)
                    dm2[g][x][y] = (x == g ? m1[y] : 0.0) + (y == g ? m1[x] : 0.0) +
                                   N * h * S[19 + i3[g][x][y]];
            }
        const double rt = N * S[32];
        // solve (double): B = -m2^-1 m1, A = 1/(m0 + B.m1), gradients
        double c00 = m2[1][1] * m2[2][2] - m2[1][2] * m2[2][1];
        double c01 = m2[1][2] * m2[2][0] - m2[1][0] * m2[2][2];
        double c02 = m2[1][0] * m2[2][1] - m2[1][1] * m2[2][0];
        double det = m2[0][0] * c00 + m2[0][1] * c01 + m2[0][2] * c02;
        double tr = m2[0][0] + m2[1][1] + m2[2][2];
        double A, B[3], dA[3], dB[3][3];
        // singular when det <= 1e-5 (tr/3)^3.  The bound sits far above the
        // float32 noise of the moment sums (about 1e-7 relative), so the two
        // precisions take the same branch except for neighbourhoods whose
        // det / (tr/3)^3 lies within a few 1e-7 of the bound, a narrow band
        // where either branch may be taken
        if (!(fabs(det) > 1e-5 * tr * tr * tr / 27.0) || !(tr > 0.0)) {
            A = 1.0 / m0;
            for (int g = 0; g < 3; ++g) {
                B[g] = 0.0;
                dA[g] = -dm0[g] / (m0 * m0);
                for (int x = 0; x < 3; ++x) dB[g][x] = 0.0;
            }
        } else {
            double inv[3][3];
            const double id = 1.0 / det;
            inv[0][0] = c00 * id;
            inv[0][1] = (m2[0][2] * m2[2][1] - m2[0][1] * m2[2][2]) * id;
            inv[0][2] = (m2[0][1] * m2[1][2] - m2[0][2] * m2[1][1]) * id;
            inv[1][0] = c01 * id;
            inv[1][1] = (m2[0][0] * m2[2][2] - m2[0][2] * m2[2][0]) * id;
            inv[1][2] = (m2[0][2] * m2[1][0] - m2[0][0] * m2[1][2]) * id;
            inv[2][0] = c02 * id;
            inv[2][1] = (m2[0][1] * m2[2][0] - m2[0][0] * m2[2][1]) * id;
            inv[2][2] = (m2[0][0] * m2[1][1] - m2[0][1] * m2[1][0]) * id;
            for (int x = 0; x < 3; ++x) {
                B[x] = 0.0;
                for (int y = 0; y < 3; ++y) B[x] -= inv[x][y] * m1[y];
            }
            A = 1.0 / (m0 + B[0] * m1[0] + B[1] * m1[1] + B[2] * m1[2]);
            for (int g = 0; g < 3; ++g) {
                double rhs[3];
                for (int x = 0; x < 3; ++x) {
                    rhs[x] = dm1[g][x];
                    for (int y = 0; y < 3; ++y) rhs[x] += dm2[g][x][y] * B[y];
                }
                for (int x = 0; x < 3; ++x) {
                    dB[g][x] = 0.0;
                    for (int y = 0; y < 3; ++y) dB[g][x] -= inv[x][y] * rhs[y];
                }
                double sg = dm0[g];
                for (int x = 0; x < 3; ++x) sg += dB[g][x] * m1[x] + B[x] * dm1[g][x];
                dA[g] = -A * A * sg;
            }
        }
        const int c = tv.perm[i];
        const int64_t n = a.n_gas;
        a.A[c] = (T)A;
        for (int g = 0; g < 3; ++g) {
            a.B[g * n + c] = (T)B[g];
            a.gA[g * n + c] = (T)dA[g];
            for (int x = 0; x < 3; ++x) a.gB[(3 * g + x) * n + c] = (T)dB[g][x];
        }
        const double rho = A * (rt + B[0] * M1[0] + B[1] * M1[1] + B[2] * M1[2]);
        const double uu = (double)a.u[i];
        a.rho[c] = (T)rho;
        a.P[c] = (T)((a.gamma - 1.0) * rho * uu);
        a.cs[c] = (T)sqrt(a.gamma * (a.gamma - 1.0) * uu);
    }
};

// --------------------------------------------------------------------------
// hydro forces
// --------------------------------------------------------------------------
// Per-particle fields, precomputed by hydro_gather_kernel (tree order), one
// contiguous record of hydro_stride(w) floats per particle (w fields, the
// stride a multiple of four so that records load as 16-byte units):
//   0 vx 1 vy 2 vz 3 ih2=1/h^2 4 a=A N 5..7 da=dA N 8..10 B
//   11..13 ab=A N B  14..22 adb=A N dB [g][x]  23 h  24 V  25 P  26 rho
//   27 cs   (N = 1/(pi h^3))
//   with the reconstruction: 28..33 the symmetric part of the velocity
//   gradient as the quadratic form x.dv x needs it: dv00 dv11 dv22
//   dv01+dv10 dv02+dv20 dv12+dv21
//   for the compatible energy update, after those: the velocities after the
//   kick, v1 = v + dt (a_grav + a_hydro) (3 planes)
// The corrected-kernel gradient of particle k at separation y:
//   g_k(y)_g = (1 + B.y)(da_g w + a wq ih2 y_g) + w (sum_x adb[g][x] y_x + ab_g)
constexpr int HF = 28;
constexpr int HF_RECON = HF + 6;
constexpr int HF_MAX = HF_RECON + 3;
__host__ __device__ constexpr int hydro_stride(int w) { return (w + 3) / 4 * 4; }

// n fields (n % 4 == 0 for the vector form) of a record into dst
template <typename T, int N>
__device__ __forceinline__ void copy_fields(T *dst, const T *src) {
    if constexpr (std::is_same<T, float>::value && N % 4 == 0) {
        const float4 *s4 = reinterpret_cast<const float4 *>(src);
        float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
        for (int k = 0; k < N / 4; ++k) d4[k] = s4[k];
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) dst[k] = src[k];
    }
}

// optional inputs of the hydro field gather
template <typename T> struct GatherExtra {
    const T *dv = nullptr;           // velocity gradient, 9 caller planes
    const T *ag[3] = {nullptr, nullptr, nullptr};  // kick accelerations
    const T *ah[3] = {nullptr, nullptr, nullptr};
    double dt = 0.0;
    // block kicks: with bins (caller order), the kick width of each
    // particle follows its bin and the substep (kick_width); dt otherwise
    const int32_t *bins = nullptr;
    int L = 0;
    int64_t substep = -1;
};

// Width of the kick at the boundary after substep s of a cycle of 2^L
// substeps for a particle of bin b (tau_b = dt / 2^b): s < 0, the opening
// half-kick of the interval, tau_b / 2; a particle ending a step after s,
// tau_b (its closing half-kick and the opening half-kick of its next step,
// one kick with the same forces), or tau_b / 2 after the last substep; any
// other particle 0.
__device__ inline double kick_width(double dt, int L, int64_t s, int b) {
    b = b < 0 ? 0 : (b > L ? L : b);
    const double tau = ldexp(dt, -b);
    if (s < 0) return 0.5 * tau;
    if ((s + 1) % ((int64_t)1 << (L - b)) != 0) return 0.0;
    return (s + 1 == ((int64_t)1 << L)) ? 0.5 * tau : tau;
}

// RECON: the viscosity acts on both velocities extrapolated linearly to the
// pair midpoint, v~_ij = v_ij - phi/2 (dv_i + dv_j) x_ij, with the limiter
// phi = 4 s_i s_j / (s_i + s_j)^2 (0 unless s_i s_j > 0), s_k = x.dv_k x,
// damped by exp(-((eta - eta_c) / eta_f)^2) for eta = r / max(h) < eta_c.
// WORK: the same pair forces, but only du/dt, with the pair work taken at
// the time-centred velocities (v + v1)/2 of the kick v1 (the compatible
// energy update)
template <typename T, bool RECON = false, bool WORK = false> struct HydroPass {
    struct Args {
        const T *f;       // records of RS floats (HFN fields), tree order
        int64_t n_gas;
        T *ax, *ay, *az, *dudt;  // caller order
        const T *m;       // tree order
        T Cl, Cq, epsQ;
        T eta_c, ieta_f;  // close-pair scale and 1 / its width (RECON)
    };
    static constexpr int W0 = RECON ? HF_RECON : HF;  // v1 planes (WORK)
    static constexpr int HFN = W0 + (WORK ? 3 : 0);
    // candidate record: fx fy fz, one pad, the HFN fields from float FO on
    // (16-byte aligned, so they load as 128-bit LDS reads), padded to an odd
    // number of 16-byte units (36 or 44 floats): records read by different
    // lanes at once then start in different 16-byte bank groups
    static constexpr int FO = 4;
    static constexpr int NJ = (((FO + HFN + 3) / 4) | 1) * 4;
    static_assert(NJ == (RECON ? 44 : 36), "hydro record layout");
    static constexpr int RS = hydro_stride(HFN);  // record stride in memory
    static constexpr int CAPF = 1;
    static constexpr int ID = 2;
    // split sweep: one phase.  The in-range candidates of one buffer are
    // clustered in space, so the per-lane counts of a two-phase sweep are
    // uneven and its longest lane costs more than the plain sweep.
    static constexpr bool MASKED = false;
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = true;  // 2 max(h_i, h_j)
    __device__ static T range(const Args &, const TreeView<T> &, int, T hI, T hJ) {
        return widen<T>(2.0 * (double)(hI > hJ ? hI : hJ));
    }
    __device__ static T sub_range(const Args &, const TreeView<T> &, int, T hg,
                                  const T *jd) {
        const T hj = jd[FO + 23];
        return widen<T>(2.0 * (double)(hg > hj ? hg : hj));
    }
    struct I {
        T ex, ey, ez;
        T Cl, Cq, epsQ, eta_c, ieta_f;
        T f[HFN];
    };
    struct Tile {
        T s[4];
        __device__ void zero() { s[0] = s[1] = s[2] = s[3] = T(0); }
    };
    struct Acc {
        CompArr<T, 4> a;
        __device__ void zero() { a.zero(); }
        __device__ void fold(Tile &t) { a.fold(t.s); }
        __device__ void quad_reduce() { a.quad_reduce(); }
    };
    __device__ static void load_i(I &is, const Args &a, const TreeView<T> &,
                                  int i, T ex, T ey, T ez, int) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        is.Cl = a.Cl;
        is.Cq = a.Cq;
        is.epsQ = a.epsQ;
        is.eta_c = a.eta_c;
        is.ieta_f = a.ieta_f;
        copy_fields<T, HFN>(is.f, a.f + (int64_t)i * RS);
    }
    // the fields are many: loaded for the culling survivors only
    static constexpr int NP = 1;
    __device__ static void fetch_j(T *, const Args &, const TreeView<T> &,
                                   int) {}
    __device__ static void store_j(T *d, const T *, const Args &a,
                                   const TreeView<T> &, int j, T fx, T fy,
                                   T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = T(0);
        // whole 16-byte units of the record (its padding included)
        copy_fields<T, RS>(d + FO, a.f + (int64_t)j * RS);
#pragma unroll
        for (int k = FO + RS; k < NJ; ++k) d[k] = T(0);
    }
    // gradient of the corrected kernel of particle with fields f at y (and
    // q = r / h of that particle)
    __device__ static void grad_rk(const T *f, T y0, T y1, T y2, T r2, T out[3],
                                   bool &on, T &qo) {
        const T q2 = r2 * f[3];
        on = q2 < T(4);
        const T rq = rsq(q2);
        const T q = q2 > T(0) ? q2 * rq : T(0);
        qo = q;
        T w, wq;
        spline(q, rq, w, wq);
        const T by1 = T(1) + f[8] * y0 + f[9] * y1 + f[10] * y2;
        const T c1 = f[4] * wq * f[3];
        const T y[3] = {y0, y1, y2};
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const T dby = f[14 + 3 * g] * y0 + f[15 + 3 * g] * y1 + f[16 + 3 * g] * y2;
            out[g] = by1 * fma(f[5 + g], w, c1 * y[g]) + w * (dby + f[11 + g]);
        }
    }
    __device__ static bool test(const I &is, const T *jd, bool self) {
        const T x0 = is.ex - jd[0], x1 = is.ey - jd[1], x2 = is.ez - jd[2];
        const T r2 = x0 * x0 + x1 * x1 + x2 * x2;
        return !self & ((r2 * is.f[3] < T(4)) | (r2 * jd[FO + 3] < T(4)));
    }
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool self) {
        const T x0 = is.ex - jd[0], x1 = is.ey - jd[1], x2 = is.ez - jd[2];
        const T r2 = x0 * x0 + x1 * x1 + x2 * x2;
        const T *fj = jd + FO;
        const T *fi = is.f;
        // both range tests evaluated (no short circuit: no branch around the
        // LDS read of the j-side 1/h^2)
        const bool near = (r2 * fi[3] < T(4)) | (r2 * fj[3] < T(4));
        if (near & !self) {
            T gi[3], gj[3], qi, qj;
            bool oi, oj;
            grad_rk(fi, x0, x1, x2, r2, gi, oi, qi);
            grad_rk(fj, -x0, -x1, -x2, r2, gj, oj, qj);
            const T v0 = fi[0] - fj[0], v1 = fi[1] - fj[1], v2 = fi[2] - fj[2];
            T vdx = v0 * x0 + v1 * x1 + v2 * x2;
            const T hi_ = fi[23], hj_ = fj[23];
            if constexpr (RECON) {
                // x.v~ = x.v_ij - phi/2 (s_i + s_j): only the projections
                // of the two extrapolations on the pair axis enter mu
                const T *Di = fi + HF, *Dj = fj + HF;
                const T q00 = x0 * x0, q11 = x1 * x1, q22 = x2 * x2;
                const T q01 = x0 * x1, q02 = x0 * x2, q12 = x1 * x2;
                const T si = fma(Di[0], q00, fma(Di[1], q11, fma(Di[2], q22,
                             fma(Di[3], q01, fma(Di[4], q02, Di[5] * q12)))));
                const T sj = fma(Dj[0], q00, fma(Dj[1], q11, fma(Dj[2], q22,
                             fma(Dj[3], q01, fma(Dj[4], q02, Dj[5] * q12)))));
                const T sp = si + sj;
                T phi = si * sj > T(0) ? T(4) * si * sj * rcp(sp * sp) : T(0);
                // eta = r / max(h_i, h_j) = min(q_i, q_j)
                const T eta = qi < qj ? qi : qj;
                const T te = (eta - is.eta_c) * is.ieta_f;
                phi = eta < is.eta_c ? phi * fexp(-te * te) : phi;
                vdx = fma(T(-0.5) * phi, sp, vdx);
            }
            T mui = hi_ * vdx * rcp(fma(is.epsQ * hi_, hi_, r2));
            T muj = hj_ * vdx * rcp(fma(is.epsQ * hj_, hj_, r2));
            mui = mui < T(0) ? mui : T(0);
            muj = muj < T(0) ? muj : T(0);
            const T Qi = fi[26] * mui * fma(is.Cq, mui, -is.Cl * fi[27]);
            const T Qj = fj[26] * muj * fma(is.Cq, muj, -is.Cl * fj[27]);
            const T pp = fi[25] + fj[25];
            const T ci = pp + Qi, cj = pp + Qj;
            const T k = T(-0.5) * fi[24] * fj[24];
            const T F0 = k * (ci * gi[0] - cj * gj[0]);
            const T F1 = k * (ci * gi[1] - cj * gj[1]);
            const T F2 = k * (ci * gi[2] - cj * gj[2]);
            if constexpr (WORK) {
                const T *wi = fi + W0, *wj = fj + W0;
                const T c0 = T(0.5) * (v0 + (wi[0] - wj[0]));
                const T c1 = T(0.5) * (v1 + (wi[1] - wj[1]));
                const T c2 = T(0.5) * (v2 + (wi[2] - wj[2]));
                tl.s[3] = fma(c0, F0, fma(c1, F1, fma(c2, F2, tl.s[3])));
            } else {
                tl.s[0] += F0;
                tl.s[1] += F1;
                tl.s[2] += F2;
                tl.s[3] = fma(v0, F0, fma(v1, F1, fma(v2, F2, tl.s[3])));
            }
        }
    }
    __device__ static void finish(const Acc &ac, const I &, const Args &a,
                                  const TreeView<T> &tv, int i) {
        const int c = tv.perm[i];
        const double im = 1.0 / (double)a.m[i];
        if constexpr (!WORK) {
            a.ax[c] = (T)(ac.a.c[0].value() * im);
            a.ay[c] = (T)(ac.a.c[1].value() * im);
            a.az[c] = (T)(ac.a.c[2].value() * im);
        }
        a.dudt[c] = (T)(-0.5 * ac.a.c[3].value() * im);
    }
};

// --------------------------------------------------------------------------
// velocity gradient
// --------------------------------------------------------------------------
// dv[a][b]_i = sum_j V_j (v_j^a - v_i^a) g_i(x_ij)_b over gas j with
// r_ij < 2 h_i, with the corrected-kernel gradient g_i of the hydro fields
// (planes 0..22 and 24 of the hydro gather); j = i adds zero.
template <typename T> struct VGradPass {
    struct Args {
        const T *f;   // hydro field records (stride hydro_stride(HF)), tree order
        int64_t n_gas;
        T *dv;        // 9 planes [a][b] of n_gas, caller order
    };
    static constexpr int RS = hydro_stride(HF);
    static constexpr int NJ = 8;  // fx fy fz V vx vy vz pad
    static constexpr int CAPF = 4;
    static constexpr int ID = 6;
    static constexpr bool MASKED = false;
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = false;
    static constexpr int NI = 23;  // i fields: v, 1/h^2, coefficients
    __device__ static T range(const Args &, const TreeView<T> &, int, T hI, T) {
        return widen<T>(2.0 * (double)hI);
    }
    __device__ static T sub_range(const Args &, const TreeView<T> &, int, T hg,
                                  const T *) {
        return widen<T>(2.0 * (double)hg);
    }
    struct I {
        T ex, ey, ez;
        T f[24];  // NI used
    };
    struct Tile {
        T s[9];
        __device__ void zero() {
#pragma unroll
            for (int k = 0; k < 9; ++k) s[k] = T(0);
        }
    };
    struct Acc {
        CompArr<T, 9> a;
        __device__ void zero() { a.zero(); }
        __device__ void fold(Tile &t) { a.fold(t.s); }
        __device__ void quad_reduce() { a.quad_reduce(); }
    };
    __device__ static void load_i(I &is, const Args &a, const TreeView<T> &,
                                  int i, T ex, T ey, T ez, int) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        copy_fields<T, 24>(is.f, a.f + (int64_t)i * RS);  // (the first NI used)
    }
    static constexpr int NP = 4;  // prefetched with the position: V, v
    __device__ static void fetch_j(T *f, const Args &a, const TreeView<T> &,
                                   int j) {
        const T *r = a.f + (int64_t)j * RS;
        f[0] = r[24];
        f[1] = r[0];
        f[2] = r[1];
        f[3] = r[2];
    }
    __device__ static void store_j(T *d, const T *f, const Args &,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = f[0];
        d[4] = f[1];
        d[5] = f[2];
        d[6] = f[3];
        d[7] = T(0);
    }
    __device__ static bool test(const I &is, const T *jd, bool) {
        const T x0 = is.ex - jd[0], x1 = is.ey - jd[1], x2 = is.ez - jd[2];
        return (x0 * x0 + x1 * x1 + x2 * x2) * is.f[3] < T(4);
    }
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool) {
        const T x0 = is.ex - jd[0], x1 = is.ey - jd[1], x2 = is.ez - jd[2];
        const T r2 = x0 * x0 + x1 * x1 + x2 * x2;
        T g[3], q;
        bool on;
        HydroPass<T>::grad_rk(is.f, x0, x1, x2, r2, g, on, q);
        if (on) {
            const T d0 = jd[3] * (jd[4] - is.f[0]);
            const T d1 = jd[3] * (jd[5] - is.f[1]);
            const T d2 = jd[3] * (jd[6] - is.f[2]);
            T *s = tl.s;
            s[0] = fma(d0, g[0], s[0]);
            s[1] = fma(d0, g[1], s[1]);
            s[2] = fma(d0, g[2], s[2]);
            s[3] = fma(d1, g[0], s[3]);
            s[4] = fma(d1, g[1], s[4]);
            s[5] = fma(d1, g[2], s[5]);
            s[6] = fma(d2, g[0], s[6]);
            s[7] = fma(d2, g[1], s[7]);
            s[8] = fma(d2, g[2], s[8]);
        }
    }
    __device__ static void finish(const Acc &ac, const I &, const Args &a,
                                  const TreeView<T> &tv, int i) {
        const int c = tv.perm[i];
#pragma unroll
        for (int k = 0; k < 9; ++k) a.dv[k * a.n_gas + c] = (T)ac.a.c[k].value();
    }
};

// --------------------------------------------------------------------------
// short-range gravity
// --------------------------------------------------------------------------
// a_i = -G sum_j m_j g(r)/r x_ij with, for xi = 2r/r_c,
//   g/r = (r^2+eps^2)^(-3/2) - (2/(35 r_c^3)) (224 - 224 xi^2 + 70 xi^3
//         + 48 xi^4 - 21 xi^5)                                  xi < 1
//   g/r = (r^2+eps^2)^(-3/2) + r^-3 ((2-xi)^5 (7 xi^3 + 22 xi^2 + 10 xi
//         + 4) / 140 - 1)                                        1 <= xi < 2
template <typename T> struct GravityPass {
    struct Args {
        const T *m;  // tree order, times G
        T *ax_g, *ay_g, *az_g, *ax_d, *ay_d, *az_d;  // caller order
        int64_t n_gas;
        const float4 *pk;  // float: (x, y, z, G m) per slot, tree order
    };
    static constexpr int NJ = 4;  // fx fy fz Gm
    static constexpr int CAPF = 4;
    static constexpr int ID = 3;
    static constexpr bool MASKED = false;  // (as for the hydro forces)
    // float: the split sweep stages candidates that are at least far_range
    // from the sub-leaf box apart and sweeps them with pair_far
    static constexpr bool FARNEAR = std::is_same<T, float>::value;
    // float: eight waves per SIMD (64 VGPRs, no spills) against seven
    // left to the compiler: 124.5 -> 122.0 ms on the 180 M-particle box
    static constexpr int MINW = std::is_same<T, float>::value ? 8 : 1;
    // float: position and G m of every slot packed in one 16-byte record
    static constexpr bool PK = std::is_same<T, float>::value;
    static constexpr bool RANGE_HJ = false;
    __device__ static const float4 *packed(const Args &a) { return a.pk; }
    __device__ static T range(const Args &, const TreeView<T> &tv, int box, T, T) {
        return widen<T>(tv.rc[box]);
    }
    __device__ static T sub_range(const Args &, const TreeView<T> &tv, int box, T,
                                  const T *) {
        return widen<T>(tv.rc[box]);
    }
    struct I {
        T ex, ey, ez;
        T rc2, eps2, two_rc, cin;
    };
    struct Tile {
        T s[3];
        __device__ void zero() { s[0] = s[1] = s[2] = T(0); }
    };
    struct Acc {
        CompArr<T, 3> a;
        __device__ void zero() { a.zero(); }
        __device__ void fold(Tile &t) { a.fold(t.s); }
        __device__ void quad_reduce() { a.quad_reduce(); }
    };
    __device__ static void load_i(I &is, const Args &, const TreeView<T> &tv,
                                  int, T ex, T ey, T ez, int box) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        const double rc = tv.rc[box], eps = tv.eps[box];
        is.rc2 = (T)(rc * rc);
        is.eps2 = (T)(eps * eps);
        is.two_rc = (T)(2.0 / rc);
        is.cin = (T)(2.0 / (35.0 * rc * rc * rc));
    }
    static constexpr int NP = 1;  // prefetched with the position: G m
    __device__ static void fetch_j(T *f, const Args &a, const TreeView<T> &,
                                   int j) {
        f[0] = a.m[j];
    }
    __device__ static void store_j(T *d, const T *f, const Args &,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = f[0];
    }
    __device__ static bool test(const I &is, const T *jd, bool) {
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        const T r2 = dx * dx + dy * dy + dz * dz;
        return (r2 > T(0)) && (r2 < is.rc2);
    }
    // out-of-range pairs leave before the arithmetic: the wave skips it when
    // no lane is in range (frequent here: the candidates fill the leaf box
    // widened by r_c), and in-range lanes accumulate under the mask with no
    // zero weight kept for the others
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool) {
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (!((r2 > T(0)) && (r2 < is.rc2))) return;
        const T rs = rsq(r2);
        const T r = r2 * rs;
        const T xi = r * is.two_rc;
        const T ps = rsq(r2 + is.eps2);
        const T plum = ps * ps * ps;
        const T x2 = xi * xi;
        T pin = fma(T(-21), xi, T(48));
        pin = fma(pin, xi, T(70));
        pin = fma(pin, xi, T(-224));
        pin = fma(pin, x2, T(224));
        const T gin = fma(-is.cin, pin, plum);
        const T u = T(2) - xi;
        const T u2 = u * u;
        const T u5 = u2 * u2 * u;
        // (7 xi^3 + 22 xi^2 + 10 xi + 4) / 140
        T po = fma(T(7.0 / 140.0), xi, T(22.0 / 140.0));
        po = fma(po, xi, T(10.0 / 140.0));
        po = fma(po, xi, T(4.0 / 140.0));
        const T val = fma(u5, po, T(-1));
        const T rs3 = rs * rs * rs;
        const T gout = fma(rs3, val, plum);
        const T gr = xi < T(1) ? gin : gout;
        const T w = jd[3] * gr;
        tl.s[0] = fma(-w, dx, tl.s[0]);
        tl.s[1] = fma(-w, dy, tl.s[1]);
        tl.s[2] = fma(-w, dz, tl.s[2]);
    }
    // Candidates at least this far from the sub-leaf box are far from every
    // particle of it: r >= r_c / 2 (the outer branch of the S2 split) and
    // r >= 15 eps (so (eps / r)^2 <= 1/225).  Relative margin against the
    // float32 branch decision, absolute margin for the rounding of the
    // shifted box bounds.
    __device__ static T far_range(const TreeView<T> &tv, int box) {
        const double rc = tv.rc[box], eps = tv.eps[box];
        return (T)(fmax(0.5 * rc, 15.0 * eps) * (1.0 + 1e-4) + 2e-6);
    }
    // pair of a far candidate: only the outer S2 branch, and the Plummer
    // factor (r^2 + eps^2)^(-3/2) = r^-3 (1 + e)^(-3/2), e = (eps/r)^2 <=
    // 1/225, from its binomial series to e^2 (the first term left out,
    // 35/16 e^3, is below 2e-7 of r^-3, and below 3e-9 where r_c/2 >= 30
    // eps): one reciprocal square root per pair instead of two
    __device__ static void pair_far(Tile &tl, const I &is, const T *jd) {
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < is.rc2)) return;
        const T rs = rsq(r2);
        const T rs2 = rs * rs;
        const T rs3 = rs2 * rs;
        const T xi = (r2 * rs) * is.two_rc;
        const T u = T(2) - xi;
        const T u2 = u * u;
        const T u5 = u2 * u2 * u;
        T po = fma(T(7.0 / 140.0), xi, T(22.0 / 140.0));
        po = fma(po, xi, T(10.0 / 140.0));
        po = fma(po, xi, T(4.0 / 140.0));
        const T e = is.eps2 * rs2;
        const T q = fma(e, T(15.0 / 8.0), T(-1.5));
        const T t = fma(u5, po, e * q);
        const T w = jd[3] * (rs3 * t);
        tl.s[0] = fma(-w, dx, tl.s[0]);
        tl.s[1] = fma(-w, dy, tl.s[1]);
        tl.s[2] = fma(-w, dz, tl.s[2]);
    }
    __device__ static void finish(const Acc &ac, const I &, const Args &a,
                                  const TreeView<T> &tv, int i) {
        const int c = tv.perm[i];
        const T x = (T)ac.a.c[0].value(), y = (T)ac.a.c[1].value(),
                z = (T)ac.a.c[2].value();
        // pointer selects (an if/else here puts the pointers in scratch)
        const bool gas = c < a.n_gas;
        const int k = gas ? c : c - (int)a.n_gas;
        T *ox = gas ? a.ax_g : a.ax_d;
        T *oy = gas ? a.ay_g : a.ay_d;
        T *oz = gas ? a.az_g : a.az_d;
        ox[k] = x;
        oy[k] = y;
        oz[k] = z;
    }
};

// --------------------------------------------------------------------------
// in-range pair counts (diagnostic; the exact pair conditions of the passes)
// --------------------------------------------------------------------------
// mode 0: gas j with r < 2 h_i, j = i included (density, coefficients)
// mode 1: gas j != i with r < 2 max(h_i, h_j)          (hydro forces)
// mode 2: any j with 0 < r < r_c                      (gravity)
// modes 3, 4, 5: every (i, candidate) pair the sweeps of modes 0, 1, 2
// evaluate after culling (the work the pair kernels actually issue)
template <typename T> struct CountPass {
    struct Args {
        int mode;
        int32_t *counts;  // tree order
    };
    static constexpr int NJ = 4;  // fx fy fz 1/h^2
    static constexpr int CAPF = 4;
    static constexpr int ID = 4;
    static constexpr bool MASKED = false;
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = true;  // 2 max(h_i, h_j)
    __device__ static T range(const Args &a, const TreeView<T> &tv, int box, T hI,
                              T hJ) {
        const int m = a.mode % 3;
        if (m == 2) return widen<T>(tv.rc[box]);
        if (m == 1) return widen<T>(2.0 * (double)(hI > hJ ? hI : hJ));
        return widen<T>(2.0 * (double)hI);
    }
    // the sub-leaf ranges of the pass each mode mirrors
    __device__ static T sub_range(const Args &a, const TreeView<T> &tv, int box,
                                  T hg, const T *jd) {
        const int m = a.mode % 3;
        if (m == 2) return widen<T>(tv.rc[box]);
        if (m == 1) {
            const double hj = 1.0 / sqrt((double)jd[3]);
            return widen<T>(2.0 * fmax((double)hg, hj));
        }
        return widen<T>(2.0 * (double)hg);
    }
    struct I {
        T ex, ey, ez, ih2, rc2;
        int mode;
    };
    struct Tile {
        int c;
        __device__ void zero() { c = 0; }
    };
    struct Acc {
        int c;
        __device__ void zero() { c = 0; }
        __device__ void fold(Tile &t) {
            c += t.c;
            t.c = 0;
        }
        __device__ void quad_reduce() {
            c += __shfl_xor(c, 1);
            c += __shfl_xor(c, 2);
        }
    };
    __device__ static void load_i(I &is, const Args &a, const TreeView<T> &tv,
                                  int i, T ex, T ey, T ez, int box) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        const T h = tv.h[i];
        is.ih2 = a.mode % 3 == 2 ? T(0) : T(1) / (h * h);
        const double rc = tv.rc[box];
        is.rc2 = (T)(rc * rc);
        is.mode = a.mode;
    }
    static constexpr int NP = 1;  // prefetched with the position: h
    __device__ static void fetch_j(T *f, const Args &, const TreeView<T> &tv,
                                   int j) {
        f[0] = tv.h[j];
    }
    __device__ static void store_j(T *d, const T *f, const Args &a,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        const T h = f[0];
        d[3] = a.mode % 3 == 1 ? T(1) / (h * h) : T(0);
    }
    __device__ static bool test(const I &is, const T *jd, bool self) {
        const T dx = is.ex - jd[0], dy = is.ey - jd[1], dz = is.ez - jd[2];
        const T r2 = dx * dx + dy * dy + dz * dz;
        if (is.mode >= 3) return true;  // swept pairs: every candidate
        if (is.mode == 0) return r2 * is.ih2 < T(4);
        if (is.mode == 1) return !self && (r2 * is.ih2 < T(4) || r2 * jd[3] < T(4));
        return r2 > T(0) && r2 < is.rc2;
    }
    __device__ static void pair(Tile &tl, const I &is, const T *jd, bool self) {
        tl.c += test(is, jd, self) ? 1 : 0;
    }
    __device__ static void finish(const Acc &ac, const I &, const Args &a,
                                  const TreeView<T> &, int i) {
        a.counts[i] = ac.c;
    }
};

// --------------------------------------------------------------------------
// friends-of-friends links (the in-situ halo finding of Sec. IV-B.3 as a
// second pair workload): union-find over caller indices
// --------------------------------------------------------------------------
// Roots always hook under smaller roots (compare-and-swap on the parent
// word), so every union loop ends and each group's root is its smallest
// index whatever the order of the links.  Parent words are read with
// device-scope atomic loads (the L1 of another compute unit may hold a
// stale copy).
__device__ inline int fof_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int fof_find(int32_t *parent, int x) {
    int p = fof_load(parent + x);
    while (p != x) {
        x = p;
        p = fof_load(parent + x);
    }
    return x;
}
__device__ inline void fof_unite(int32_t *parent, int a, int b) {
    while (true) {
        a = fof_find(parent, a);
        b = fof_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        // hook root a under the smaller root b
        if (atomicCAS(parent + a, a, b) == a) return;
    }
}

template <typename T> struct FofPass {
    struct Args {
        int32_t *parent;  // caller index space (gas, then dm)
        double b;         // linking length
    };
    static constexpr int NJ = 4;  // fx fy fz, caller index of j
    static constexpr int CAPF = 4;
    static constexpr int ID = 5;
    static constexpr bool MASKED = false;
    static constexpr bool FARNEAR = false;
    static constexpr bool PK = false;
    static constexpr bool RANGE_HJ = false;
    __device__ static T range(const Args &a, const TreeView<T> &, int, T, T) {
        return widen<T>(a.b);
    }
    __device__ static T sub_range(const Args &a, const TreeView<T> &, int, T,
                                  const T *) {
        return widen<T>(a.b);
    }
    struct I {
        T ex, ey, ez;
        int c;
        int32_t *parent;
        double b2;
    };
    struct Tile {
        __device__ void zero() {}
    };
    struct Acc {
        __device__ void zero() {}
        __device__ void fold(Tile &) {}
        __device__ void quad_reduce() {}
    };
    __device__ static void load_i(I &is, const Args &a, const TreeView<T> &tv,
                                  int i, T ex, T ey, T ez, int) {
        is.ex = ex;
        is.ey = ey;
        is.ez = ez;
        is.c = tv.perm[i];
        is.parent = a.parent;
        is.b2 = a.b * a.b;
    }
    // the caller index travels with the position (bit copy for float,
    // exact value for double)
    static constexpr int NP = 1;
    __device__ static void fetch_j(T *f, const Args &, const TreeView<T> &tv,
                                   int j) {
        f[0] = enc(tv.perm[j]);
    }
    __device__ static void store_j(T *d, const T *f, const Args &,
                                   const TreeView<T> &, int, T fx, T fy, T fz) {
        d[0] = fx;
        d[1] = fy;
        d[2] = fz;
        d[3] = f[0];
    }
    __device__ static T enc(int c) {
        if constexpr (sizeof(T) == 4) return __int_as_float(c);
        else return (T)c;
    }
    __device__ static int dec(T v) {
        if constexpr (sizeof(T) == 4) return __float_as_int(v);
        else return (int)v;
    }
    // r^2 in double from the exact float separations, summed in a fixed
    // order (no contraction): the same decision as a double evaluation of
    // the minimum-image separations
    __device__ static double r2_of(const I &is, const T *jd) {
#pragma clang fp contract(off)
        const double dx = (double)(is.ex - jd[0]);
        const double dy = (double)(is.ey - jd[1]);
        const double dz = (double)(is.ez - jd[2]);
        const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        return (xx + yy) + zz;
    }
    __device__ static bool test(const I &is, const T *jd, bool self) {
        return !self && r2_of(is, jd) < is.b2;
    }
    __device__ static void pair(Tile &, const I &is, const T *jd, bool self) {
        if (!self && r2_of(is, jd) < is.b2) fof_unite(is.parent, is.c, dec(jd[3]));
    }
    __device__ static void finish(const Acc &, const I &, const Args &,
                                  const TreeView<T> &, int) {}
};

__global__ void fof_init_kernel(int32_t *__restrict__ parent, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        parent[i] = (int32_t)i;
}

// final labels: every index's root (its group's smallest index)
__global__ void fof_label_kernel(int32_t *__restrict__ parent, int64_t n,
                                 int64_t n_gas, int32_t *__restrict__ lg,
                                 int32_t *__restrict__ ld) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = fof_find(parent, (int)i);
        if (i < n_gas) lg[i] = r;
        else ld[i - n_gas] = r;
    }
}

__global__ void sum_counts_kernel(const int32_t *__restrict__ c, int64_t n,
                                  unsigned long long *__restrict__ total) {
    __shared__ unsigned long long part[256];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += (unsigned long long)c[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, part[0]);
}

// --------------------------------------------------------------------------
// gathers (caller order -> tree order, with derived per-particle fields)
// --------------------------------------------------------------------------

#define GRID_STRIDE(i, n)                                                     \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

inline unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 1048576) g = 1048576;
    return (unsigned)g;
}

template <typename T>
__global__ void gather1_kernel(const int32_t *__restrict__ perm,
                               const T *__restrict__ a, int64_t n,
                               T *__restrict__ out) {
    GRID_STRIDE(p, n) out[p] = a[perm[p]];
}

// masses of all tree slots (gas, then dm), times G
// (x, y, z, G m) per slot in tree order, for the float gravity pass
__global__ void gather_grav_packed_kernel(const int32_t *__restrict__ perm,
                                          const float *__restrict__ px,
                                          const float *__restrict__ py,
                                          const float *__restrict__ pz,
                                          const float *__restrict__ mg,
                                          const float *__restrict__ md,
                                          int64_t n_gas, int64_t n, float G,
                                          float4 *__restrict__ out) {
    GRID_STRIDE(p, n) {
        const int c = perm[p];
        out[p] = make_float4(px[p], py[p], pz[p],
                             G * (c < n_gas ? mg[c] : md[c - n_gas]));
    }
}

template <typename T>
__global__ void gather_mass_kernel(const int32_t *__restrict__ perm,
                                   const T *__restrict__ mg,
                                   const T *__restrict__ md, int64_t n_gas,
                                   int64_t n, T G, T *__restrict__ out) {
    GRID_STRIDE(p, n) {
        int c = perm[p];
        out[p] = G * (c < n_gas ? mg[c] : md[c - n_gas]);
    }
}

// The hydro field records, one thread per gas particle in caller order: the
// field planes are read with consecutive threads on consecutive particles
// (coalesced), the record is assembled in registers and stored whole, in
// 16-byte units, at the particle's slot iperm[c] (a record of S values per
// slot; entries past the fields written are zero).
template <typename T, int S>
__global__ void hydro_gather_kernel(
    const int32_t *__restrict__ iperm, int64_t n, const T *__restrict__ h,
    const T *__restrict__ vx, const T *__restrict__ vy,
    const T *__restrict__ vz, const T *__restrict__ V,
    const T *__restrict__ rho, const T *__restrict__ P,
    const T *__restrict__ cs, const T *__restrict__ A,
    const T *__restrict__ B, const T *__restrict__ gA,
    const T *__restrict__ gB, const GatherExtra<T> ex, T *__restrict__ f) {
    static_assert((S * sizeof(T)) % 16 == 0, "records of whole 16-byte units");
    GRID_STRIDE(c, n) {
        const int p = iperm[c];
        T r[S];
#pragma unroll
        for (int k = 0; k < S; ++k) r[k] = T(0);
        const T hh = h[p];
        const T N = (T)(1.0 / (PI_D * (double)hh * (double)hh * (double)hh));
        const T a = A[c] * N;
        r[0] = vx[c];
        r[1] = vy[c];
        r[2] = vz[c];
        r[3] = T(1) / (hh * hh);
        r[4] = a;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            r[5 + g] = gA[g * n + c] * N;
            r[8 + g] = B[g * n + c];
            r[11 + g] = a * B[g * n + c];
#pragma unroll
            for (int x = 0; x < 3; ++x) r[14 + 3 * g + x] = a * gB[(3 * g + x) * n + c];
        }
        r[23] = hh;
        r[24] = V[c];
        // (the velocity-gradient pass needs neither the state nor the mass)
        if (P) {
            r[25] = P[c];
            r[26] = rho[c];
            r[27] = cs[c];
        }
        if constexpr (S >= HF_RECON) {
            if (ex.dv) {
                const T *d = ex.dv + c;
                r[HF + 0] = d[0];
                r[HF + 1] = d[4 * n];
                r[HF + 2] = d[8 * n];
                r[HF + 3] = d[1 * n] + d[3 * n];
                r[HF + 4] = d[2 * n] + d[6 * n];
                r[HF + 5] = d[5 * n] + d[7 * n];
            }
        }
        // the kick's velocities: records of stride hydro_stride(HF + 3)
        // (after the plain fields) or hydro_stride(HF_MAX) (after the
        // reconstruction's)
        if constexpr (S == hydro_stride(HF + 3) || S == hydro_stride(HF_MAX)) {
            constexpr int W0 = S == hydro_stride(HF_MAX) ? HF_RECON : HF;
            const T *vv[3] = {vx, vy, vz};
            const double w =
                ex.bins ? kick_width(ex.dt, ex.L, ex.substep, ex.bins[c]) : ex.dt;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double acc = (double)ex.ag[q][c];
                if (ex.ah[q]) acc += (double)ex.ah[q][c];
                r[W0 + q] = (T)((double)vv[q][c] + w * acc);
            }
        }
        uint4 *dst = reinterpret_cast<uint4 *>(f + (int64_t)p * S);
        const uint4 *src = reinterpret_cast<const uint4 *>(r);
#pragma unroll
        for (int k = 0; k < (int)(S * sizeof(T) / 16); ++k) dst[k] = src[k];
    }
}

// --------------------------------------------------------------------------
// launch helpers
// --------------------------------------------------------------------------

template <typename T>
TreeView<T> tree_view(crk_tree *t, bool hydro, const int32_t *n_items) {
    TreeView<T> tv;
    const int cur = t->cur_nodes;
    tv.leaf_start = t->nd_start[cur].as<int32_t>();
    tv.leaf_count = t->nd_count[cur].as<int32_t>();
    tv.leaf_box = t->leaf_box.as<int32_t>();
    tv.list_off = hydro ? t->h_off.as<int64_t>() : t->g_off.as<int64_t>();
    tv.list = hydro ? t->h_list.as<uint32_t>() : t->g_list.as<uint32_t>();
    tv.n_items = n_items;
    tv.n_leaves = t->counters.as<int32_t>() + C_NN;
    tv.list_cap = hydro ? t->hydro_cap : t->grav_cap;
    tv.perm = t->perm.as<int32_t>();
    tv.px = t->pos[0].as<T>();
    tv.py = t->pos[1].as<T>();
    tv.pz = t->pos[2].as<T>();
    tv.h = t->hsm.as<T>();
    tv.lo = t->leaf_lo.as<T>();
    tv.hi = t->leaf_hi.as<T>();
    tv.hmax = t->leaf_hmax.as<T>();
    tv.lcap = t->leaf_cap;
    tv.xcd_remap = t->owner->tuning.xcd_remap;
    tv.tile = t->owner->tuning.tile;
    tv.walk_mask = t->owner->tuning.walk_mask;
    tv.groups = t->has_sub ? t->owner->tuning.sub_sweep : 0;
    tv.nsub = t->sub_nsub.as<int32_t>();
    tv.sst = t->sub_start.as<int32_t>();
    tv.scnt = t->sub_count.as<int32_t>();
    tv.slo = t->sub_lo.as<T>();
    tv.shi = t->sub_hi.as<T>();
    tv.shm = t->sub_hmax.as<T>();
    tv.sidx = nullptr;
    tv.jns = tv.nsub;
    tv.jst = tv.sst;
    tv.jcn = tv.scnt;
    tv.jlo = tv.slo;
    tv.jhi = tv.shi;
    tv.jhm = tv.shm;
    if (t->act_on && t->grp_on) {
        tv.nsub = t->grp_nsub.as<int32_t>();
        tv.scnt = t->grp_cnt.as<int32_t>();
        tv.sidx = t->grp_idx.as<int32_t>();
        tv.slo = t->grp_lo.as<T>();
        tv.shi = t->grp_hi.as<T>();
        tv.shm = t->grp_hmax.as<T>();
    }
    tv.rc = t->d_rc.as<double>();
    tv.eps = t->d_eps.as<double>();
    tv.n_gas = t->n_gas;
    tv.items = t->act_on ? t->act_items.as<int32_t>() : nullptr;
    tv.act = t->act_on ? t->act_flags.as<uint8_t>() : nullptr;
    tv.slist = tv.n_slist = nullptr;
    if (t->act_on && t->slist_on) {
        // n_items is the count of all active leaves (act_count[0]) or of
        // the active gas leaves ([1]); their entries are counted at [4], [5]
        const int32_t *c = t->act_count.as<int32_t>();
        tv.slist = t->act_slist.as<int32_t>();
        tv.n_slist = n_items == c ? c + 4 : c + 5;
    }
    return tv;
}

template <typename T, typename P>
int launch_pair(crk_ctx *ctx, crk_tree *t, const TreeView<T> &tv,
                const typename P::Args &pa, int64_t n_items_bound, int pass,
                bool gas_queue) {
    const int L = t->leaf_max;
    hipEvent_t ev = nullptr;
    const bool queue = ctx->tuning.grid_mult > 0 && t->orders_built && !t->act_on;
    int *head = nullptr;
    const int32_t *order = nullptr;
    unsigned grid = (unsigned)std::max<int64_t>(1, n_items_bound);
    if (queue) {
        // one queue head per launch slot so consecutive passes never share
        head = t->q_counter.as<int>() + (pass >= 0 ? pass : 15);
        order = gas_queue ? t->h_order.as<int32_t>() : t->g_order.as<int32_t>();
        CRK_HIP(fill_i32(head, 0, 1, ctx->stream));
        grid = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(n_items_bound,
                                 (int64_t)ctx->tuning.grid_mult * ctx->n_cu));
    }
    if (pass >= 0) span_begin(ctx, pass, true, &ev);
#define CRK_LAUNCH_PAIR(B)                                                      \
    if (queue)                                                                  \
        hipLaunchKernelGGL((pair_kernel_queue<T, P, B>), dim3(grid), dim3(B), 0, \
                           ctx->stream, tv, pa, order, head);                   \
    else                                                                        \
        hipLaunchKernelGGL((pair_kernel<T, P, B, SWEEP_BROADCAST>), dim3(grid), \
                           dim3(B), 0, ctx->stream, tv, pa);
    // the sub-leaf forms (split, leaf) have persistent queue forms of their
    // own; the walk and group forms run one workgroup per leaf only
    const int mode = L > 64 ? SWEEP_BROADCAST
                     : tv.groups == 2 ? SWEEP_SPLIT
                     : tv.groups == 3 ? SWEEP_LEAF
                     : queue ? SWEEP_BROADCAST
                     : ((ctx->tuning.walk_mask >> P::ID) & 1) ? SWEEP_WALK
                     : tv.groups == 1 ? SWEEP_GROUPED : SWEEP_BROADCAST;
    const size_t split_lds =
        (size_t)split_cap_of<T, P>(ctx->tuning.tile) * (P::NJ * sizeof(T) + 4);
    if (mode == SWEEP_LEAF && queue) {
        hipLaunchKernelGGL((pair_kernel_leaf_queue<T, P>), dim3(grid), dim3(256),
                           0, ctx->stream, tv, pa, order, head);
    } else if (mode == SWEEP_LEAF) {
        hipLaunchKernelGGL((pair_kernel_leaf<T, P>), dim3(grid), dim3(256), 0,
                           ctx->stream, tv, pa);
    } else if (mode == SWEEP_SPLIT && queue) {
        const unsigned g4 = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>(4 * n_items_bound,
                                 (int64_t)ctx->tuning.grid_mult * ctx->n_cu * 4));
        hipLaunchKernelGGL((pair_kernel_split_queue<T, P>), dim3(g4), dim3(64),
                           split_lds, ctx->stream, tv, pa, order, head);
    } else if (mode == SWEEP_SPLIT) {
        const unsigned g4 = (unsigned)std::max<int64_t>(1, 4 * n_items_bound);
        hipLaunchKernelGGL((pair_kernel_split<T, P>), dim3(g4), dim3(64),
                           split_lds, ctx->stream, tv, pa);
    } else if (mode == SWEEP_WALK) {
        hipLaunchKernelGGL((pair_kernel<T, P, 64, SWEEP_WALK>), dim3(grid),
                           dim3(64), 0, ctx->stream, tv, pa);
    } else if (mode == SWEEP_GROUPED) {
        hipLaunchKernelGGL((pair_kernel<T, P, 64, SWEEP_GROUPED>), dim3(grid),
                           dim3(64), 0, ctx->stream, tv, pa);
    } else if (L <= 64) {
        CRK_LAUNCH_PAIR(64)
    } else if (L <= 128) {
        CRK_LAUNCH_PAIR(128)
    } else {
        CRK_LAUNCH_PAIR(256)
    }
#undef CRK_LAUNCH_PAIR
    if (pass >= 0) span_end(ctx, pass, true, ev);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

// number of gas leaves lives in bin_leaf[total_bins]; all leaves in C_NN;
// with an active subset, the active leaves (gas first) and active gas
// leaves counted by crk_tree_set_active
inline const int32_t *gas_leaf_count(crk_tree *t) {
    if (t->act_on) return t->act_count.as<int32_t>() + 1;
    return t->bin_leaf.as<int32_t>() + t->total_bins;
}
inline const int32_t *all_leaf_count(crk_tree *t) {
    if (t->act_on) return t->act_count.as<int32_t>();
    return t->counters.as<int32_t>() + C_NN;
}
// launch bounds set by the tree build: the exact counts when built eagerly,
// the graph bounds (checked on the device) when built under capture; the
// active counts (read back by crk_tree_set_active) with an active subset
inline int64_t gas_bound(crk_ctx *, crk_tree *t) {
    return t->act_on ? t->act_ngas : t->ngb_launch;
}
inline int64_t all_bound(crk_ctx *, crk_tree *t) {
    return t->act_on ? t->act_nall : t->nb_launch;
}

template <typename T>
int density_impl(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                 void *rho_t, void *scratch) {
    const int64_t ng = t->n_gas;
    // masses in tree order: the tree's pass scratch, or (allocation-free
    // form) the caller's scratch, timed by no event either
    T *mt = static_cast<T *>(scratch);
    if (!mt) {
        CRK_TRY(t->pf[4].ensure(std::max<int64_t>(ng, 1) * sizeof(T), ctx->capturing));
        mt = t->pf[4].as<T>();
    }
    hipLaunchKernelGGL((gather1_kernel<T>), dim3(grid_for(ng)), dim3(256), 0,
                       ctx->stream, t->perm.as<int32_t>(),
                       static_cast<const T *>(m), ng, mt);
    CRK_HIP(hipGetLastError());
    typename DensityPass<T>::Args pa{mt, static_cast<T *>(V),
                                     static_cast<T *>(rho_t)};
    return launch_pair<T, DensityPass<T>>(ctx, t, tree_view<T>(t, true, gas_leaf_count(t)),
                                          pa, gas_bound(ctx, t),
                                          scratch ? -1 : P_DENSITY, true);
}

template <typename T>
int coeff_impl(crk_ctx *ctx, crk_tree *t, const void *m, const void *V,
               const void *u, void *A, void *B, void *gA, void *gB, void *rho,
               void *P, void *cs) {
    const int64_t ng = t->n_gas;
    const size_t bytes = std::max<int64_t>(ng, 1) * sizeof(T);
    for (int k = 4; k < 7; ++k) CRK_TRY(t->pf[k].ensure(bytes, ctx->capturing));
    T *mt = t->pf[4].as<T>(), *Vt = t->pf[5].as<T>(), *ut = t->pf[6].as<T>();
    const int32_t *perm = t->perm.as<int32_t>();
    hipLaunchKernelGGL((gather1_kernel<T>), dim3(grid_for(ng)), dim3(256), 0,
                       ctx->stream, perm, static_cast<const T *>(m), ng, mt);
    hipLaunchKernelGGL((gather1_kernel<T>), dim3(grid_for(ng)), dim3(256), 0,
                       ctx->stream, perm, static_cast<const T *>(V), ng, Vt);
    hipLaunchKernelGGL((gather1_kernel<T>), dim3(grid_for(ng)), dim3(256), 0,
                       ctx->stream, perm, static_cast<const T *>(u), ng, ut);
    CRK_HIP(hipGetLastError());
    typename CoeffPass<T>::Args pa{mt, Vt, ut,
                                   static_cast<T *>(A), static_cast<T *>(B),
                                   static_cast<T *>(gA), static_cast<T *>(gB),
                                   static_cast<T *>(rho), static_cast<T *>(P),
                                   static_cast<T *>(cs), ng, ctx->params.gamma};
    return launch_pair<T, CoeffPass<T>>(ctx, t, tree_view<T>(t, true, gas_leaf_count(t)),
                                        pa, gas_bound(ctx, t), P_COEFF, true);
}

// the hydro field records of every gas particle in tree order (pf[7]);
// P == nullptr: the kinematic and coefficient planes only (no state, no
// masses); dv != nullptr: also the reconstruction planes
template <typename T>
int hydro_fields(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
                 const void *vy, const void *vz, const void *V, const void *rho,
                 const void *P, const void *cs, const void *A, const void *B,
                 const void *gA, const void *gB, const GatherExtra<T> &ex) {
    const int64_t ng = t->n_gas;
    const size_t n1 = std::max<int64_t>(ng, 1);
    CRK_TRY(t->pf[7].ensure(n1 * hydro_stride(HF_MAX) * sizeof(T),
                            ctx->capturing));
    // the record stride of the fields this call writes (the passes read
    // records of the same stride: hydro_stride of their field count)
    const int S = hydro_stride(HF + (ex.dv ? 6 : 0) + (ex.ag[0] ? 3 : 0));
    CRK_TRY(t->pf[4].ensure(n1 * sizeof(T), ctx->capturing));
    const int32_t *ip = t->iperm.as<int32_t>();
    const T *hs = t->hsm.as<T>();
    const T *cvx = static_cast<const T *>(vx), *cvy = static_cast<const T *>(vy),
            *cvz = static_cast<const T *>(vz), *cV = static_cast<const T *>(V),
            *crho = static_cast<const T *>(rho), *cP = static_cast<const T *>(P),
            *ccs = static_cast<const T *>(cs), *cA = static_cast<const T *>(A),
            *cB = static_cast<const T *>(B), *cgA = static_cast<const T *>(gA),
            *cgB = static_cast<const T *>(gB);
    T *f = t->pf[7].as<T>();
    const dim3 g(grid_for(ng)), b(256);
    switch (S) {
    case hydro_stride(HF):
        hipLaunchKernelGGL((hydro_gather_kernel<T, hydro_stride(HF)>), g, b, 0,
                           ctx->stream, ip, ng, hs, cvx, cvy, cvz, cV, crho, cP,
                           ccs, cA, cB, cgA, cgB, ex, f);
        break;
    case hydro_stride(HF + 3):
        hipLaunchKernelGGL((hydro_gather_kernel<T, hydro_stride(HF + 3)>), g, b,
                           0, ctx->stream, ip, ng, hs, cvx, cvy, cvz, cV, crho,
                           cP, ccs, cA, cB, cgA, cgB, ex, f);
        break;
    case hydro_stride(HF_RECON):
        hipLaunchKernelGGL((hydro_gather_kernel<T, hydro_stride(HF_RECON)>), g, b,
                           0, ctx->stream, ip, ng, hs, cvx, cvy, cvz, cV, crho,
                           cP, ccs, cA, cB, cgA, cgB, ex, f);
        break;
    default:
        hipLaunchKernelGGL((hydro_gather_kernel<T, hydro_stride(HF_MAX)>), g, b,
                           0, ctx->stream, ip, ng, hs, cvx, cvy, cvz, cV, crho,
                           cP, ccs, cA, cB, cgA, cgB, ex, f);
        break;
    }
    CRK_HIP(hipGetLastError());
    // the masses in tree order (the force passes divide by them)
    if (P) {
        hipLaunchKernelGGL((gather1_kernel<T>), g, b, 0, ctx->stream,
                           t->perm.as<int32_t>(), static_cast<const T *>(m), ng,
                           t->pf[4].as<T>());
        CRK_HIP(hipGetLastError());
    }
    return CRK_OK;
}

template <typename T>
int hydro_impl(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
               const void *vy, const void *vz, const void *V, const void *rho,
               const void *P, const void *cs, const void *A, const void *B,
               const void *gA, const void *gB, const void *dv, double eta_c,
               double eta_f, void *ax, void *ay, void *az, void *dudt) {
    GatherExtra<T> ex;
    ex.dv = static_cast<const T *>(dv);
    CRK_TRY(hydro_fields<T>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB,
                            ex));
    const int64_t ng = t->n_gas;
    T *f = t->pf[7].as<T>(), *mt = t->pf[4].as<T>();
    const TreeView<T> tv = tree_view<T>(t, true, gas_leaf_count(t));
    if (dv) {
        typename HydroPass<T, true>::Args pa{
            f, ng, static_cast<T *>(ax), static_cast<T *>(ay),
            static_cast<T *>(az), static_cast<T *>(dudt), mt,
            (T)ctx->params.Cl, (T)ctx->params.Cq, (T)ctx->params.epsQ,
            (T)eta_c, (T)(1.0 / eta_f)};
        return launch_pair<T, HydroPass<T, true>>(ctx, t, tv, pa,
                                                  gas_bound(ctx, t), P_HYDRO, true);
    }
    typename HydroPass<T>::Args pa{f, ng, static_cast<T *>(ax),
                                   static_cast<T *>(ay), static_cast<T *>(az),
                                   static_cast<T *>(dudt), mt,
                                   (T)ctx->params.Cl, (T)ctx->params.Cq,
                                   (T)ctx->params.epsQ, T(0), T(0)};
    return launch_pair<T, HydroPass<T>>(ctx, t, tv, pa, gas_bound(ctx, t),
                                        P_HYDRO, true);
}

template <typename T>
int energy_impl(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
                const void *vy, const void *vz, const void *V, const void *rho,
                const void *P, const void *cs, const void *A, const void *B,
                const void *gA, const void *gB, const void *dv, double eta_c,
                double eta_f, double dt, const int32_t *bins, int L,
                int64_t substep, const void *const ag[3],
                const void *const ah[3], void *dudt) {
    GatherExtra<T> ex;
    ex.dv = static_cast<const T *>(dv);
    for (int a = 0; a < 3; ++a) {
        ex.ag[a] = static_cast<const T *>(ag[a]);
        ex.ah[a] = ah ? static_cast<const T *>(ah[a]) : nullptr;
    }
    ex.dt = dt;
    ex.bins = bins;
    ex.L = L;
    ex.substep = substep;
    CRK_TRY(hydro_fields<T>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB,
                            ex));
    const int64_t ng = t->n_gas;
    T *f = t->pf[7].as<T>(), *mt = t->pf[4].as<T>();
    const TreeView<T> tv = tree_view<T>(t, true, gas_leaf_count(t));
    if (dv) {
        typename HydroPass<T, true, true>::Args pa{
            f, ng, nullptr, nullptr, nullptr, static_cast<T *>(dudt), mt,
            (T)ctx->params.Cl, (T)ctx->params.Cq, (T)ctx->params.epsQ,
            (T)eta_c, (T)(1.0 / eta_f)};
        return launch_pair<T, HydroPass<T, true, true>>(ctx, t, tv, pa,
                                                        gas_bound(ctx, t), P_ENERGY,
                                                        true);
    }
    typename HydroPass<T, false, true>::Args pa{
        f, ng, nullptr, nullptr, nullptr, static_cast<T *>(dudt), mt,
        (T)ctx->params.Cl, (T)ctx->params.Cq, (T)ctx->params.epsQ, T(0), T(0)};
    return launch_pair<T, HydroPass<T, false, true>>(ctx, t, tv, pa,
                                                     gas_bound(ctx, t), P_ENERGY,
                                                     true);
}

template <typename T>
int vgrad_impl(crk_ctx *ctx, crk_tree *t, const void *vx, const void *vy,
               const void *vz, const void *V, const void *A, const void *B,
               const void *gA, const void *gB, void *dv) {
    CRK_TRY(hydro_fields<T>(ctx, t, nullptr, vx, vy, vz, V, nullptr, nullptr,
                            nullptr, A, B, gA, gB, GatherExtra<T>()));
    typename VGradPass<T>::Args pa{t->pf[7].as<T>(), t->n_gas,
                                   static_cast<T *>(dv)};
    return launch_pair<T, VGradPass<T>>(ctx, t, tree_view<T>(t, true, gas_leaf_count(t)),
                                        pa, gas_bound(ctx, t), P_VGRAD, true);
}

template <typename T>
int gravity_impl(crk_ctx *ctx, crk_tree *t, const void *mg, const void *md,
                 void *axg, void *ayg, void *azg, void *axd, void *ayd,
                 void *azd) {
    const int64_t n = t->n;
    CRK_TRY(t->pf[8].ensure(std::max<int64_t>(n, 1) * sizeof(T), ctx->capturing));
    T *mt = t->pf[8].as<T>();
    hipLaunchKernelGGL((gather_mass_kernel<T>), dim3(grid_for(n)), dim3(256), 0,
                       ctx->stream, t->perm.as<int32_t>(),
                       static_cast<const T *>(mg), static_cast<const T *>(md),
                       t->n_gas, n, (T)ctx->params.G, mt);
    const float4 *pk = nullptr;
    if constexpr (std::is_same<T, float>::value) {
        CRK_TRY(t->pf[11].ensure(std::max<int64_t>(n, 1) * sizeof(float4),
                                 ctx->capturing));
        hipLaunchKernelGGL(gather_grav_packed_kernel, dim3(grid_for(n)), dim3(256),
                           0, ctx->stream, t->perm.as<int32_t>(),
                           t->pos[0].as<float>(), t->pos[1].as<float>(),
                           t->pos[2].as<float>(), static_cast<const float *>(mg),
                           static_cast<const float *>(md), t->n_gas, n,
                           (float)ctx->params.G, t->pf[11].as<float4>());
        pk = t->pf[11].as<float4>();
    }
    CRK_HIP(hipGetLastError());
    typename GravityPass<T>::Args pa{mt,
                                     static_cast<T *>(axg), static_cast<T *>(ayg),
                                     static_cast<T *>(azg), static_cast<T *>(axd),
                                     static_cast<T *>(ayd), static_cast<T *>(azd),
                                     t->n_gas, pk};
    return launch_pair<T, GravityPass<T>>(ctx, t, tree_view<T>(t, false, all_leaf_count(t)),
                                          pa, all_bound(ctx, t), P_GRAV, false);
}

template <typename T>
int count_impl(crk_ctx *ctx, crk_tree *t, int64_t totals[6]) {
    const int64_t n = t->n;
    CRK_TRY(t->pf[9].ensure(std::max<int64_t>(n, 1) * 4, ctx->capturing));
    int32_t *cnt = t->pf[9].as<int32_t>();
    unsigned long long *tot =
        reinterpret_cast<unsigned long long *>(t->counters.as<int64_t>() + 16);
    CRK_HIP(fill_i64(reinterpret_cast<int64_t *>(tot), 0, 6, ctx->stream));
    for (int mode = 0; mode < 6; ++mode) {
        const bool gas = mode % 3 < 2;
        CRK_HIP(fill_i32(cnt, 0, n, ctx->stream));
        typename CountPass<T>::Args pa{mode, cnt};
        CRK_TRY((launch_pair<T, CountPass<T>>(
            ctx, t, tree_view<T>(t, gas, gas ? gas_leaf_count(t) : all_leaf_count(t)),
            pa, gas ? gas_bound(ctx, t) : all_bound(ctx, t), -1, gas)));
        hipLaunchKernelGGL(sum_counts_kernel, dim3(256), dim3(256), 0, ctx->stream,
                           cnt, gas ? t->n_gas : n, tot + mode);
        CRK_HIP(hipGetLastError());
    }
    int64_t *hb = ctx->err_host.as<int64_t>() + 16;
    CRK_HIP(hipMemcpyAsync(hb, tot, 48, hipMemcpyDeviceToHost, ctx->stream));
    CRK_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 6; ++k) totals[k] = hb[k];
    return CRK_OK;
}

template <typename T>
int fof_impl(crk_ctx *ctx, crk_tree *t, double b, int32_t *lg, int32_t *ld) {
    const int64_t n = t->n;
    CRK_TRY(t->pf[10].ensure(std::max<int64_t>(n, 1) * 4, ctx->capturing));
    int32_t *parent = t->pf[10].as<int32_t>();
    hipLaunchKernelGGL(fof_init_kernel, dim3(grid_for(n)), dim3(256), 0,
                       ctx->stream, parent, n);
    CRK_HIP(hipGetLastError());
    typename FofPass<T>::Args pa{parent, b};
    CRK_TRY((launch_pair<T, FofPass<T>>(ctx, t,
                                         tree_view<T>(t, false, all_leaf_count(t)),
                                         pa, all_bound(ctx, t), -1, false)));
    hipLaunchKernelGGL(fof_label_kernel, dim3(grid_for(n)), dim3(256), 0,
                       ctx->stream, parent, n, t->n_gas, lg, ld);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

}  // namespace

int fof_groups(crk_ctx *ctx, crk_tree *t, double b, int32_t *labels_gas,
               int32_t *labels_dm) {
    if (ctx->precision == CRK_FP64) return fof_impl<double>(ctx, t, b, labels_gas, labels_dm);
    return fof_impl<float>(ctx, t, b, labels_gas, labels_dm);
}

int pass_density(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                 void *rho_tilde) {
    if (ctx->precision == CRK_FP64)
        return density_impl<double>(ctx, t, m, V, rho_tilde, nullptr);
    return density_impl<float>(ctx, t, m, V, rho_tilde, nullptr);
}

int pass_density_scratch(crk_ctx *ctx, crk_tree *t, const void *m, void *V,
                         void *rho_tilde, void *scratch) {
    if (ctx->precision == CRK_FP64)
        return density_impl<double>(ctx, t, m, V, rho_tilde, scratch);
    return density_impl<float>(ctx, t, m, V, rho_tilde, scratch);
}

int pass_coefficients(crk_ctx *ctx, crk_tree *t, const void *m, const void *V,
                      const void *u, void *A, void *B, void *gradA,
                      void *gradB, void *rho, void *P, void *cs) {
    if (ctx->precision == CRK_FP64)
        return coeff_impl<double>(ctx, t, m, V, u, A, B, gradA, gradB, rho, P, cs);
    return coeff_impl<float>(ctx, t, m, V, u, A, B, gradA, gradB, rho, P, cs);
}

int pass_hydro(crk_ctx *ctx, crk_tree *t, const void *m, const void *vx,
               const void *vy, const void *vz, const void *V, const void *rho,
               const void *P, const void *cs, const void *A, const void *B,
               const void *gradA, const void *gradB, const void *dv,
               double eta_crit, double eta_fold, void *ax, void *ay, void *az,
               void *dudt) {
    if (ctx->precision == CRK_FP64)
        return hydro_impl<double>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B,
                                  gradA, gradB, dv, eta_crit, eta_fold, ax, ay,
                                  az, dudt);
    return hydro_impl<float>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA,
                             gradB, dv, eta_crit, eta_fold, ax, ay, az, dudt);
}

int pass_energy_compatible(crk_ctx *ctx, crk_tree *t, const void *m,
                           const void *vx, const void *vy, const void *vz,
                           const void *V, const void *rho, const void *P,
                           const void *cs, const void *A, const void *B,
                           const void *gradA, const void *gradB, const void *dv,
                           double eta_crit, double eta_fold, double dt,
                           const int32_t *bins, int max_level, int64_t substep,
                           const void *const a_grav[3],
                           const void *const a_hydro[3], void *dudt) {
    if (ctx->precision == CRK_FP64)
        return energy_impl<double>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B,
                                   gradA, gradB, dv, eta_crit, eta_fold, dt,
                                   bins, max_level, substep, a_grav, a_hydro,
                                   dudt);
    return energy_impl<float>(ctx, t, m, vx, vy, vz, V, rho, P, cs, A, B, gradA,
                              gradB, dv, eta_crit, eta_fold, dt, bins,
                              max_level, substep, a_grav, a_hydro, dudt);
}

int pass_velocity_gradient(crk_ctx *ctx, crk_tree *t, const void *vx,
                           const void *vy, const void *vz, const void *V,
                           const void *A, const void *B, const void *gradA,
                           const void *gradB, void *dv) {
    if (ctx->precision == CRK_FP64)
        return vgrad_impl<double>(ctx, t, vx, vy, vz, V, A, B, gradA, gradB, dv);
    return vgrad_impl<float>(ctx, t, vx, vy, vz, V, A, B, gradA, gradB, dv);
}

int count_pairs(crk_ctx *ctx, crk_tree *t, int64_t totals[6]) {
    if (ctx->precision == CRK_FP64) return count_impl<double>(ctx, t, totals);
    return count_impl<float>(ctx, t, totals);
}

int pass_gravity(crk_ctx *ctx, crk_tree *t, const void *m_gas,
                 const void *m_dm, void *ax_gas, void *ay_gas, void *az_gas,
                 void *ax_dm, void *ay_dm, void *az_dm) {
    if (ctx->precision == CRK_FP64)
        return gravity_impl<double>(ctx, t, m_gas, m_dm, ax_gas, ay_gas, az_gas,
                                    ax_dm, ay_dm, az_dm);
    return gravity_impl<float>(ctx, t, m_gas, m_dm, ax_gas, ay_gas, az_gas,
                               ax_dm, ay_dm, az_dm);
}

}  // namespace crk
