// build_interaction_lists: leaf-leaf interaction lists (Sec. IV-B.1).
//
// One wavefront per i-leaf takes the leaves of the 27 chaining-mesh bins
// around the leaf's bin (own box, periodic images), both species, as one
// flattened candidate sequence, and tests the bounding box of every
// candidate leaf against its own in double precision.  Accepted leaves are
// compacted with a ballot, so each list is in a fixed order (stencil order,
// species, leaf index) independent of scheduling.  Two passes: count, then
// (after a prefix sum) fill.
//   gravity: all species, range r_c of the box
//   hydro:   gas i-leaves only, gas j-leaves, range 2 max(h_max_I, h_max_J)
// Ranges are widened by a relative 1e-5 so that every pair a float32 pair
// test could accept is in the list; the pass kernels apply the exact test.
#include <algorithm>

#include "crk_internal.h"

namespace crk {

namespace {

constexpr int LB = 256;  // four wavefronts = four i-leaves per workgroup
constexpr double RANGE_WIDEN = 1.0 + 1e-5;

template <typename T>
__global__ __launch_bounds__(LB) void lists_kernel(
    int fill, const int32_t *__restrict__ nn_ptr, int64_t cap,
    const int32_t *__restrict__ leaf_key, const int32_t *__restrict__ leaf_box,
    const T *__restrict__ lo_, const T *__restrict__ hi_,
    const T *__restrict__ lhmax, const int32_t *__restrict__ bin_leaf,
    int64_t total_bins, const int *__restrict__ ncm,
    const int64_t *__restrict__ bin_base, const double *__restrict__ rc,
    const int32_t *__restrict__ leaf_count, int32_t *__restrict__ g_cost,
    int32_t *__restrict__ h_cost,
    int32_t *__restrict__ g_cnt, int32_t *__restrict__ h_cnt,
    const int64_t *__restrict__ g_off, const int64_t *__restrict__ h_off,
    uint32_t *__restrict__ g_list, uint32_t *__restrict__ h_list,
    int64_t g_cap, int64_t h_cap, const int32_t *__restrict__ act_leaf,
    int *__restrict__ err) {
    const int lane = threadIdx.x & 63;
    const int64_t I = (int64_t)blockIdx.x * (LB / 64) + (threadIdx.x >> 6);
    const int64_t nn = *nn_ptr;
    if (I >= nn) return;  // whole wavefront leaves together
    // with an active subset only the active leaves get lists (the others
    // keep the zero counts filled before the launch)
    if (act_leaf && !act_leaf[I]) return;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int key = leaf_key[I];
    const bool gasI = key < total_bins;
    const int64_t gbin = gasI ? key : key - total_bins;
    const int b = leaf_box[I];
    const int nc = ncm[b];
    const int64_t lb = gbin - bin_base[b];
    const int cx = (int)(lb / ((int64_t)nc * nc));
    const int cy = (int)((lb / nc) % nc);
    const int cz = (int)(lb % nc);
    double loI[3], hiI[3];
    for (int a = 0; a < 3; ++a) {
        loI[a] = (double)lo_[a * cap + I];
        hiI[a] = (double)hi_[a * cap + I];
    }
    const double hmI = (double)lhmax[I];
    const double Rg = rc[b] * RANGE_WIDEN;
    const double Rg2 = Rg * Rg;
    int64_t gpos = fill ? g_off[I] : 0;
    int64_t hpos = fill ? h_off[I] : 0;
    int32_t gc = 0, hc = 0;
    int64_t gcost = 0, hcost = 0;  // candidate j particles (per lane)
    // The 54 candidate ranges (27 stencil bins x 2 species, stencil order,
    // species inner) are flattened: lane q2 < 54 computes range q2, a wave
    // prefix sum gives their offsets, and every lane then takes candidates
    // c = lane, lane + 64, ... in that flattened order.
    int r0 = 0, rlen = 0;
    uint32_t rcode = 0;
    if (lane < 54) {
        const int q = lane >> 1, sp = lane & 1;
        const int ox = q / 9 - 1, oy = (q / 3) % 3 - 1, oz = q % 3 - 1;
        int nx = cx + ox, ny = cy + oy, nz = cz + oz;
        int sx = 0, sy = 0, sz = 0;
        if (nx < 0) { nx += nc; sx = -1; } else if (nx >= nc) { nx -= nc; sx = 1; }
        if (ny < 0) { ny += nc; sy = -1; } else if (ny >= nc) { ny -= nc; sy = 1; }
        if (nz < 0) { nz += nc; sz = -1; } else if (nz >= nc) { nz -= nc; sz = 1; }
        const int64_t ngbin = bin_base[b] + ((int64_t)nx * nc + ny) * nc + nz;
        const int64_t k = sp * total_bins + ngbin;
        r0 = bin_leaf[k];
        rlen = bin_leaf[k + 1] - r0;
        rcode = (uint32_t)((sx + 1) * 9 + (sy + 1) * 3 + (sz + 1)) | ((uint32_t)sp << 8);
    }
    // inclusive scan of the range lengths across the wave
    int incl = rlen;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const int total = __shfl(incl, 63);
    const int excl = incl - rlen;
    for (int base = 0; base < total; base += 64) {
        const int c = base + lane;
        const bool valid = c < total;
        // range of candidate c: the last q2 with excl(q2) <= c (binary
        // lifting over the lanes, same six steps on every lane; lanes 54-63
        // hold excl = total, which no valid c reaches)
        int q2 = 0;
        for (int step = 32; step > 0; step >>= 1) {
            const int em = __shfl(excl, q2 + step);
            if (em <= c) q2 += step;
        }
        const int J = __shfl(r0, q2) + (c - __shfl(excl, q2));
        const uint32_t rc_ = __shfl(rcode, q2);
        const uint32_t code = rc_ & 0xFFu;
        const int sp = (int)(rc_ >> 8);
        const int sx = (int)(code / 9u) - 1, sy = (int)((code / 3u) % 3u) - 1,
                  sz = (int)(code % 3u) - 1;
        bool gok = false, hok = false;
        if (valid) {
            const double S[3] = {(double)sx, (double)sy, (double)sz};
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double l = (double)lo_[a * cap + J] + S[a];
                double h = (double)hi_[a * cap + J] + S[a];
                double g = fmax(0.0, fmax(l - hiI[a], loI[a] - h));
                d2 += g * g;
            }
            gok = d2 < Rg2;
            if (gasI && sp == 0) {
                double hm = fmax(hmI, (double)lhmax[J]);
                double Rh = 2.0 * hm * RANGE_WIDEN;
                hok = d2 < Rh * Rh;
            }
        }
        if (!fill) {
            if (gok) gcost += leaf_count[J];
            if (hok) hcost += leaf_count[J];
        }
        const uint64_t gm = __ballot(gok);
        const uint64_t hm = __ballot(hok);
        if (fill) {
            if (gok) {
                int64_t p = gpos + __popcll(gm & lt_mask);
                if (p < g_cap) g_list[p] = (uint32_t)J | (code << LIST_LEAF_BITS);
                else atomicOr(err, DEV_ERR_CAPACITY);
            }
            if (hok) {
                int64_t p = hpos + __popcll(hm & lt_mask);
                if (p < h_cap) h_list[p] = (uint32_t)J | (code << LIST_LEAF_BITS);
                else atomicOr(err, DEV_ERR_CAPACITY);
            }
        }
        gpos += __popcll(gm);
        hpos += __popcll(hm);
        gc += __popcll(gm);
        hc += __popcll(hm);
    }
    if (!fill) {
        // queue cost = i particles x candidate j particles
        for (int off = 32; off > 0; off >>= 1) {
            gcost += __shfl_xor(gcost, off);
            hcost += __shfl_xor(hcost, off);
        }
        if (lane == 0) {
            const int64_t ci = leaf_count[I];
            g_cnt[I] = gc;
            h_cnt[I] = hc;
            g_cost[I] = (int32_t)min(ci * gcost, (int64_t)0x7FFFFFFF);
            h_cost[I] = gasI ? (int32_t)min(ci * hcost, (int64_t)0x7FFFFFFF) : -1;
        }
    }
}

// Queue keys: cost-descending, ties by leaf index (stable sort); slots
// beyond the leaf count (and dm leaves for the hydro queue) sort last.
__global__ void order_keys_kernel(const int32_t *__restrict__ cost,
                                  const int32_t *__restrict__ nn_ptr,
                                  int64_t cap, uint64_t *__restrict__ k,
                                  int32_t *__restrict__ v) {
    const int64_t nn = *nn_ptr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = i < nn ? cost[i] : -1;
        k[i] = c >= 0 ? (uint64_t)(0x7FFFFFFF - c) : 0xFFFFFFFFull;
        v[i] = (int32_t)i;
    }
}

__global__ void copy_order_kernel(const int32_t *__restrict__ a,
                                  int32_t *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename T>
int lists_impl(crk_ctx *ctx, crk_tree *t) {
    hipStream_t s = ctx->stream;
    const bool cap = ctx->capturing;
    const int64_t lcap = t->leaf_cap;
    const int cur = t->cur_nodes;
    int32_t *cnt = t->counters.as<int32_t>();
    int64_t *cnt64 = t->counters.as<int64_t>();
    int *err = dev_err_word(ctx);
    CRK_TRY(t->g_cnt.ensure((lcap + 1) * 4, cap));
    CRK_TRY(t->g_cost.ensure((lcap + 1) * 4, cap));
    CRK_TRY(t->h_cost.ensure((lcap + 1) * 4, cap));
    CRK_TRY(t->h_cnt.ensure((lcap + 1) * 4, cap));
    CRK_TRY(t->g_off.ensure((lcap + 1) * 8, cap));
    CRK_TRY(t->h_off.ensure((lcap + 1) * 8, cap));
    CRK_TRY(ctx->scratch.ensure(scan_tmp_bytes(lcap + 1), cap));
    // leaves in [0, nbl) at most: the tree build's launch bound
    const int64_t nbl = std::max<int64_t>(1, t->nb_launch);
    CRK_HIP(fill_i32(t->g_cnt.as<int32_t>(), 0, nbl + 1, s));
    CRK_HIP(fill_i32(t->h_cnt.as<int32_t>(), 0, nbl + 1, s));
    const unsigned grid = (unsigned)((nbl + 3) / 4);
    auto launch = [&](int fill) -> int {
        hipLaunchKernelGGL((lists_kernel<T>), dim3(grid), dim3(LB), 0, s, fill,
                           cnt + C_NN, lcap, t->nd_key[cur].as<int32_t>(),
                           t->leaf_box.as<int32_t>(), t->leaf_lo.as<T>(),
                           t->leaf_hi.as<T>(), t->leaf_hmax.as<T>(),
                           t->bin_leaf.as<int32_t>(), t->total_bins,
                           t->d_ncm.as<int>(), t->d_bin_base.as<int64_t>(),
                           t->d_rc.as<double>(), t->nd_count[cur].as<int32_t>(),
                           t->g_cost.as<int32_t>(), t->h_cost.as<int32_t>(),
                           t->g_cnt.as<int32_t>(),
                           t->h_cnt.as<int32_t>(), t->g_off.as<int64_t>(),
                           t->h_off.as<int64_t>(), t->g_list.as<uint32_t>(),
                           t->h_list.as<uint32_t>(), t->grav_cap, t->hydro_cap,
                           t->act_on ? t->act_leaf.as<int32_t>() : nullptr, err);
        CRK_HIP(hipGetLastError());
        return CRK_OK;
    };
    CRK_TRY(launch(0));
    CRK_HIP(exclusive_scan_i32_to_i64(t->g_cnt.as<int32_t>(), t->g_off.as<int64_t>(),
                                      nbl + 1, cnt64 + C64_GTOT, ctx->scratch.p, s));
    CRK_HIP(exclusive_scan_i32_to_i64(t->h_cnt.as<int32_t>(), t->h_off.as<int64_t>(),
                                      nbl + 1, cnt64 + C64_HTOT, ctx->scratch.p, s));
    if (!cap) {
        int64_t *hb = ctx->err_host.as<int64_t>() + 8;
        CRK_HIP(hipMemcpyAsync(hb, cnt64 + C64_GTOT, 16, hipMemcpyDeviceToHost, s));
        CRK_HIP(hipStreamSynchronize(s));
        t->grav_entries = hb[0];
        t->hydro_entries = hb[1];
        if (t->grav_entries > t->grav_cap) {
            int64_t c = t->grav_entries + t->grav_entries / 8 + 1024;
            CRK_TRY(t->g_list.ensure((size_t)c * 4, false));
            t->grav_cap = c;
        }
        if (t->hydro_entries > t->hydro_cap) {
            int64_t c = t->hydro_entries + t->hydro_entries / 8 + 1024;
            CRK_TRY(t->h_list.ensure((size_t)c * 4, false));
            t->hydro_cap = c;
        }
    }
    CRK_TRY(launch(1));
    // cost-ordered work queues for the persistent pass kernels
    t->orders_built = false;
    if (ctx->tuning.grid_mult > 0) {
        // buffers sized by the capacity (no growth under capture), work
        // over the launch bound
        const int64_t mc = lcap + 1;
        const int64_t m = nbl + 1;
        for (int i = 0; i < 2; ++i) {
            CRK_TRY(t->ord_k[i].ensure(mc * 8, cap));
            CRK_TRY(t->ord_v[i].ensure(mc * 4, cap));
        }
        CRK_TRY(t->g_order.ensure(mc * 4, cap));
        CRK_TRY(t->h_order.ensure(mc * 4, cap));
        CRK_TRY(t->q_counter.ensure(64, cap));
        CRK_TRY(ctx->scratch.ensure(radix_tmp_bytes(mc), cap));
        uint64_t *K[2] = {t->ord_k[0].as<uint64_t>(), t->ord_k[1].as<uint64_t>()};
        int32_t *V[2] = {t->ord_v[0].as<int32_t>(), t->ord_v[1].as<int32_t>()};
        const unsigned g = (unsigned)std::min<int64_t>((m + 255) / 256, 65536);
        for (int h = 0; h < 2; ++h) {
            hipLaunchKernelGGL(order_keys_kernel, dim3(g), dim3(256), 0, s,
                               h ? t->h_cost.as<int32_t>() : t->g_cost.as<int32_t>(),
                               cnt + C_NN, m, K[0], V[0]);
            CRK_HIP(hipGetLastError());
            hipError_t he;
            int r = radix_sort_u64_i32(K, V, m, 32, ctx->scratch.p, s, &he);
            CRK_HIP(he);
            hipLaunchKernelGGL(copy_order_kernel, dim3(g), dim3(256), 0, s, V[r],
                               h ? t->h_order.as<int32_t>() : t->g_order.as<int32_t>(),
                               m);
            CRK_HIP(hipGetLastError());
        }
        t->orders_built = true;
    }
    t->lists_built = true;
    return CRK_OK;
}

}  // namespace

int lists_build(crk_ctx *ctx, crk_tree *t) {
    if (ctx->precision == CRK_FP64) return lists_impl<double>(ctx, t);
    return lists_impl<float>(ctx, t);
}

}  // namespace crk
