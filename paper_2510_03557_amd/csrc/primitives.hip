// Device-wide primitives used by the tree and list builders: exclusive
// prefix sums, a stable LSD radix sort of (uint64 key, int32 value) pairs and
// fill kernels.  Written for wave64 (gfx950): workgroups of 256 threads =
// four waves, wave-level ranking with 64-bit ballots.
#include "crk_internal.h"

namespace crk {

template <typename T>
__global__ void fill_kernel_any(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Inclusive workgroup scan of one value per thread (Hillis-Steele in LDS).
template <typename T>
__device__ T block_inclusive_scan(T v, T *lds) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        T add = (t >= off) ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    T r = lds[t];
    __syncthreads();
    return r;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce_kernel(
    const Tin *__restrict__ in, int64_t n, Tout *__restrict__ partial) {
    __shared__ Tout lds[SCAN_THREADS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    Tout s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)k * SCAN_THREADS + threadIdx.x;
        if (i < n) s += (Tout)in[i];
    }
    Tout tot = block_inclusive_scan<Tout>(s, lds);
    if (threadIdx.x == SCAN_THREADS - 1) partial[blockIdx.x] = tot;
}

// Exclusive scan of the per-tile partial sums by one workgroup.
template <typename Tout>
__global__ __launch_bounds__(SCAN_THREADS) void scan_partials_kernel(
    Tout *__restrict__ partial, int64_t nb, Tout *__restrict__ d_total) {
    __shared__ Tout lds[SCAN_THREADS];
    Tout carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
        int64_t i = base + threadIdx.x;
        Tout v = (i < nb) ? partial[i] : Tout(0);
        Tout inc = block_inclusive_scan<Tout>(v, lds);
        if (i < nb) partial[i] = carry + inc - v;
        // the last thread's inclusive value is the chunk total
        if (threadIdx.x == SCAN_THREADS - 1) lds[0] = inc;
        __syncthreads();
        carry += lds[0];
        __syncthreads();
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

// Each thread owns SCAN_ITEMS consecutive elements of the tile.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_THREADS) void scan_apply_kernel(
    const Tin *__restrict__ in, Tout *__restrict__ out, int64_t n,
    const Tout *__restrict__ partial) {
    __shared__ Tout lds[SCAN_THREADS];
    const int64_t base =
        (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    Tout v[SCAN_ITEMS];
    Tout s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? (Tout)in[i] : Tout(0);
        s += v[k];
    }
    Tout inc = block_inclusive_scan<Tout>(s, lds);
    Tout run = partial[blockIdx.x] + inc - s;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

template <typename Tin, typename Tout>
hipError_t exclusive_scan_impl(const Tin *in, Tout *out, int64_t n,
                               Tout *d_total, void *tmp, hipStream_t s) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    Tout *partial = static_cast<Tout *>(tmp);
    if (n > 0)
        hipLaunchKernelGGL((scan_reduce_kernel<Tin, Tout>), dim3((unsigned)nb),
                           dim3(SCAN_THREADS), 0, s, in, n, partial);
    else
        hipLaunchKernelGGL((fill_kernel_any<Tout>), dim3(1), dim3(64), 0, s,
                           partial, Tout(0), (int64_t)1);
    hipLaunchKernelGGL((scan_partials_kernel<Tout>), dim3(1),
                       dim3(SCAN_THREADS), 0, s, partial, nb, d_total);
    if (n > 0)
        hipLaunchKernelGGL((scan_apply_kernel<Tin, Tout>), dim3((unsigned)nb),
                           dim3(SCAN_THREADS), 0, s, in, out, n, partial);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// radix sort
// --------------------------------------------------------------------------

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;  // elements per thread per tile
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / 64;

__global__ __launch_bounds__(RS_THREADS) void radix_hist_kernel(
    const uint64_t *__restrict__ keys, int64_t n, int shift, int nblocks,
    int32_t *__restrict__ hist) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: element order inside a tile is round-major, then thread;
// equal digits keep that order.  Ranks inside a wave come from matching the
// digit bit by bit with ballots; ranks across the tile from per-wave digit
// counts in LDS.
__global__ __launch_bounds__(RS_THREADS) void radix_scatter_kernel(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
    int shift, int nblocks, const int32_t *__restrict__ offs) {
    __shared__ int32_t wcount[RS_WAVES][256];
    __shared__ int32_t running[256];
    __shared__ int32_t goff[256];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    goff[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    running[t] = 0;
    for (int w = 0; w < RS_WAVES; ++w) wcount[w][t] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int64_t i = base + (int64_t)r * RS_THREADS + t;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        int32_t val = valid ? vin[i] : 0;
        uint32_t d = (uint32_t)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcount[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = running[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][d];
            int64_t dst = (int64_t)goff[d] + pos;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int32_t add = 0;
        for (int w = 0; w < RS_WAVES; ++w) {
            add += wcount[w][t];
            wcount[w][t] = 0;
        }
        running[t] += add;
        __syncthreads();
    }
}

}  // namespace

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel_any<int32_t>, dim3((unsigned)blocks),
                       dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel_any<int64_t>, dim3((unsigned)blocks),
                       dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE + 1;
    return (size_t)nb * sizeof(int64_t) + 256;
}

hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n,
                              int32_t *d_total, void *tmp, hipStream_t s) {
    return exclusive_scan_impl<int32_t, int32_t>(in, out, n, d_total, tmp, s);
}

hipError_t exclusive_scan_i32_to_i64(const int32_t *in, int64_t *out,
                                     int64_t n, int64_t *d_total, void *tmp,
                                     hipStream_t s) {
    return exclusive_scan_impl<int32_t, int64_t>(in, out, n, d_total, tmp, s);
}

size_t radix_tmp_bytes(int64_t n) {
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    if (nb == 0) nb = 1;
    size_t hist = (size_t)nb * 256 * sizeof(int32_t);
    hist = (hist + 255) & ~size_t(255);
    return 2 * hist + scan_tmp_bytes(nb * 256);
}

int radix_sort_u64_i32(uint64_t *keys[2], int32_t *vals[2], int64_t n,
                       int bits, void *tmp, hipStream_t s, hipError_t *err) {
    *err = hipSuccess;
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    if (nb == 0 || n <= 1) return 0;
    size_t hist_bytes = ((size_t)nb * 256 * sizeof(int32_t) + 255) & ~size_t(255);
    int32_t *hist = static_cast<int32_t *>(tmp);
    int32_t *offs = reinterpret_cast<int32_t *>(static_cast<char *>(tmp) + hist_bytes);
    void *stmp = static_cast<char *>(tmp) + 2 * hist_bytes;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb),
                           dim3(RS_THREADS), 0, s, keys[cur], n, shift,
                           (int)nb, hist);
        *err = exclusive_scan_i32(hist, offs, nb * 256, nullptr, stmp, s);
        if (*err != hipSuccess) return cur;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb),
                           dim3(RS_THREADS), 0, s, keys[cur], vals[cur],
                           keys[cur ^ 1], vals[cur ^ 1], n, shift, (int)nb,
                           offs);
        *err = hipGetLastError();
        if (*err != hipSuccess) return cur;
        cur ^= 1;
    }
    return cur;
}

}  // namespace crk
