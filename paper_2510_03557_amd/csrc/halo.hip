// Group properties of a friends-of-friends labelling (the in-situ halo
// finding of Sec. IV-B.3): per group, indexed by its label (the smallest
// combined caller index of its members), the member count, the total mass
// and the periodic centre of mass -- every member taken at its minimum
// image about the labelling particle, the mass-weighted mean of those
// images in double, wrapped into [1, 2).  One thread per particle adds its
// contributions with atomics (double sums: the order of the additions, and
// so the last bits, can differ from run to run); a second pass turns the
// sums into centres.  Elementwise and atomic-bound.
#include <algorithm>
#include <cmath>

#include "crk_internal.h"

namespace crk {

namespace {

inline unsigned grid_halo(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)std::max<int64_t>(1, g);
}

template <typename T> struct HaloIn {
    int64_t ng, n;
    const int32_t *lg, *ld;
    const T *g[3], *d[3];
    const T *mg, *md;
    __device__ double pos(int64_t q, int a) const {
        return q < ng ? (double)g[a][q] : (double)d[a][q - ng];
    }
};

template <typename T>
__global__ void halo_sum_kernel(const HaloIn<T> in, int32_t *__restrict__ count,
                                double *__restrict__ mass,
                                double *__restrict__ cen, int *__restrict__ err) {
    const int64_t n = in.n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const bool gas = p < in.ng;
        const int64_t k = gas ? p : p - in.ng;
        const int64_t r = gas ? in.lg[k] : in.ld[k];
        if (r < 0 || r >= n) {  // not a labelling of this set
            atomicOr(err, DEV_ERR_INPUT);
            continue;
        }
        const double mp = gas ? (double)in.mg[k] : (double)in.md[k];
        atomicAdd(&count[r], 1);
        atomicAdd(&mass[r], mp);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double dd = in.pos(p, a) - in.pos(r, a);
            dd -= rint(dd);
            atomicAdd(&cen[a * n + r], mp * dd);
        }
    }
}

template <typename T>
__global__ void halo_centre_kernel(const HaloIn<T> in,
                                   const int32_t *__restrict__ count,
                                   const double *__restrict__ mass,
                                   double *__restrict__ cen) {
    const int64_t n = in.n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (count[q] == 0) continue;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double c = in.pos(q, a) + cen[a * n + q] / mass[q];
            if (c >= 2.0) c -= 1.0;
            if (c < 1.0) c += 1.0;
            cen[a * n + q] = c;
        }
    }
}

template <typename T>
int halo_impl(crk_ctx *ctx, int64_t ng, int64_t nd, const int32_t *lg,
              const int32_t *ld, const void *const g[3], const void *mg,
              const void *const d[3], const void *md, int32_t *count,
              double *mass, double *cen) {
    const int64_t n = ng + nd;
    HaloIn<T> in;
    in.ng = ng;
    in.n = n;
    in.lg = lg;
    in.ld = ld;
    for (int a = 0; a < 3; ++a) {
        in.g[a] = g ? static_cast<const T *>(g[a]) : nullptr;
        in.d[a] = d ? static_cast<const T *>(d[a]) : nullptr;
    }
    in.mg = static_cast<const T *>(mg);
    in.md = static_cast<const T *>(md);
    // (fill kernels, not memsets: the calls may be captured in a graph)
    CRK_HIP(fill_i32(count, 0, n, ctx->stream));
    CRK_HIP(fill_i64(reinterpret_cast<int64_t *>(mass), 0, n, ctx->stream));
    CRK_HIP(fill_i64(reinterpret_cast<int64_t *>(cen), 0, 3 * n, ctx->stream));
    hipLaunchKernelGGL((halo_sum_kernel<T>), dim3(grid_halo(n)), dim3(256), 0,
                       ctx->stream, in, count, mass, cen, ctx->err.as<int>());
    hipLaunchKernelGGL((halo_centre_kernel<T>), dim3(grid_halo(n)), dim3(256), 0,
                       ctx->stream, in, count, mass, cen);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

}  // namespace

int fof_properties(crk_ctx *ctx, int64_t n_gas, int64_t n_dm,
                   const int32_t *labels_gas, const int32_t *labels_dm,
                   const void *const g[3], const void *m_gas,
                   const void *const d[3], const void *m_dm, int32_t *count,
                   double *mass, double *centre) {
    if (ctx->precision == CRK_FP64)
        return halo_impl<double>(ctx, n_gas, n_dm, labels_gas, labels_dm, g,
                                 m_gas, d, m_dm, count, mass, centre);
    return halo_impl<float>(ctx, n_gas, n_dm, labels_gas, labels_dm, g, m_gas,
                            d, m_dm, count, mass, centre);
}

}  // namespace crk
