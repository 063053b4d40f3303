// crk_integrate: one kick-drift of the double-precision state, then the
// refresh of the context-precision copies read by the pair passes (the
// mixed-precision pattern of Sec. IV-A).  HBM-bound and elementwise.
#include "crk_internal.h"

namespace crk {

namespace {

template <typename T>
__global__ void integrate_kernel(int64_t n, double dt, double *__restrict__ x64,
                                 double *__restrict__ v64, double *__restrict__ u64,
                                 const T *__restrict__ g0, const T *__restrict__ g1,
                                 const T *__restrict__ g2, const T *__restrict__ h0,
                                 const T *__restrict__ h1, const T *__restrict__ h2,
                                 const T *__restrict__ dudt, T *__restrict__ x0,
                                 T *__restrict__ x1, T *__restrict__ x2,
                                 T *__restrict__ v0, T *__restrict__ v1,
                                 T *__restrict__ v2, T *__restrict__ u) {
    const T *g[3] = {g0, g1, g2};
    const T *h[3] = {h0, h1, h2};
    T *xo[3] = {x0, x1, x2};
    T *vo[3] = {v0, v1, v2};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double acc = (double)g[a][i];
            if (h0) acc += (double)h[a][i];
            double v = v64[a * n + i] + dt * acc;
            double x = x64[a * n + i] + dt * v;
            if (x >= 2.0) x -= 1.0;
            if (x < 1.0) x += 1.0;
            v64[a * n + i] = v;
            x64[a * n + i] = x;
            T xs = (T)x;
            if (xs >= T(2)) xs = T(1);  // rounding up to 2 wraps to 1
            xo[a][i] = xs;
            vo[a][i] = (T)v;
        }
        if (u64) {
            double uu = u64[i] + dt * (double)dudt[i];
            u64[i] = uu;
            u[i] = (T)uu;
        }
    }
}

template <typename T>
int integrate_impl(crk_ctx *ctx, int64_t n, double dt, double *x64, double *v64,
                   double *u64, const void *const ag[3], const void *const ah[3],
                   const void *dudt, void *const x[3], void *const v[3], void *u) {
    if (n == 0) return CRK_OK;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipEvent_t ev = nullptr;
    span_begin(ctx, P_INTEG, true, &ev);
    auto C = [](const void *p) { return static_cast<const T *>(p); };
    hipLaunchKernelGGL((integrate_kernel<T>), dim3((unsigned)g), dim3(256), 0,
                       ctx->stream, n, dt, x64, v64, u64, C(ag[0]), C(ag[1]),
                       C(ag[2]), ah ? C(ah[0]) : nullptr, ah ? C(ah[1]) : nullptr,
                       ah ? C(ah[2]) : nullptr, C(dudt), static_cast<T *>(x[0]),
                       static_cast<T *>(x[1]), static_cast<T *>(x[2]),
                       static_cast<T *>(v[0]), static_cast<T *>(v[1]),
                       static_cast<T *>(v[2]), static_cast<T *>(u));
    span_end(ctx, P_INTEG, true, ev);
    CRK_HIP(hipGetLastError());
    return CRK_OK;
}

}  // namespace

int integrate(crk_ctx *ctx, int64_t n, double dt, double *x64, double *v64,
              double *u64, const void *const a_grav[3],
              const void *const a_hydro[3], const void *dudt, void *const x[3],
              void *const v[3], void *u) {
    if (ctx->precision == CRK_FP64)
        return integrate_impl<double>(ctx, n, dt, x64, v64, u64, a_grav, a_hydro,
                                      dudt, x, v, u);
    return integrate_impl<float>(ctx, n, dt, x64, v64, u64, a_grav, a_hydro,
                                 dudt, x, v, u);
}

}  // namespace crk
