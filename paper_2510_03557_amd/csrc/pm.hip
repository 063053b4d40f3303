// Long-range gravity on a mesh, matched to the short-range split: the
// spectral particle-mesh half of the force decomposition (Sec. IV-A), for
// one periodic unit box on one GPU.  The short-range kernel subtracts the
// force between two S2 clouds of diameter r_c; this part supplies exactly
// that force, so short + long is the periodic Newtonian force up to the
// mesh error.  Cloud-in-cell deposit (double atomics), real-to-complex FFT,
// multiplication by 4 pi G S2(k)^2 / (k^2 W(k)^2) and the spectral
// gradient i k (W the CIC window of deposit and interpolation; the k = 0
// mode and the Nyquist planes of each gradient component removed), three
// complex-to-real FFTs and cloud-in-cell interpolation.  hipFFT transforms
// are unnormalised: depositing masses rather than densities makes the two
// factors N^3 cancel.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>

#include "crk_internal.h"

namespace crk {

namespace {

constexpr double PI_PM = 3.14159265358979323846;

inline unsigned grid_pm(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)std::max<int64_t>(1, g);
}

#define PM_LOOP(i, n)                                                        \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

__global__ void zero_f64_kernel(double *__restrict__ p, int64_t n) {
    PM_LOOP(i, n) p[i] = 0.0;
}

// positions the mesh can index: finite and within a million boxes (larger
// values would overflow the cell index); others deposit nothing and get a
// zero acceleration
__device__ inline bool pm_ok(double x, double y, double z) {
    return fabs(x - 1.5) < 1e6 && fabs(y - 1.5) < 1e6 && fabs(z - 1.5) < 1e6;
}

// CIC cell and weights of coordinate x on nodes j / N
__device__ inline void cic(double x, int N, int &i0, int &i1, double &f) {
    const double u = (x - 1.0) * N;
    const double fl = floor(u);
    f = u - fl;
    int i = (int)fl % N;
    if (i < 0) i += N;
    i0 = i;
    i1 = i + 1 == N ? 0 : i + 1;
}

template <typename T>
__global__ void deposit_kernel(int64_t n, int N, const T *__restrict__ x,
                               const T *__restrict__ y, const T *__restrict__ z,
                               const T *__restrict__ m, double *__restrict__ rho) {
    PM_LOOP(p, n) {
        if (!pm_ok((double)x[p], (double)y[p], (double)z[p])) continue;
        int x0, x1, y0, y1, z0, z1;
        double fx, fy, fz;
        cic((double)x[p], N, x0, x1, fx);
        cic((double)y[p], N, y0, y1, fy);
        cic((double)z[p], N, z0, z1, fz);
        const double mp = (double)m[p];
        const int64_t NN = N;
        const int ix[2] = {x0, x1}, iy[2] = {y0, y1}, iz[2] = {z0, z1};
        const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy},
                     wz[2] = {1.0 - fz, fz};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    atomicAdd(&rho[((int64_t)ix[a] * NN + iy[b]) * NN + iz[c]],
                              mp * wx[a] * wy[b] * wz[c]);
    }
}

template <typename T>
__global__ void to_real_kernel(const double *__restrict__ a, T *__restrict__ b,
                               int64_t n) {
    PM_LOOP(i, n) b[i] = (T)a[i];
}

// S2 cloud of diameter rc: 12 (2 - 2 cos x - x sin x) / x^4 at x = k rc / 2
__device__ inline double s2_form(double k, double rc) {
    const double x = 0.5 * k * rc;
    if (x <= 1e-2) {
        const double x2 = x * x;
        return 1.0 - x2 / 15.0 + x2 * x2 / 560.0;
    }
    const double x2 = x * x;
    return 12.0 * (2.0 - 2.0 * cos(x) - x * sin(x)) / (x2 * x2);
}

__device__ inline double sinc_pm(double t) { return t == 0.0 ? 1.0 : sin(t) / t; }

// o_a = i K_a G(k) in for the three components at once (G evaluated once
// per mode); layout [N][N][N/2+1]
template <typename C, typename T>
__global__ void green_kernel(int N, double rc, double G, const C *__restrict__ in,
                             C *__restrict__ o0, C *__restrict__ o1,
                             C *__restrict__ o2) {
    const int Nh = N / 2 + 1;
    const int64_t total = (int64_t)N * N * Nh;
    PM_LOOP(q, total) {
        const int iz = (int)(q % Nh);
        const int iy = (int)((q / Nh) % N);
        const int ix = (int)(q / ((int64_t)Nh * N));
        const int nx = ix <= N / 2 ? ix : ix - N;
        const int ny = iy <= N / 2 ? iy : iy - N;
        const int nz = iz;
        const double kx = 2.0 * PI_PM * nx, ky = 2.0 * PI_PM * ny,
                     kz = 2.0 * PI_PM * nz;
        const double k2 = kx * kx + ky * ky + kz * kz;
        double g = 0.0;
        if (k2 > 0.0) {
            const double h = 0.5 / N;
            const double w = sinc_pm(kx * h) * sinc_pm(ky * h) * sinc_pm(kz * h);
            const double W = w * w;
            const double s = s2_form(sqrt(k2), rc);
            g = 4.0 * PI_PM * G * s * s / (k2 * W * W);
        }
        // each component's Nyquist plane carries no gradient
        const double gx = (nx == N / 2 || nx == -N / 2) ? 0.0 : g * kx;
        const double gy = (ny == N / 2 || ny == -N / 2) ? 0.0 : g * ky;
        const double gz = (nz == N / 2) ? 0.0 : g * kz;
        const double re = (double)in[q].x, im = (double)in[q].y;
        // i g (re + i im) = -g im + i g re
        o0[q].x = (T)(-gx * im);
        o0[q].y = (T)(gx * re);
        o1[q].x = (T)(-gy * im);
        o1[q].y = (T)(gy * re);
        o2[q].x = (T)(-gz * im);
        o2[q].y = (T)(gz * re);
    }
}

template <typename T>
__global__ void interp_kernel(int64_t n, int N, const T *__restrict__ x,
                              const T *__restrict__ y, const T *__restrict__ z,
                              const T *__restrict__ field, T *__restrict__ out) {
    PM_LOOP(p, n) {
        if (!pm_ok((double)x[p], (double)y[p], (double)z[p])) {
            out[p] = T(0);
            continue;
        }
        int x0, x1, y0, y1, z0, z1;
        double fx, fy, fz;
        cic((double)x[p], N, x0, x1, fx);
        cic((double)y[p], N, y0, y1, fy);
        cic((double)z[p], N, z0, z1, fz);
        const int64_t NN = N;
        const int ix[2] = {x0, x1}, iy[2] = {y0, y1}, iz[2] = {z0, z1};
        const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy},
                     wz[2] = {1.0 - fz, fz};
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc += wx[a] * wy[b] * wz[c] *
                           (double)field[((int64_t)ix[a] * NN + iy[b]) * NN + iz[c]];
        out[p] = (T)acc;
    }
}

const char *fft_msg(hipfftResult r) {
    switch (r) {
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_EXEC_FAILED: return "execution failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    default: return "error";
    }
}

#define CRK_FFT(call)                                                        \
    do {                                                                     \
        hipfftResult r_ = (call);                                            \
        if (r_ != HIPFFT_SUCCESS)                                            \
            return set_error(CRK_EDEVICE, std::string(#call ": ") + fft_msg(r_)); \
    } while (0)

template <typename T> struct FftTypes;
template <> struct FftTypes<float> {
    using C = hipfftComplex;
    static constexpr hipfftType R2C = HIPFFT_R2C, C2R = HIPFFT_C2R;
    static hipfftResult fwd(hipfftHandle p, float *in, C *out) {
        return hipfftExecR2C(p, in, out);
    }
    static hipfftResult inv(hipfftHandle p, C *in, float *out) {
        return hipfftExecC2R(p, in, out);
    }
};
template <> struct FftTypes<double> {
    using C = hipfftDoubleComplex;
    static constexpr hipfftType R2C = HIPFFT_D2Z, C2R = HIPFFT_Z2D;
    static hipfftResult fwd(hipfftHandle p, double *in, C *out) {
        return hipfftExecD2Z(p, in, out);
    }
    static hipfftResult inv(hipfftHandle p, C *in, double *out) {
        return hipfftExecZ2D(p, in, out);
    }
};

template <typename T>
int pm_impl(crk_ctx *ctx, int N, double rc, int64_t ng, const void *gx,
            const void *gy, const void *gz, const void *gm, int64_t nd,
            const void *dx, const void *dy, const void *dz, const void *dmm,
            void *const ag[3], void *const ad[3]) {
    using F = FftTypes<T>;
    using C = typename F::C;
    hipStream_t s = ctx->stream;
    crk_pm &pm = ctx->pm;
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t nc = (int64_t)N * N * (N / 2 + 1);
    CRK_TRY(pm.rho.ensure((size_t)n3 * 8, false));
    CRK_TRY(pm.real.ensure((size_t)n3 * sizeof(T), false));
    CRK_TRY(pm.rhok.ensure((size_t)nc * sizeof(C), false));
    CRK_TRY(pm.tmpk.ensure((size_t)3 * nc * sizeof(C), false));
    if (pm.n != N || pm.elem != (int)sizeof(T)) {
        if (pm.plans) {
            alloc_generation_bump();  // the plans' work areas go with them
            (void)hipfftDestroy(pm.fwd);
            (void)hipfftDestroy(pm.inv);
            pm.plans = false;
        }
        CRK_FFT(hipfftPlan3d(&pm.fwd, N, N, N, F::R2C));
        CRK_FFT(hipfftPlan3d(&pm.inv, N, N, N, F::C2R));
        pm.plans = true;
        pm.n = N;
        pm.elem = (int)sizeof(T);
    }
    CRK_FFT(hipfftSetStream(pm.fwd, s));
    CRK_FFT(hipfftSetStream(pm.inv, s));
    auto cp = [](const void *p) { return static_cast<const T *>(p); };
    double *rho = pm.rho.as<double>();
    T *real = pm.real.as<T>();
    C *rhok = pm.rhok.as<C>();
    C *tmpk = pm.tmpk.as<C>();
    hipLaunchKernelGGL(zero_f64_kernel, dim3(grid_pm(n3)), dim3(256), 0, s, rho, n3);
    if (ng)
        hipLaunchKernelGGL((deposit_kernel<T>), dim3(grid_pm(ng)), dim3(256), 0, s,
                           ng, N, cp(gx), cp(gy), cp(gz), cp(gm), rho);
    if (nd)
        hipLaunchKernelGGL((deposit_kernel<T>), dim3(grid_pm(nd)), dim3(256), 0, s,
                           nd, N, cp(dx), cp(dy), cp(dz), cp(dmm), rho);
    hipLaunchKernelGGL((to_real_kernel<T>), dim3(grid_pm(n3)), dim3(256), 0, s,
                       rho, real, n3);
    CRK_HIP(hipGetLastError());
    CRK_FFT(F::fwd(pm.fwd, real, rhok));
    hipLaunchKernelGGL((green_kernel<C, T>), dim3(grid_pm(nc)), dim3(256), 0, s, N,
                       rc, ctx->params.G, rhok, tmpk, tmpk + nc, tmpk + 2 * nc);
    CRK_HIP(hipGetLastError());
    for (int a = 0; a < 3; ++a) {
        CRK_FFT(F::inv(pm.inv, tmpk + a * nc, real));
        if (ng)
            hipLaunchKernelGGL((interp_kernel<T>), dim3(grid_pm(ng)), dim3(256), 0,
                               s, ng, N, cp(gx), cp(gy), cp(gz), real,
                               static_cast<T *>(ag[a]));
        if (nd)
            hipLaunchKernelGGL((interp_kernel<T>), dim3(grid_pm(nd)), dim3(256), 0,
                               s, nd, N, cp(dx), cp(dy), cp(dz), real,
                               static_cast<T *>(ad[a]));
        CRK_HIP(hipGetLastError());
    }
    return CRK_OK;
}

}  // namespace

void pm_release(crk_pm &pm) {
    if (pm.plans) {
        alloc_generation_bump();
        (void)hipfftDestroy(pm.fwd);
        (void)hipfftDestroy(pm.inv);
        pm.plans = false;
    }
    pm.rho.release();
    pm.real.release();
    pm.rhok.release();
    pm.tmpk.release();
    pm.n = 0;
}

int pm_gravity(crk_ctx *ctx, int n_mesh, double r_c, int64_t n_gas,
               const void *gx, const void *gy, const void *gz, const void *m_gas,
               int64_t n_dm, const void *dx, const void *dy, const void *dz,
               const void *m_dm, void *const a_gas[3], void *const a_dm[3]) {
    if (ctx->precision == CRK_FP64)
        return pm_impl<double>(ctx, n_mesh, r_c, n_gas, gx, gy, gz, m_gas, n_dm,
                               dx, dy, dz, m_dm, a_gas, a_dm);
    return pm_impl<float>(ctx, n_mesh, r_c, n_gas, gx, gy, gz, m_gas, n_dm, dx,
                          dy, dz, m_dm, a_gas, a_dm);
}

}  // namespace crk
