// sources.hip -- the source parameterisations of the paper's source
// applications (include/seisgrad.h: source_gaussian, source_gaussian_grad,
// source_rupture, source_rupture_grad) and the plane-wave row of the
// layered-model inversion (source_plane_wave): wavelets of several source nodes from
// a few parameters, and the chain rule from dJ/dwavelet (adjoint_gradient's
// g_wavelet) back to those parameters.  Reductions over time steps and nodes
// are FP64 in a fixed order.
#include "../../include/seisgrad.h"
#include "sg_error.h"

#include <hip/hip_runtime.h>

#include <cmath>

using sg::fail;

namespace {

constexpr int ST = 256;

// Weight of node j of a Gaussian footprint: dx dz exp(-r^2/(2 sigma^2)) / (2 pi sigma^2).
__device__ __forceinline__ double gauss_w(const int *cells, int j, double x0, double z0, double sigma, double dx)
{
    const double xj = cells[2 * j] * dx, zj = cells[2 * j + 1] * dx;
    const double r2 = (xj - x0) * (xj - x0) + (zj - z0) * (zj - z0);
    return dx * dx * exp(-r2 / (2.0 * sigma * sigma)) / (2.0 * M_PI * sigma * sigma);
}

__global__ void gauss_wav_kernel(int nsrc, int nt, const int *cells, double x0, double z0, double sigma, double dx,
                                 const float *g, float *wav)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nsrc * nt) return;
    const int j = (int)(i / nt), k = (int)(i - (long long)j * nt);
    wav[i] = (float)(gauss_w(cells, j, x0, z0, sigma, dx) * g[k]);
}

__device__ double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = ST / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One workgroup: dg[k] = sum_j gw[j][k] w_j (k strided over threads) and
// (dx0, dz0) = sum_j (sum_k gw[j][k] g[k]) dw_j/d(x0, z0), dw_j/dx0 = w_j (x_j - x0)/sigma^2.
__global__ __launch_bounds__(ST) void gauss_grad_kernel(int nsrc, int nt, const int *cells, double x0, double z0,
                                                        double sigma, double dx, const float *g, const float *gw,
                                                        float *dg, double *dxz)
{
    __shared__ double red[ST];
    for (int k = threadIdx.x; k < nt; k += ST) {
        double v = 0.0;
        for (int j = 0; j < nsrc; ++j) v += (double)gw[(long long)j * nt + k] * gauss_w(cells, j, x0, z0, sigma, dx);
        dg[k] = (float)v;
    }
    double ax = 0.0, az = 0.0;
    for (int j = 0; j < nsrc; ++j) {
        double c = 0.0;
        for (int k = threadIdx.x; k < nt; k += ST) c += (double)gw[(long long)j * nt + k] * g[k];
        c = block_sum(c, red);
        const double w = gauss_w(cells, j, x0, z0, sigma, dx);
        ax += c * w * (cells[2 * j] * dx - x0) / (sigma * sigma);
        az += c * w * (cells[2 * j + 1] * dx - z0) / (sigma * sigma);
    }
    if (threadIdx.x == 0) {
        dxz[0] = ax;
        dxz[1] = az;
    }
}

__global__ void rupture_wav_kernel(int npt, int nt, const float *A0, const float *t0, double sigma_t, double dt,
                                   float *wav)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)npt * nt) return;
    const int j = (int)(i / nt), k = (int)(i - (long long)j * nt);
    const double d = k * dt - (double)t0[j];
    wav[i] = (float)((double)A0[j] * exp(-d * d / (2.0 * sigma_t * sigma_t)));
}

// One workgroup per point j: dA0_j = sum_k gw e, dt0_j = sum_k gw A0 e (t_k - t0)/sigma_t^2.
__global__ __launch_bounds__(ST) void rupture_grad_kernel(int nt, const float *A0, const float *t0, double sigma_t,
                                                          double dt, const float *gw, double *dA0, double *dt0)
{
    __shared__ double red[ST];
    const int j = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nt; k += ST) {
        const double d = k * dt - (double)t0[j];
        const double e = exp(-d * d / (2.0 * sigma_t * sigma_t));
        const double v = (double)gw[(long long)j * nt + k];
        a += v * e;
        b += v * (double)A0[j] * e * d / (sigma_t * sigma_t);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        dA0[j] = a;
        dt0[j] = b;
    }
}

#define LAUNCH_CHECK(what)                                                               \
    do {                                                                                 \
        const hipError_t e_ = hipGetLastError();                                         \
        if (e_ != hipSuccess) return fail(SG_EDEVICE, what ": %s", hipGetErrorString(e_)); \
    } while (0)

// Row of nodes x_j = x_first + j spacing firing the Ricker wavelet with
// delays tau_j = (x_j - x_ref) sin(theta) / c, x_ref the first node to fire.
__global__ void plane_wave_kernel(int n, int nt, double x_first, double spacing, double s_over_c, double f0,
                                  double t0, double dt, float *wav)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * nt) return;
    const int j = (int)(i / nt), k = (int)(i - (long long)j * nt);
    const double x_ref = s_over_c >= 0.0 ? x_first : x_first + (n - 1) * spacing;
    const double tau = (x_first + j * spacing - x_ref) * s_over_c;
    double a = M_PI * f0 * (k * dt - t0 - tau);
    a *= a;
    wav[i] = (float)((1.0 - 2.0 * a) * exp(-a));
}

} // namespace

extern "C" {

int source_plane_wave(int32_t n, int32_t nt, double x_first, double spacing, double theta_deg, double c, double f0,
                      double t0, double dt, float *wav, sg_stream_t stream)
{
    if (n < 1 || nt < 1 || !(c > 0) || !(f0 > 0) || !(dt > 0) || !(std::fabs(theta_deg) < 90.0))
        return fail(SG_EINVAL, "bad plane-wave arguments");
    if (!wav) return fail(SG_EINVAL, "NULL pointer argument");
    const long long m = (long long)n * nt;
    plane_wave_kernel<<<(unsigned)((m + ST - 1) / ST), ST, 0, (hipStream_t)stream>>>(
        n, nt, x_first, spacing, std::sin(theta_deg * M_PI / 180.0) / c, f0, t0, dt, wav);
    LAUNCH_CHECK("source_plane_wave");
    return SG_OK;
}

int source_gaussian(int32_t nsrc, int32_t nt, const int32_t *cells, double x0, double z0, double sigma, double dx,
                    const float *g, float *wav, sg_stream_t stream)
{
    if (nsrc < 1 || nt < 1 || !(sigma > 0) || !(dx > 0)) return fail(SG_EINVAL, "bad Gaussian source arguments");
    if (!cells || !g || !wav) return fail(SG_EINVAL, "NULL pointer argument");
    const long long n = (long long)nsrc * nt;
    gauss_wav_kernel<<<(unsigned)((n + ST - 1) / ST), ST, 0, (hipStream_t)stream>>>(nsrc, nt, cells, x0, z0, sigma,
                                                                                    dx, g, wav);
    LAUNCH_CHECK("source_gaussian");
    return SG_OK;
}

int source_gaussian_grad(int32_t nsrc, int32_t nt, const int32_t *cells, double x0, double z0, double sigma,
                         double dx, const float *g, const float *gw, float *dg, double *dxz, sg_stream_t stream)
{
    if (nsrc < 1 || nt < 1 || !(sigma > 0) || !(dx > 0)) return fail(SG_EINVAL, "bad Gaussian source arguments");
    if (!cells || !g || !gw || !dg || !dxz) return fail(SG_EINVAL, "NULL pointer argument");
    gauss_grad_kernel<<<1, ST, 0, (hipStream_t)stream>>>(nsrc, nt, cells, x0, z0, sigma, dx, g, gw, dg, dxz);
    LAUNCH_CHECK("source_gaussian_grad");
    return SG_OK;
}

int source_rupture(int32_t npt, int32_t nt, const float *A0, const float *t0, double sigma_t, double dt, float *wav,
                   sg_stream_t stream)
{
    if (npt < 1 || nt < 1 || !(sigma_t > 0) || !(dt > 0)) return fail(SG_EINVAL, "bad rupture arguments");
    if (!A0 || !t0 || !wav) return fail(SG_EINVAL, "NULL pointer argument");
    const long long n = (long long)npt * nt;
    rupture_wav_kernel<<<(unsigned)((n + ST - 1) / ST), ST, 0, (hipStream_t)stream>>>(npt, nt, A0, t0, sigma_t, dt,
                                                                                      wav);
    LAUNCH_CHECK("source_rupture");
    return SG_OK;
}

int source_rupture_grad(int32_t npt, int32_t nt, const float *A0, const float *t0, double sigma_t, double dt,
                        const float *gw, double *dA0, double *dt0, sg_stream_t stream)
{
    if (npt < 1 || nt < 1 || !(sigma_t > 0) || !(dt > 0)) return fail(SG_EINVAL, "bad rupture arguments");
    if (!A0 || !t0 || !gw || !dA0 || !dt0) return fail(SG_EINVAL, "NULL pointer argument");
    rupture_grad_kernel<<<npt, ST, 0, (hipStream_t)stream>>>(nt, A0, t0, sigma_t, dt, gw, dA0, dt0);
    LAUNCH_CHECK("source_rupture_grad");
    return SG_OK;
}

} // extern "C"
