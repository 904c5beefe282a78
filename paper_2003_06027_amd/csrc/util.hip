// util.hip -- small kernels: fill, Ricker wavelet, FP64 misfit and dot
// reductions (fixed reduction order, so results are bitwise reproducible).
#include "sg_internal.h"

#include <mutex>

namespace sg {

__global__ void fill_kernel(float *p, long long n, float v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill(float *p, long long n, float v, hipStream_t s)
{
    if (n <= 0) return;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
    fill_kernel<<<blocks, 256, 0, s>>>(p, n, v);
}

// Ricker wavelet r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2, in FP64.
__global__ void ricker_kernel(double f0, double t0, double dt, int nt, float *out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    double a = M_PI * f0 * (k * dt - t0);
    a *= a;
    out[k] = (float)((1.0 - 2.0 * a) * exp(-a));
}

void launch_ricker(double f0, double t0, double dt, int nt, float *out, hipStream_t s)
{
    ricker_kernel<<<(nt + 255) / 256, 256, 0, s>>>(f0, t0, dt, nt, out);
}

// Block-wide FP64 sum in a fixed tree order (wavefront shuffles, then LDS).
__device__ double block_sum(double v)
{
    __shared__ double part[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) part[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) r += part[i];
    }
    return r; // valid in thread 0
}

// Pass 1: block b handles [b*chunk, min(n, (b+1)*chunk)); resid = pred - obs,
// partial[b] = sum 1/2 resid^2 (FP64).
__global__ __launch_bounds__(256) void misfit_kernel(const float *pred, const float *obs, long long n,
                                                     long long chunk, float *resid, double *partial)
{
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = min(n, lo + chunk);
    double acc = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const float r = pred[i] - obs[i];
        if (resid) resid[i] = r;
        acc += 0.5 * (double)r * (double)r;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The final sum; a non-finite result also raises *flag (when given), which
// the host reads at its next synchronising status query.
__global__ __launch_bounds__(256) void sum_partials_kernel(const double *partial, int np, double *out, int *flag)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) {
        *out = s;
        if (flag && !isfinite(s)) *flag = 1;
    }
}

void launch_misfit(const float *pred, const float *obs, long long n, float *resid,
                   double *partials, int nparts, double *J, int *flag, hipStream_t s)
{
    if (nparts <= 1 || partials == nullptr) {
        misfit_kernel<<<1, 256, 0, s>>>(pred, obs, n, n > 0 ? n : 1, resid, J);
        return;
    }
    long long chunk = (n + nparts - 1) / nparts;
    if (chunk < 1) chunk = 1;
    const int nb = (int)((n + chunk - 1) / chunk);
    if (nb <= 0) {
        misfit_kernel<<<1, 256, 0, s>>>(pred, obs, 0, 1, resid, J);
        return;
    }
    misfit_kernel<<<nb, 256, 0, s>>>(pred, obs, n, chunk, resid, partials);
    sum_partials_kernel<<<1, 256, 0, s>>>(partials, nb, J, flag);
}

__global__ __launch_bounds__(1024) void dot_kernel(const float *x, const float *y, long long n, double *out)
{
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) acc += (double)x[i] * (double)y[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) *out = s;
}

void launch_dot(const float *x, const float *y, long long n, double *out, hipStream_t s)
{
    dot_kernel<<<1, 1024, 0, s>>>(x, y, n, out);
}

// Partial sums of the allocation-free misfit: a static device array, one per
// device, held until the process ends.  Host code never passes `scratch`
// itself (on the host it names a stand-in, not the device address): the
// address is taken once per device with hipGetSymbolAddress and kept.
static __device__ __align__(256) double scratch[NOALLOC_PARTS];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[256] = {};
} // namespace

int noalloc_scratch(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) return -1;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

} // namespace sg
