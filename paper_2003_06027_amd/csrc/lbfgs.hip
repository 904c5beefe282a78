// lbfgs.hip -- limited-memory BFGS helpers of the outer inversion loop
// (include/seisgrad.h: lbfgs_push, lbfgs_direction).
//
// The paper's inversions use L-BFGS-B (Applications, FWI); here the bounds
// are kept by clipping the model after each step and the direction is the
// two-loop recursion (Nocedal & Wright, Algorithm 7.4).  Models of a batch
// keep separate histories; one workgroup of 1024 threads serves one model,
// every inner product is an FP64 block reduction in a fixed order, so the
// direction is bitwise reproducible.
#include "../../include/seisgrad.h"
#include "sg_error.h"

#include <hip/hip_runtime.h>

using sg::fail;

namespace {

constexpr int LB_THREADS = 1024;
constexpr int LB_MAXMEM = 64;

// Sum of one double per thread in a fixed tree order; every thread gets it.
__device__ double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = LB_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(LB_THREADS) void lbfgs_push_kernel(int nmodels, long long n, int mem,
                                                                const int *slot, const float *m_new,
                                                                const float *m_old, const float *g_new,
                                                                const float *g_old, float *S, float *Y,
                                                                double *ysyy)
{
    __shared__ double red[LB_THREADS];
    const int b = blockIdx.x;
    const int k = slot[b];
    if (k < 0 || k >= mem) return;                 // this model keeps its history unchanged
    const long long o = (long long)b * n;
    float *s = S + ((long long)k * nmodels + b) * n, *y = Y + ((long long)k * nmodels + b) * n;
    double ys = 0.0, yy = 0.0;
    for (long long i = threadIdx.x; i < n; i += LB_THREADS) {
        const float si = m_new[o + i] - m_old[o + i], yi = g_new[o + i] - g_old[o + i];
        s[i] = si;
        y[i] = yi;
        ys += (double)yi * si;
        yy += (double)yi * yi;
    }
    ys = block_sum(ys, red);
    yy = block_sum(yy, red);
    if (threadIdx.x == 0) {
        ysyy[2 * ((long long)k * nmodels + b)] = ys;
        ysyy[2 * ((long long)k * nmodels + b) + 1] = yy;
    }
}

// p = -H g for model b over hist[2b] pairs ending at ring slot hist[2b+1];
// p holds q, then r, in place.
__global__ __launch_bounds__(LB_THREADS) void lbfgs_direction_kernel(int nmodels, long long n, int mem,
                                                                     const int *hist, const float *S,
                                                                     const float *Y, const double *ysyy,
                                                                     const float *g, float *p)
{
    __shared__ double red[LB_THREADS];
    __shared__ double alpha[LB_MAXMEM];
    const int b = blockIdx.x;
    const int newest = hist[2 * b + 1];
    const int count = (newest < 0 || newest >= mem) ? 0 : max(0, min(hist[2 * b], mem));
    const long long o = (long long)b * n;
    float *q = p + o;
    for (long long i = threadIdx.x; i < n; i += LB_THREADS) q[i] = g[o + i];
    __syncthreads();
    auto slot_of = [&](int j) { return (newest - j + mem) % mem; };   // j = 0: newest
    for (int j = 0; j < count; ++j) {
        const int k = slot_of(j);
        const float *s = S + ((long long)k * nmodels + b) * n, *y = Y + ((long long)k * nmodels + b) * n;
        double sq = 0.0;
        for (long long i = threadIdx.x; i < n; i += LB_THREADS) sq += (double)s[i] * q[i];
        sq = block_sum(sq, red);
        const double a = sq / ysyy[2 * ((long long)k * nmodels + b)];
        if (threadIdx.x == 0) alpha[j] = a;
        const float af = (float)a;
        for (long long i = threadIdx.x; i < n; i += LB_THREADS) q[i] -= af * y[i];
        __syncthreads();
    }
    float gamma = 1.f;
    if (count > 0) {
        const long long k = slot_of(0);
        gamma = (float)(ysyy[2 * (k * nmodels + b)] / ysyy[2 * (k * nmodels + b) + 1]);
    }
    for (long long i = threadIdx.x; i < n; i += LB_THREADS) q[i] *= gamma;
    __syncthreads();
    for (int j = count - 1; j >= 0; --j) {
        const int k = slot_of(j);
        const float *s = S + ((long long)k * nmodels + b) * n, *y = Y + ((long long)k * nmodels + b) * n;
        double yr = 0.0;
        for (long long i = threadIdx.x; i < n; i += LB_THREADS) yr += (double)y[i] * q[i];
        yr = block_sum(yr, red);
        const double beta = yr / ysyy[2 * ((long long)k * nmodels + b)];
        const float c = (float)(alpha[j] - beta);
        for (long long i = threadIdx.x; i < n; i += LB_THREADS) q[i] += c * s[i];
        __syncthreads();
    }
    for (long long i = threadIdx.x; i < n; i += LB_THREADS) q[i] = -q[i];
}

} // namespace

extern "C" {

int lbfgs_push(int32_t nmodels, int64_t n, int32_t mem, const int32_t *slot, const float *m_new,
               const float *m_old, const float *g_new, const float *g_old, float *S, float *Y, double *ysyy,
               sg_stream_t stream)
{
    if (nmodels < 1 || n < 1 || mem < 1 || mem > LB_MAXMEM)
        return fail(SG_EINVAL, "need nmodels, n >= 1 and 1 <= mem <= %d", LB_MAXMEM);
    if (!slot || !m_new || !m_old || !g_new || !g_old || !S || !Y || !ysyy)
        return fail(SG_EINVAL, "NULL pointer argument");
    lbfgs_push_kernel<<<nmodels, LB_THREADS, 0, (hipStream_t)stream>>>(nmodels, n, mem, slot, m_new, m_old, g_new,
                                                                       g_old, S, Y, ysyy);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SG_EDEVICE, "lbfgs_push launch: %s", hipGetErrorString(e));
    return SG_OK;
}

int lbfgs_direction(int32_t nmodels, int64_t n, int32_t mem, const int32_t *hist, const float *S, const float *Y,
                    const double *ysyy, const float *g, float *p, sg_stream_t stream)
{
    if (nmodels < 1 || n < 1 || mem < 1 || mem > LB_MAXMEM)
        return fail(SG_EINVAL, "need nmodels, n >= 1 and 1 <= mem <= %d", LB_MAXMEM);
    if (!hist || !S || !Y || !ysyy || !g || !p) return fail(SG_EINVAL, "NULL pointer argument");
    if (p == g) return fail(SG_EINVAL, "p must not alias g");
    lbfgs_direction_kernel<<<nmodels, LB_THREADS, 0, (hipStream_t)stream>>>(nmodels, n, mem, hist, S, Y, ysyy, g, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SG_EDEVICE, "lbfgs_direction launch: %s", hipGetErrorString(e));
    return SG_OK;
}

} // extern "C"
