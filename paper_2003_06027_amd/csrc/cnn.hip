// cnn.hip -- kernels and C ABI of the learned gradient preconditioner
// (include/sg_cnn.h).
//
// The 32 -> 32 channel 3x3 layers are implicit GEMMs on the matrix cores:
// v_mfma_f32_16x16x32_bf16 with one 3x3 tap (32 input channels) per
// K-block.  A workgroup of four wavefronts computes a 4 x 64 output tile,
// one row per wavefront; the 6 x 66 input tile (one-pixel zero halo) goes
// straight from global memory into LDS (direct 16-byte loads) in swizzled
// slots, which makes the 16-byte fragment reads of 16 consecutive pixels
// bank-conflict free.  The weight gradient uses the pixels as the K
// dimension and reduces per workgroup, then over workgroups in a fixed
// order.  The thin layers c1 (1 -> 32) and c6 (32 -> 1) are per-pixel FP32
// kernels: as GEMMs they would have K = 9 or N = 1, which matrix cores
// cannot fill.  Every reduction has a fixed order, so results are bitwise
// reproducible from call to call.
#include "../../include/seisgrad.h"
#include "../../include/sg_cnn.h"
#include "sg_error.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

using sg::fail;

namespace {

using u16 = unsigned short;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int CH = CNN_CHANNELS;
constexpr int TH = 4, TW = 64;           // output tile: 4 rows x 64 columns
constexpr int LH = TH + 2, LW = TW + 2;  // input tile with a one-pixel halo
constexpr int NT = 256;                  // threads per workgroup (4 wavefronts)
constexpr int WMID = CH * 9 * CH;        // weights of one 32 -> 32 layer
constexpr int PMID = WMID + CH;          // ... with its biases
constexpr int OFF_C1 = 0, OFF_C2 = 9 * CH + CH, OFF_C6 = OFF_C2 + 4 * PMID;
constexpr int MAX_WG_WGRAD = 512;        // workgroups (partials) of the MFMA weight gradient
constexpr int MAX_WG_THIN = 1024;        // ... of the thin-layer weight gradients
constexpr int THIN_STRIDE = 320;         // partial row of a thin layer (289 or 320 used)
constexpr int MAX_WG_LOSS = 1024;
static_assert(OFF_C6 + 9 * CH + 1 == CNN_NPARAMS, "parameter layout");

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ u16 f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)                 // inf stays inf, NaN stays NaN
        return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest, ties to even
    return (u16)(u >> 16);
}

__device__ __forceinline__ unsigned pack2(float a, float b)
{
    return (unsigned)f2bf(a) | ((unsigned)f2bf(b) << 16);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// The 6 x 66 halo tile (pixels y0-1 .. y0+4, x0-1 .. x0+64 of image n) straight
// from global memory into LDS, 16 bytes (8 channels) per lane and load: item
// i = (pixel i / 4, slot i % 4) fills 16-byte slot i, which holds chunk
// (i % 4) ^ sw(pixel) of the pixel.  The swizzle sw(p) = (p / 4) % 4 puts the
// same chunk of 16 consecutive pixels on 16 distinct 16-byte bank groups.
// Pixels outside the image get zeros from a plain LDS store of their slots.
// The caller waits for the loads and synchronises.
__device__ __forceinline__ int halo_slot(int pix, int q) { return pix * 4 + (q ^ ((pix >> 2) & 3)); }

__device__ __forceinline__ void dma_halo_swizzled(const u16 *__restrict__ x, int n, int H, int W, int y0, int x0,
                                                  unsigned char *lds)
{
    constexpr int NV = LH * LW * 4, K = (NV + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * NT;
        if (i >= NV) continue;
        const int pix = i >> 2, q = (i & 3) ^ ((pix >> 2) & 3);
        const int rr = pix / LW, c = pix - rr * LW;
        const int y = y0 - 1 + rr, xx = x0 - 1 + c;
        if (y >= 0 && y < H && xx >= 0 && xx < W)
            __builtin_amdgcn_global_load_lds((const void *)(x + (((long long)n * H + y) * W + xx) * CH + q * 8),
                                             (void __attribute__((address_space(3))) *)(lds + (k * NT + (threadIdx.x & ~63)) * 16),
                                             16, 0, 0);
        else
            *(u32x4 *)(lds + i * 16) = u32x4{0u, 0u, 0u, 0u};
    }
}

// ------------------------------------------------------------ 32 -> 32 layer
struct ConvArgs {
    const u16 *x, *w;
    const float *bias;
    const u16 *res, *gate;
    u16 *y;
    float *y32;
    int N, H, W, relu;
};

// grid (ceil(W/64), ceil(H/4), N).  Lane l of a wavefront: r = l % 16 is the
// fragment row (a pixel for A, an output channel for B), g = l / 16 selects
// the 8 channels 8g .. 8g+7 of the K-block; the accumulator holds output
// pixels 4g .. 4g+3 of each 16-pixel block for output channel r.  The
// accumulators go through LDS ([pixel][channel], FP32) so that the epilogue
// reads and writes 8 channels of a pixel per lane in 16- and 32-byte
// accesses instead of single 2- and 4-byte elements.
constexpr int OS = CH + 4;                 // FP32 stride of an output pixel in LDS
constexpr int CONV_LDS = LH * LW * 64 > 4 * TW * OS * 4 ? LH * LW * 64 : 4 * TW * OS * 4;
__global__ __launch_bounds__(NT) void conv3x3_mfma_kernel(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[CONV_LDS];
    u16 *lds = reinterpret_cast<u16 *>(lds_raw);
    const int n = blockIdx.z, y0 = blockIdx.y * TH, x0 = blockIdx.x * TW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;

    bf16x8 bw[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            bw[t][nb] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(a.w + ((16 * nb + r) * 9 + t) * CH + 8 * g));

    dma_halo_swizzled(a.x, n, a.H, a.W, y0, x0, lds_raw);
    __builtin_amdgcn_s_waitcnt(0);         // this thread's direct loads have landed in LDS
    __syncthreads();

    f32x4 acc[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
        acc[mb][0] = acc[mb][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ky = t / 3, kx = t - 3 * (t / 3);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const u16 *p = lds + halo_slot((wv + ky) * LW + 16 * mb + r + kx, g) * 8;
            const bf16x8 av = __builtin_bit_cast(bf16x8, *(const u32x4 *)p);
            acc[mb][0] = mfma(av, bw[t][0], acc[mb][0]);
            acc[mb][1] = mfma(av, bw[t][1], acc[mb][1]);
        }
    }

    __syncthreads();                       // every wavefront is done with the input tile
    float *orow = reinterpret_cast<float *>(lds_raw) + wv * TW * OS;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) orow[(16 * mb + 4 * g + j) * OS + 16 * nb + r] = acc[mb][nb][j];
    __syncthreads();

    const int y = y0 + wv;
    if (y >= a.H) return;
    const long long rowbase = ((long long)n * a.H + y) * a.W;
#pragma unroll
    for (int it = 0; it < TW * 4 / 64; ++it) {
        const int item = lane + 64 * it, px = item >> 2, q = item & 3;   // 8 channels 8q .. 8q+7 of pixel px
        if (x0 + px >= a.W) continue;
        const long long idx = (rowbase + x0 + px) * CH + 8 * q;
        const f32x4 lo = *reinterpret_cast<const f32x4 *>(orow + px * OS + 8 * q);
        const f32x4 hi = *reinterpret_cast<const f32x4 *>(orow + px * OS + 8 * q + 4);
        const float acc8[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        u16x8 rv = {0, 0, 0, 0, 0, 0, 0, 0}, gv = {0, 0, 0, 0, 0, 0, 0, 0};
        if (a.res) rv = *reinterpret_cast<const u16x8 *>(a.res + idx);
        if (a.gate) gv = *reinterpret_cast<const u16x8 *>(a.gate + idx);
        float v8[8];
        u16x8 o;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float b = a.bias ? a.bias[8 * q + k] : 0.f;
            float v = acc8[k] + b;
            if (a.res) v += bf2f(rv[k]);
            if (a.relu) v = fmaxf(v, 0.f);
            if (a.gate && !(bf2f(gv[k]) > 0.f)) v = 0.f;
            v8[k] = v;
            o[k] = f2bf(v);
        }
        *reinterpret_cast<u16x8 *>(a.y + idx) = o;
        if (a.y32) {
            *reinterpret_cast<f32x4 *>(a.y32 + idx) = f32x4{v8[0], v8[1], v8[2], v8[3]};
            *reinterpret_cast<f32x4 *>(a.y32 + idx + 4) = f32x4{v8[4], v8[5], v8[6], v8[7]};
        }
    }
}

// Stage an image tile of ROWS x COLS pixels starting at (y0 - HALO, x0 - HALO)
// straight from global memory into LDS: 16 bytes (8 channels) per lane and
// load into consecutive 16-byte slots, slot i = chunk i % 4 of tile pixel
// i / 4 (a 64-byte pixel stride); pixels outside the image get zeros from
// plain LDS stores.  The caller waits for the loads and synchronises.
template <int ROWS, int COLS, int HALO>
__device__ __forceinline__ void dma_tile(const u16 *__restrict__ x, int n, int H, int W, int y0, int x0,
                                         unsigned char *lds)
{
    constexpr int NV = ROWS * COLS * 4, K = (NV + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = threadIdx.x + k * NT;
        if (i >= NV) continue;
        const int pix = i >> 2, q = i & 3;
        const int rr = pix / COLS, c = pix - rr * COLS;
        const int y = y0 - HALO + rr, xx = x0 - HALO + c;
        if (y >= 0 && y < H && xx >= 0 && xx < W)
            __builtin_amdgcn_global_load_lds((const void *)(x + (((long long)n * H + y) * W + xx) * CH + q * 8),
                                             (void __attribute__((address_space(3))) *)(lds + (k * NT + (threadIdx.x & ~63)) * 16),
                                             16, 0, 0);
        else
            *(u32x4 *)(lds + i * 16) = u32x4{0u, 0u, 0u, 0u};
    }
}

// Weight gradient, K = pixels.  Each wavefront owns one tile row (two
// K-blocks of 32 pixels); K index 8g + e of a lane maps to pixel 4e + g of
// the block, the same for both operands, so that the eight 2-byte LDS reads
// of a fragment hit distinct banks across the lane groups.
struct WgradArgs {
    const u16 *dy, *x;
    float *part;  // [gridDim.x][PMID]
    int N, H, W, tx, ty, ntiles;
};

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void wgrad3x3_mfma_kernel(WgradArgs a)
{
    constexpr int PW = 32;                 // u16 stride of a staged pixel (the slots of dma_tile)
    __shared__ __attribute__((aligned(16))) u16 smem[LH * LW * PW + TH * TW * PW];
    static_assert((LH * LW * PW + TH * TW * PW) * 2 >= PMID * 4, "the reduction reuses the staging space");
    u16 *lx = smem, *lg = smem + LH * LW * PW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const bf16x8 ones = __builtin_bit_cast(bf16x8, u16x8{0x3f80, 0x3f80, 0x3f80, 0x3f80,
                                                         0x3f80, 0x3f80, 0x3f80, 0x3f80});
    f32x4 acc[9][2][2];
    f32x4 accb[2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        acc[t][0][0] = acc[t][0][1] = acc[t][1][0] = acc[t][1][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    accb[0] = accb[1] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const int per = a.tx * a.ty;
        const int n = tile / per, rem = tile - n * per;
        const int y0 = (rem / a.tx) * TH, x0 = (rem - (rem / a.tx) * a.tx) * TW;
        __syncthreads();
        dma_tile<LH, LW, 1>(a.x, n, a.H, a.W, y0, x0, reinterpret_cast<unsigned char *>(lx));
        dma_tile<TH, TW, 0>(a.dy, n, a.H, a.W, y0, x0, reinterpret_cast<unsigned char *>(lg));
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            u16x8 ga0, ga1;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const u16 *p = lg + (wv * TW + kb * 32 + 4 * e + g) * PW + r;
                ga0[e] = p[0];
                ga1[e] = p[16];
            }
            const bf16x8 A0 = __builtin_bit_cast(bf16x8, ga0), A1 = __builtin_bit_cast(bf16x8, ga1);
            accb[0] = mfma(A0, ones, accb[0]);
            accb[1] = mfma(A1, ones, accb[1]);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int ky = t / 3, kx = t - 3 * (t / 3);
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    u16x8 xb;
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        xb[e] = lx[((wv + ky) * LW + kb * 32 + 4 * e + g + kx) * PW + 16 * ib + r];
                    const bf16x8 B = __builtin_bit_cast(bf16x8, xb);
                    acc[t][0][ib] = mfma(A0, B, acc[t][0][ib]);
                    acc[t][1][ib] = mfma(A1, B, acc[t][1][ib]);
                }
            }
        }
    }

    // fixed-order sum over the four wavefronts in LDS, then one partial row
    float *red = reinterpret_cast<float *>(smem);
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wv == w) {
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int co = 16 * cb + 4 * g + j, ci = 16 * ib + r;
                            const int idx = (co * 9 + t) * CH + ci;
                            red[idx] = (w == 0 ? 0.f : red[idx]) + acc[t][cb][ib][j];
                        }
            if (r == 0)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int idx = WMID + 16 * cb + 4 * g + j;
                        red[idx] = (w == 0 ? 0.f : red[idx]) + accb[cb][j];
                    }
        }
    }
    __syncthreads();
    float *out = a.part + (long long)blockIdx.x * PMID;
    for (int i = threadIdx.x; i < PMID; i += NT) out[i] = red[i];
}

// out[i] = sum over b of part[b][i] in FP64, in a fixed order: lane l of
// output i sums rows b = l, l + 16, ... in ascending order, then the 16 lane
// sums are added in lane order.  256 threads = 16 outputs x 16 lanes.  A lane
// issues the loads of 16 of its rows before adding them, so that a chain of
// nb / 16 rows costs nb / 256 memory latencies.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float *__restrict__ part, int nb, int stride,
                                                              int count, float *__restrict__ out)
{
    constexpr int U = 16;
    __shared__ double red[16][17];
    const int o = threadIdx.x & 15, l = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + o;
    double s = 0.0;
    if (i < count) {
        int b = l;
        for (; b + 16 * (U - 1) < nb; b += 16 * U) {
            float v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) v[k] = part[(long long)(b + 16 * k) * stride + i];
#pragma unroll
            for (int k = 0; k < U; ++k) s += (double)v[k];
        }
        for (; b < nb; b += 16) s += (double)part[(long long)b * stride + i];
    }
    red[l][o] = s;
    __syncthreads();
    if (l == 0 && i < count) {
        double t = red[0][o];
        for (int k = 1; k < 16; ++k) t += red[k][o];
        out[i] = (float)t;
    }
}

// BF16 copies of c2..c5: wf[L] as stored ([co][tap][ci]) and wt[L] flipped
// and transposed ([ci][8 - tap][co]), the weights of the input gradient.
__global__ void prep_weights_kernel(const float *__restrict__ params, u16 *__restrict__ wf, u16 *__restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * WMID) return;
    const int L = i / WMID, k = i - L * WMID;
    const int co = k / (9 * CH), t = (k / CH) % 9, ci = k % CH;
    const u16 b = f2bf(params[OFF_C2 + L * PMID + k]);
    wf[i] = b;
    wt[L * WMID + (ci * 9 + (8 - t)) * CH + co] = b;
}

// ------------------------------------------------------------- thin layers
__device__ __forceinline__ void pixel_of(long long p, int H, int W, int &n, int &y, int &x)
{
    x = (int)(p % W);
    const long long q = p / W;
    y = (int)(q % H);
    n = (int)(q / H);
}

// c1: x1 = relu(b + sum_t w[co][t] g[pix + off_t]) in FP32, stored BF16.
// The thin layers c1 and c6's input gradient work on runs of NT consecutive
// pixels (flat n, y, x order), whose 32 channels are NT x 64 contiguous
// bytes: a thread computes one pixel (the weights are then the same for every
// lane), and the 64-byte pixels pass through LDS in the swizzled slots of
// halo_slot, so that global memory sees whole 1 KiB runs per instruction.
__device__ __forceinline__ void store_pixels(const unsigned char *lds, long long p0, long long total, u16 *dst)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = threadIdx.x + k * NT, pix = j >> 2, q = j & 3;
        if (p0 + pix < total)
            *(u32x4 *)(dst + (p0 + pix) * CH + q * 8) = *(const u32x4 *)(lds + halo_slot(pix, q) * 16);
    }
}

__global__ __launch_bounds__(NT) void conv_in_kernel(const float *__restrict__ g, const float *__restrict__ params,
                                                     u16 *__restrict__ x1, int N, int H, int W)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[NT * 64];
    const long long total = (long long)N * H * W, p0 = (long long)blockIdx.x * NT, p = p0 + threadIdx.x;
    if (p < total) {
        int n, y, x;
        pixel_of(p, H, W, n, y, x);
        float v[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            v[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? g[((long long)n * H + yy) * W + xx] : 0.f;
        }
        const float *w = params + OFF_C1, *b = params + OFF_C1 + 9 * CH;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float o[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int co = 8 * q + e;
                float s = b[co];
#pragma unroll
                for (int t = 0; t < 9; ++t) s = fmaf(w[co * 9 + t], v[t], s);
                o[e] = fmaxf(s, 0.f);
            }
            *(u32x4 *)(lds + halo_slot(threadIdx.x, q) * 16) =
                u32x4{pack2(o[0], o[1]), pack2(o[2], o[3]), pack2(o[4], o[5]), pack2(o[6], o[7])};
        }
    }
    __syncthreads();
    store_pixels(lds, p0, total, x1);
}

// c6 and the global residual: p = -g + b + sum_t sum_ci w[t][ci] x3[pix + off_t][ci].
// On the 4 x 64 tiles of the 32 -> 32 layers, x3 with its halo staged in LDS
// as for those layers; one thread per pixel, the sum in tap, channel order.
__global__ __launch_bounds__(NT) void conv_out_kernel(const u16 *__restrict__ x3, const float *__restrict__ g,
                                                      const float *__restrict__ params, float *__restrict__ p,
                                                      int N, int H, int W)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[LH * LW * 64];
    const int n = blockIdx.z, y0 = blockIdx.y * TH, x0 = blockIdx.x * TW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    dma_halo_swizzled(x3, n, H, W, y0, x0, lds);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int y = y0 + wv, x = x0 + lane;
    if (y >= H || x >= W) return;
    const float *w = params + OFF_C6;
    float s = params[OFF_C6 + 9 * CH];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
        const int pix = (wv + t / 3) * LW + lane + t % 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const u32x4 u = *(const u32x4 *)(lds + halo_slot(pix, q) * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s = fmaf(w[t * CH + 8 * q + 2 * e], __uint_as_float(u[e] << 16), s);
                s = fmaf(w[t * CH + 8 * q + 2 * e + 1], __uint_as_float(u[e] & 0xffff0000u), s);
            }
        }
    }
    const long long i = ((long long)n * H + y) * W + x;
    p[i] = s - g[i];
}

// Input gradient of c6 gated by x3 > 0: G[pix][ci] = [x3 > 0] sum_t w[t][ci] dp[pix - off_t].
__global__ __launch_bounds__(NT) void dgrad_out_kernel(const float *__restrict__ dp, const u16 *__restrict__ x3,
                                                       const float *__restrict__ params, u16 *__restrict__ G,
                                                       int N, int H, int W)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[NT * 64];
    const long long total = (long long)N * H * W, p0 = (long long)blockIdx.x * NT, p = p0 + threadIdx.x;
    // the gates x3 of the run, straight into the swizzled slots (16 bytes per lane and load)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = threadIdx.x + k * NT, pix = j >> 2, q = (j & 3) ^ ((pix >> 2) & 3);
        if (p0 + pix < total)
            __builtin_amdgcn_global_load_lds((const void *)(x3 + (p0 + pix) * CH + q * 8),
                                             (void __attribute__((address_space(3))) *)(lds + (k * NT + (threadIdx.x & ~63)) * 16),
                                             16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (p < total) {
        int n, y, x;
        pixel_of(p, H, W, n, y, x);
        float d[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
            d[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? dp[((long long)n * H + yy) * W + xx] : 0.f;
        }
        const float *w = params + OFF_C6;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u32x4 *slot = (u32x4 *)(lds + halo_slot(threadIdx.x, q) * 16);
            const u32x4 gt = *slot;
            float o[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int ci = 8 * q + e;
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < 9; ++t) s = fmaf(w[t * CH + ci], d[t], s);
                const unsigned gv = (e & 1) ? (gt[e >> 1] & 0xffff0000u) : (gt[e >> 1] << 16);
                o[e] = __uint_as_float(gv) > 0.f ? s : 0.f;
            }
            *slot = u32x4{pack2(o[0], o[1]), pack2(o[2], o[3]), pack2(o[4], o[5]), pack2(o[6], o[7])};
        }
    }
    __syncthreads();
    store_pixels(lds, p0, total, G);
}

// Weight gradients of the thin layers, on the 4 x 64 pixel tiles of the
// 32 -> 32 layers (grid-stride over tiles, per-thread register sums, one
// partial row per workgroup; the rows are reduced in a fixed order after).
// c6: out[t * 32 + ci] = sum_p dp[p] x3[p + off_t][ci] (t < 9), out[288] = sum dp.
// c1: out[co * 9 + t] = sum_p G[p][co] g[p + off_t], out[288 + co] = sum_p G[p][co].
template <bool OUT>
__global__ __launch_bounds__(NT) void wgrad_thin_kernel(const float *__restrict__ img, const u16 *__restrict__ act,
                                                        float *__restrict__ part, int H, int W, int tx, int ty,
                                                        int ntiles)
{
    constexpr int PW = 32;                 // u16 stride of a staged pixel (the slots of dma_tile)
    __shared__ __attribute__((aligned(16))) u16 la[(OUT ? LH * LW : TH * TW) * PW];
    __shared__ float li[OUT ? TH * TW : LH * LW];
    constexpr int NOUT = OUT ? 9 * CH + 1 : 9 * CH + CH;
    float acc0 = 0.f, acc1 = 0.f;
    const int o0 = threadIdx.x, o1 = threadIdx.x + NT;   // o1 valid when < NOUT
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int per = tx * ty;
        const int n = tile / per, rem = tile - n * per;
        const int y0 = (rem / tx) * TH, x0 = (rem - (rem / tx) * tx) * TW;
        __syncthreads();
        if (OUT) {
            dma_tile<LH, LW, 1>(act, n, H, W, y0, x0, reinterpret_cast<unsigned char *>(la));
            for (int i = threadIdx.x; i < TH * TW; i += NT) {
                const int y = y0 + i / TW, x = x0 + i % TW;
                li[i] = (y < H && x < W) ? img[((long long)n * H + y) * W + x] : 0.f;
            }
        } else {
            dma_tile<TH, TW, 0>(act, n, H, W, y0, x0, reinterpret_cast<unsigned char *>(la));
            for (int i = threadIdx.x; i < LH * LW; i += NT) {
                const int y = y0 - 1 + i / LW, x = x0 - 1 + i % LW;
                li[i] = (y >= 0 && y < H && x >= 0 && x < W) ? img[((long long)n * H + y) * W + x] : 0.f;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);     // this thread's direct loads have landed in LDS
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int o = q ? o1 : o0;
            if (o >= NOUT) continue;
            float s = 0.f;
            if (OUT) {
                if (o < 9 * CH) {
                    const int t = o / CH, ci = o % CH, ky = t / 3, kx = t % 3;
                    for (int r = 0; r < TH; ++r)
                        for (int c = 0; c < TW; ++c)
                            s = fmaf(li[r * TW + c], bf2f(la[((r + ky) * LW + c + kx) * PW + ci]), s);
                } else {
                    for (int i = 0; i < TH * TW; ++i) s += li[i];
                }
            } else {
                if (o < 9 * CH) {
                    const int co = o / 9, t = o % 9, ky = t / 3, kx = t % 3;
                    for (int r = 0; r < TH; ++r)
                        for (int c = 0; c < TW; ++c)
                            s = fmaf(bf2f(la[(r * TW + c) * PW + co]), li[(r + ky) * LW + c + kx], s);
                } else {
                    const int co = o - 9 * CH;
                    for (int i = 0; i < TH * TW; ++i) s += bf2f(la[i * PW + co]);
                }
            }
            if (q) acc1 += s; else acc0 += s;
        }
    }
    float *out = part + (long long)blockIdx.x * THIN_STRIDE;
    if (o0 < NOUT) out[o0] = acc0;
    if (o1 < NOUT) out[o1] = acc1;
}

// --------------------------------------------------------- loss and Adam
__device__ void block_sum2(double &a, double &b)
{
    __shared__ double sa[256], sb[256];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
}

__global__ __launch_bounds__(256) void loss_partial_kernel(const float *__restrict__ p, const float *__restrict__ t,
                                                           const float *__restrict__ m, long long n, long long per_wg,
                                                           double *__restrict__ part)
{
    const long long i0 = blockIdx.x * per_wg, i1 = i0 + per_wg < n ? i0 + per_wg : n;
    double s = 0.0, c = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += 256) {
        const double r = (double)p[i] - (double)t[i];
        s += (double)m[i] * r * r;
        c += (double)m[i];
    }
    block_sum2(s, c);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = c;
    }
}

__global__ __launch_bounds__(256) void loss_final_kernel(const double *__restrict__ part, int nb, double *L,
                                                         double *count)
{
    double s = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        s += part[2 * b];
        c += part[2 * b + 1];
    }
    block_sum2(s, c);
    if (threadIdx.x == 0) {
        *L = c > 0 ? s / c : 0.0;
        *count = c;
    }
}

__global__ void loss_grad_kernel(const float *__restrict__ p, const float *__restrict__ t, const float *__restrict__ m,
                                 long long n, const double *__restrict__ count, float *__restrict__ dp)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = *count;
    dp[i] = c > 0 ? (float)(2.0 * (double)m[i] * ((double)p[i] - (double)t[i]) / c) : 0.f;
}

__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ----------------------------------------------------------------- packing
__global__ __launch_bounds__(256) void field_inv_rms_kernel(const float *__restrict__ a, const float *__restrict__ b,
                                                            int nsrc, const int *__restrict__ order, int fh, int fw,
                                                            double *__restrict__ inv)
{
    const int s = blockIdx.x;
    const int f = order ? order[s] : s;
    const bool valid = f >= 0 && f < nsrc;
    const long long n = (long long)fh * fw, base = (long long)f * n;
    double acc = 0.0, dummy = 0.0;
    for (long long i = threadIdx.x; valid && i < n; i += 256) {
        const float v = b ? a[base + i] - b[base + i] : a[base + i];
        acc += (double)v * (double)v;
    }
    block_sum2(acc, dummy);
    if (threadIdx.x == 0) inv[s] = acc > 0 ? 1.0 / sqrt(acc / (double)n) : 0.0;
}

__global__ void pack_kernel(const float *__restrict__ a, const float *__restrict__ b, int nsrc,
                            const int *__restrict__ order, int nfields, int fh, int fw, int frame, const double *__restrict__ inv,
                            float *__restrict__ patches, float *__restrict__ mask, long long total)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int P = 2 * frame;
    const int xx = (int)(i % P), yy = (int)((i / P) % P);
    const long long q = i / ((long long)P * P);
    const long long s = q * 4 + (yy / frame) * 2 + xx / frame;
    const int ly = yy % frame, lx = xx % frame;
    const long long f = s < nfields ? (order ? order[s] : s) : -1;
    const bool inside = f >= 0 && f < nsrc && ly < fh && lx < fw;
    float v = 0.f;
    if (inside) {
        const long long k = (f * fh + ly) * fw + lx;
        v = b ? a[k] - b[k] : a[k];
        if (inv) v *= (float)inv[s];
    }
    patches[i] = v;
    if (mask) mask[i] = inside ? 1.f : 0.f;
}

__global__ void unpack_kernel(const float *__restrict__ patches, int nfields, int fh, int fw, int frame,
                              float *__restrict__ fields)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nfields * fh * fw) return;
    const int lx = (int)(i % fw), ly = (int)((i / fw) % fh);
    const long long s = i / ((long long)fh * fw);
    const int P = 2 * frame;
    const int k = (int)(s % 4);
    const long long src = ((s / 4) * P + (k / 2) * frame + ly) * P + (k % 2) * frame + lx;
    fields[i] = patches[src];
}

// --------------------------------------------------------------- host side
#define HIPCHECK(x)                                                                  \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            return fail(SG_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));     \
    } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct CnnLayout {
    size_t wf, wt, act[5], gbuf[3], part, loss, total;
};

CnnLayout cnn_layout(int n, int h, int w)
{
    CnnLayout L;
    const size_t A = up((size_t)n * h * w * CH * sizeof(u16));
    size_t o = 0;
    L.wf = o; o += up(4 * WMID * sizeof(u16));
    L.wt = o; o += up(4 * WMID * sizeof(u16));
    for (auto &x : L.act) { x = o; o += A; }
    for (auto &x : L.gbuf) { x = o; o += A; }
    L.part = o;
    const size_t pm = (size_t)MAX_WG_WGRAD * PMID, pt = (size_t)MAX_WG_THIN * THIN_STRIDE;
    o += up((pm > pt ? pm : pt) * sizeof(float));
    L.loss = o; o += up((2 * MAX_WG_LOSS + 2) * sizeof(double));
    L.total = o;
    return L;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int check_dims(int n, int h, int w)
{
    if (n < 1 || h < 1 || w < 1) return fail(SG_EINVAL, "image extents must be positive (n=%d h=%d w=%d)", n, h, w);
    if ((long long)n * h * w >= (1LL << 29)) return fail(SG_EINVAL, "images too large (n h w >= 2^29 pixels)");
    return SG_OK;
}

int launch_conv(const u16 *x, int n, int h, int w, const u16 *wgt, const float *bias, const u16 *res,
                const u16 *gate, int relu, u16 *y, float *y32, hipStream_t s)
{
    ConvArgs a{x, wgt, bias, res, gate, y, y32, n, h, w, relu};
    dim3 grid((w + TW - 1) / TW, (h + TH - 1) / TH, n);
    if (grid.y > 65535u || grid.z > 65535u) return fail(SG_EINVAL, "image batch too large for one launch");
    conv3x3_mfma_kernel<<<grid, NT, 0, s>>>(a);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int launch_wgrad(const u16 *dy, const u16 *x, int n, int h, int w, float *part, float *out, hipStream_t s)
{
    WgradArgs a;
    a.dy = dy;
    a.x = x;
    a.part = part;
    a.N = n;
    a.H = h;
    a.W = w;
    a.tx = (w + TW - 1) / TW;
    a.ty = (h + TH - 1) / TH;
    const long long nt = (long long)a.tx * a.ty * n;
    if (nt > (1LL << 31) - 1) return fail(SG_EINVAL, "too many tiles");
    a.ntiles = (int)nt;
    const int nwg = a.ntiles < MAX_WG_WGRAD ? a.ntiles : MAX_WG_WGRAD;
    wgrad3x3_mfma_kernel<<<nwg, NT, 0, s>>>(a);
    HIPCHECK(hipGetLastError());
    reduce_partials_kernel<<<(PMID + 15) / 16, 256, 0, s>>>(part, nwg, PMID, PMID, out);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

template <bool OUT>
int launch_wgrad_thin(const float *img, const u16 *act, int n, int h, int w, float *part, float *out, hipStream_t s)
{
    const int tx = (w + TW - 1) / TW, ty = (h + TH - 1) / TH;
    const long long nt = (long long)tx * ty * n;
    if (nt > (1LL << 31) - 1) return fail(SG_EINVAL, "too many tiles");
    const int nwg = nt < MAX_WG_THIN ? (int)nt : MAX_WG_THIN;
    wgrad_thin_kernel<OUT><<<nwg, NT, 0, s>>>(img, act, part, h, w, tx, ty, (int)nt);
    HIPCHECK(hipGetLastError());
    const int count = OUT ? 9 * CH + 1 : 9 * CH + CH;
    reduce_partials_kernel<<<(count + 15) / 16, 256, 0, s>>>(part, nwg, THIN_STRIDE, count, out);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

} // namespace

extern "C" {

size_t cnn_workspace_bytes(int32_t n, int32_t h, int32_t w)
{
    if (n < 1 || h < 1 || w < 1) return 0;
    return cnn_layout(n, h, w).total;
}

int cnn_forward(const float *params, const float *g, int32_t n, int32_t h, int32_t w, float *p, void *ws,
                size_t ws_bytes, sg_stream_t stream)
{
    if (int e = check_dims(n, h, w)) return e;
    if (!params || !g || !p || !ws) return fail(SG_EINVAL, "NULL pointer argument");
    const CnnLayout L = cnn_layout(n, h, w);
    if (ws_bytes < L.total || !aligned16(ws))
        return fail(SG_EINVAL, "workspace too small or misaligned (%zu < %zu bytes)", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    u16 *wf = (u16 *)(base + L.wf), *wt = (u16 *)(base + L.wt);
    u16 *x1 = (u16 *)(base + L.act[0]), *a2 = (u16 *)(base + L.act[1]), *x2 = (u16 *)(base + L.act[2]);
    u16 *a4 = (u16 *)(base + L.act[3]), *x3 = (u16 *)(base + L.act[4]);
    const long long pix = (long long)n * h * w;
    prep_weights_kernel<<<blocks(4 * WMID), 256, 0, s>>>(params, wf, wt);
    HIPCHECK(hipGetLastError());
    conv_in_kernel<<<blocks(pix, NT), NT, 0, s>>>(g, params, x1, n, h, w);
    HIPCHECK(hipGetLastError());
    const float *bias = params + OFF_C2 + WMID;
    if (int e = launch_conv(x1, n, h, w, wf + 0 * WMID, bias + 0 * PMID, nullptr, nullptr, 1, a2, nullptr, s)) return e;
    if (int e = launch_conv(a2, n, h, w, wf + 1 * WMID, bias + 1 * PMID, x1, nullptr, 1, x2, nullptr, s)) return e;
    if (int e = launch_conv(x2, n, h, w, wf + 2 * WMID, bias + 2 * PMID, nullptr, nullptr, 1, a4, nullptr, s)) return e;
    if (int e = launch_conv(a4, n, h, w, wf + 3 * WMID, bias + 3 * PMID, x2, nullptr, 1, x3, nullptr, s)) return e;
    conv_out_kernel<<<dim3((w + TW - 1) / TW, (h + TH - 1) / TH, n), NT, 0, s>>>(x3, g, params, p, n, h, w);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int cnn_backward(const float *params, const float *g, const float *dp, int32_t n, int32_t h, int32_t w, float *grad,
                 void *ws, size_t ws_bytes, sg_stream_t stream)
{
    if (int e = check_dims(n, h, w)) return e;
    if (!params || !g || !dp || !grad || !ws) return fail(SG_EINVAL, "NULL pointer argument");
    const CnnLayout L = cnn_layout(n, h, w);
    if (ws_bytes < L.total || !aligned16(ws))
        return fail(SG_EINVAL, "workspace too small or misaligned (%zu < %zu bytes)", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    const u16 *wt = (const u16 *)(base + L.wt);
    const u16 *x1 = (u16 *)(base + L.act[0]), *a2 = (u16 *)(base + L.act[1]), *x2 = (u16 *)(base + L.act[2]);
    const u16 *a4 = (u16 *)(base + L.act[3]), *x3 = (u16 *)(base + L.act[4]);
    u16 *G0 = (u16 *)(base + L.gbuf[0]), *G1 = (u16 *)(base + L.gbuf[1]), *G2 = (u16 *)(base + L.gbuf[2]);
    float *part = (float *)(base + L.part);
    const long long pix = (long long)n * h * w;

    if (int e = launch_wgrad_thin<true>(dp, x3, n, h, w, part, grad + OFF_C6, s)) return e;
    dgrad_out_kernel<<<blocks(pix, NT), NT, 0, s>>>(dp, x3, params, G0, n, h, w);           // G0 = d pre(x3)
    HIPCHECK(hipGetLastError());
    float *gm = grad + OFF_C2;
    if (int e = launch_wgrad(G0, a4, n, h, w, part, gm + 3 * PMID, s)) return e;
    if (int e = launch_conv(G0, n, h, w, wt + 3 * WMID, nullptr, nullptr, a4, 0, G1, nullptr, s)) return e; // d pre(a4)
    if (int e = launch_wgrad(G1, x2, n, h, w, part, gm + 2 * PMID, s)) return e;
    if (int e = launch_conv(G1, n, h, w, wt + 2 * WMID, nullptr, G0, x2, 0, G2, nullptr, s)) return e;     // d pre(x2)
    if (int e = launch_wgrad(G2, a2, n, h, w, part, gm + 1 * PMID, s)) return e;
    if (int e = launch_conv(G2, n, h, w, wt + 1 * WMID, nullptr, nullptr, a2, 0, G0, nullptr, s)) return e; // d pre(a2)
    if (int e = launch_wgrad(G0, x1, n, h, w, part, gm + 0 * PMID, s)) return e;
    if (int e = launch_conv(G0, n, h, w, wt + 0 * WMID, nullptr, G2, x1, 0, G1, nullptr, s)) return e;     // d pre(x1)
    if (int e = launch_wgrad_thin<false>(g, G1, n, h, w, part, grad + OFF_C1, s)) return e;
    return SG_OK;
}

int cnn_loss(const float *p, const float *t, const float *mask, int64_t count, double *L_dev, float *dp, void *ws,
             size_t ws_bytes, sg_stream_t stream)
{
    if (!p || !t || !mask || !L_dev || !ws) return fail(SG_EINVAL, "NULL pointer argument");
    if (count < 1) return fail(SG_EINVAL, "count must be positive");
    const CnnLayout L = cnn_layout(1, 1, 1);
    if (ws_bytes < L.total) return fail(SG_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, L.total);
    // the reduction area sits at the end of every layout; use the last bytes
    double *part = (double *)((char *)ws + ws_bytes / ALIGN * ALIGN - up((2 * MAX_WG_LOSS + 2) * sizeof(double)));
    hipStream_t s = (hipStream_t)stream;
    long long nwg = (count + 4095) / 4096;
    if (nwg > MAX_WG_LOSS) nwg = MAX_WG_LOSS;
    const long long per = (count + nwg - 1) / nwg;
    nwg = (count + per - 1) / per;
    loss_partial_kernel<<<(unsigned)nwg, 256, 0, s>>>(p, t, mask, count, per, part);
    HIPCHECK(hipGetLastError());
    double *cnt = part + 2 * MAX_WG_LOSS;
    loss_final_kernel<<<1, 256, 0, s>>>(part, (int)nwg, L_dev, cnt);
    HIPCHECK(hipGetLastError());
    if (dp) {
        loss_grad_kernel<<<blocks(count), 256, 0, s>>>(p, t, mask, count, cnt, dp);
        HIPCHECK(hipGetLastError());
    }
    return SG_OK;
}

int cnn_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
             float eps, int32_t step, sg_stream_t stream)
{
    if (!params || !grad || !m || !v) return fail(SG_EINVAL, "NULL pointer argument");
    if (n < 1 || step < 1) return fail(SG_EINVAL, "n and step must be positive");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return fail(SG_EINVAL, "Adam needs 0 <= beta < 1 and eps > 0");
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    adam_kernel<<<blocks(n), 256, 0, (hipStream_t)stream>>>(params, grad, m, v, n, lr, beta1, beta2, eps, c1, c2);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int cnn_pack(const float *a, const float *b, int32_t nsrc, const int32_t *order, int32_t nfields, int32_t fh,
             int32_t fw, int32_t frame, int32_t normalise, double *inv_rms, float *patches, float *mask,
             sg_stream_t stream)
{
    if (!a || !patches) return fail(SG_EINVAL, "NULL pointer argument");
    if (nfields < 1 || nsrc < 1 || fh < 1 || fw < 1 || frame < fh || frame < fw)
        return fail(SG_EINVAL, "need nfields, nsrc, fh, fw >= 1 and fh, fw <= frame");
    if (normalise && !inv_rms) return fail(SG_EINVAL, "normalise needs inv_rms");
    hipStream_t s = (hipStream_t)stream;
    if (normalise) {
        field_inv_rms_kernel<<<nfields, 256, 0, s>>>(a, b, nsrc, order, fh, fw, inv_rms);
        HIPCHECK(hipGetLastError());
    }
    const long long total = (long long)((nfields + 3) / 4) * 4 * frame * frame;
    pack_kernel<<<blocks(total), 256, 0, s>>>(a, b, nsrc, order, nfields, fh, fw, frame, normalise ? inv_rms : nullptr,
                                               patches, mask, total);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int cnn_unpack(const float *patches, int32_t nfields, int32_t fh, int32_t fw, int32_t frame, float *fields,
               sg_stream_t stream)
{
    if (!patches || !fields) return fail(SG_EINVAL, "NULL pointer argument");
    if (nfields < 1 || fh < 1 || fw < 1 || frame < fh || frame < fw)
        return fail(SG_EINVAL, "need nfields, fh, fw >= 1 and fh, fw <= frame");
    unpack_kernel<<<blocks((long long)nfields * fh * fw), 256, 0, (hipStream_t)stream>>>(patches, nfields, fh, fw,
                                                                                         frame, fields);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int cnn_conv3x3(const uint16_t *x, int32_t n, int32_t h, int32_t w, const uint16_t *wgt, const float *bias,
                const uint16_t *res, const uint16_t *gate, int32_t relu, uint16_t *y, float *y32, sg_stream_t stream)
{
    if (int e = check_dims(n, h, w)) return e;
    if (!x || !wgt || !y) return fail(SG_EINVAL, "NULL pointer argument");
    if (!aligned16(x) || !aligned16(wgt) || !aligned16(res) || !aligned16(gate) || !aligned16(y) || !aligned16(y32))
        return fail(SG_EINVAL, "x, wgt, res, gate, y and y32 must be 16-byte aligned");
    return launch_conv(x, n, h, w, wgt, bias, res, gate, relu, y, y32, (hipStream_t)stream);
}

int cnn_conv3x3_wgrad(const uint16_t *dy, const uint16_t *x, int32_t n, int32_t h, int32_t w, float *dw, void *ws,
                      size_t ws_bytes, sg_stream_t stream)
{
    if (int e = check_dims(n, h, w)) return e;
    if (!dy || !x || !dw || !ws) return fail(SG_EINVAL, "NULL pointer argument");
    if (!aligned16(dy) || !aligned16(x)) return fail(SG_EINVAL, "dy and x must be 16-byte aligned");
    const CnnLayout L = cnn_layout(1, 1, 1);
    if (ws_bytes < L.total) return fail(SG_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, L.total);
    return launch_wgrad(dy, x, n, h, w, (float *)((char *)ws + L.part), dw, (hipStream_t)stream);
}

} // extern "C"
