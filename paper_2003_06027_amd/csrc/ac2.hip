// ac2.hip -- gfx950 kernels of the 2-D acoustic recursion and its adjoint.
//
// Forward step k (paper: U_{k+1} = A(theta) U_k + F_k, Eq. (1); PDE Eq. (12)
// in the constant-density form u_tt = c^2 lap(u) + f with an auxiliary-field
// absorbing layer).  In scaled variables (chat = dt^2 c^2/dx^2, phi~ = dx*phi,
// h = zeta dt/2, L~ and D~ the 8th-order stencils without the 1/dx factors):
//   pass A (layer cells only):
//     phi~_j^k = p_j phi~_j^{k-1} + q_j D~_j u^k,   p_j = (1-h_j)/(1+h_j),
//                                                  q_j = 2(h_other - h_j)/(1+h_j)
//   pass B (every cell):
//     w~^k    = L~ u^k + D~_x phi~_x^k + D~_z phi~_z^k
//     u^{k+1} = alpha (beta u^k - gamma u^{k-1} + chat w~^k + dt^2 f^k)
// with alpha = 1/(1+h_x+h_z), beta = 2 - 4 h_x h_z, gamma = 1 - h_x - h_z
// (1, 2, 1 in the interior).  The stored state after step k is
// (u^{k+1}, u^k, phi~^k); outside the layer phi~ stays exactly zero.
// Tiles more than 4 cells from the layer ("interior" tiles) skip the phi
// terms and the damping coefficients.  The others ("near" tiles) run pass A
// themselves on the tile + 4, from u^k on the tile + 8 in LDS, then pass B
// from LDS: phi~^k of a cell is then computed by its own tile and by the
// neighbours whose ring covers it (the same expression, the same value),
// and written by its own tile only, into the other buffer of a pair
// (phi~^{k-1} and phi~^k live in different buffers, so a neighbour that
// still reads phi~^{k-1} of the cell is not disturbed).
//
// Adjoint step k (Eq. (4): lambda_k = A^T lambda_{k+1} + residual; Eq. (5)
// for the gradient), in the alpha-scaled variable s = alpha * dJ/du and the
// q-scaled layer adjoint c_j = q_j * dJ/dphi~_j (q is constant in time, so
// c obeys the same recursion as dJ/dphi~ multiplied by q):
//   pass A (layer cells):
//     c_j^{k+1} = p_j c_j^{k+2} - q_j D~_j(chat s^{k+2})
//   pass B (every cell):
//     a^{k+1} = R^T dJ/dd^{k+1} - D~_x c_x^{k+1} - D~_z c_z^{k+1}
//               + beta s^{k+2} + L~(chat s^{k+2}) - gamma s^{k+3}
//     s^{k+1} = alpha a^{k+1};   dJ/dchat += s^{k+1} w~^k
// using L~^T = L~ and D~^T = -D~ (zero cells beyond the grid).  Near tiles
// fold pass A in as in the forward step (chat s^{k+2} on the tile + 8 in
// LDS; c^{k+2} and c^{k+1} in the two buffers of a pair).
//
// Cache policy: an operand that only its own cell reads or writes in a step
// (u^{k-1} and s^{k+3} in the one-step kernels, the new wavefields, the
// snapshots, the gradient accumulators) is loaded and stored non-temporally,
// so that it does not displace what neighbouring tiles share (u^k, chat s,
// chat, the layer auxiliaries).  A load that the ring of a neighbouring tile
// repeats (u^{k-1}, s^{k+3} in the blocked kernels) stays cached: streaming
// it made the blocked adjoint 2 % slower.
#include "sg_internal.h"

namespace sg {

// 8th-order centred weights: second derivative (a_1..a_4; the centre weight
// -205/72 = -2 sum a_m is folded into the difference form below) and first
// derivative.
constexpr float A1 = (float)(8.0 / 5.0);
constexpr float A2 = (float)(-1.0 / 5.0);
constexpr float A3 = (float)(8.0 / 315.0);
constexpr float A4 = (float)(-1.0 / 560.0);
constexpr float D1 = (float)(4.0 / 5.0);
constexpr float D2 = (float)(-1.0 / 5.0);
constexpr float D3 = (float)(4.0 / 105.0);
constexpr float D4 = (float)(-1.0 / 280.0);

__device__ __forceinline__ long long fidx(const Grid2 &g, int iz, int ix)
{
    return (long long)(iz + OZ) * g.SX + (ix + OX);
}

// 8th-order Laplacian (x + z) of an LDS tile with row stride W.  The weights
// sum to zero, so L~u = sum_m a_m ((u_{+m} - u_0) + (u_{-m} - u_0)) along each
// axis: neighbour differences of a smooth field are exact or nearly so in
// FP32, which keeps the rounding error proportional to L~u instead of u.
// The multiply-adds are explicit so that every kernel evaluating the
// stencil rounds identically (the one- and two-step paths agree bitwise).
__device__ __forceinline__ float lap8(const float *c, int W)
{
    const float c0 = c[0];
    auto pair = [&](int o) { return (c[o] - c0) + (c[-o] - c0); };
    float t = A4 * (pair(4) + pair(4 * W));
    t = fmaf(A3, pair(3) + pair(3 * W), t);
    t = fmaf(A2, pair(2) + pair(2 * W), t);
    return fmaf(A1, pair(1) + pair(W), t);
}

template <class T>
__device__ __forceinline__ float d8(const T *c, long long s)
{
    return D1 * (c[s] - c[-s]) + D2 * (c[2 * s] - c[-2 * s])
         + D3 * (c[3 * s] - c[-3 * s]) + D4 * (c[4 * s] - c[-4 * s]);
}

// Work id of this workgroup with consecutive ids on one XCD: the hardware
// hands workgroups to the 8 XCDs round-robin, so id b runs on XCD b % 8; the
// remap gives each XCD a contiguous range of (tile, shot) work, which keeps
// neighbouring tiles -- and their shared halos -- in the same L2.
__device__ __forceinline__ int xcd_work_id(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, j = b / NXCD;
    return x * per + min(x, rem) + j;
}

// Is a tile within 4 cells of the absorbing layer (its cells need the phi
// terms or damping coefficients)?
__device__ __forceinline__ bool near_layer(const Grid2 &g, int x0, int z0)
{
    return g.P > 0 && (x0 - 4 < g.P || x0 + TX + 4 > g.P + g.nx ||
                       z0 - 4 < g.P || z0 + TZ + 4 > g.P + g.nz);
}

// Fill the (TZ+8) x (TX+8) LDS tile: own cells by the caller, the 4-cell
// halo here (value f(frame index)).
template <class Fn>
__device__ __forceinline__ void load_halo(const Grid2 &g, float *lds, int x0, int z0, Fn f)
{
    constexpr int H = 4, W = TX + 2 * H;
    constexpr int NH = 2 * H * W + 2 * TZ * H;
    for (int i = threadIdx.x; i < NH; i += NTH) {
        int r, c;
        if (i < 2 * H * W) {
            const int s = i / W;
            c = i - s * W;
            r = s < H ? s : s + TZ;
        } else {
            const int j = i - 2 * H * W;
            const int rr = j / (2 * H), cc = j - rr * (2 * H);
            r = H + rr;
            c = cc < H ? cc : cc + TX;
        }
        lds[r * W + c] = f(fidx(g, z0 - H + r, x0 - H + c));
    }
}

// The source term dt^2 f^k of one node: a separately rounded product, so
// that no kernel fuses it into the addition that injects it (whether the
// compiler would fuse depends on the kernel's shape; every kernel injecting
// a source must round identically for the one- and two-step paths to agree).
__device__ __forceinline__ float src_value(float scale, float w)
{
    return __fmul_rn(scale, w);
}

// A layer cell of the padded grid.
__device__ __forceinline__ bool layer_cell_at(const Grid2 &g, int iz, int ix)
{
    return iz < g.P || iz >= g.P + g.nz || ix < g.P || ix >= g.P + g.nx;
}

// Sum of dt^2/(dx dz) r_j(t_k) over the source nodes j of this shot at
// local tile cell `cell` (several source nodes per shot; a handful of
// entries per tile, only in the tiles that hold them).
__device__ __forceinline__ float node_sources(const Ac2FwdArgs &a, int tile, int shot, int cell)
{
    const int ntiles = a.g.ntx * a.g.ntz;
    const int *off = a.src_off + (long long)shot * (ntiles + 1);
    float v = 0.f;
    for (int e = off[tile]; e < off[tile + 1]; ++e) {
        const int ent = a.src_ent[e];
        if (src_cell(ent) == cell)
            v += a.src_scale * a.wav[((long long)shot * a.nsrc + src_node(ent)) * a.nt + a.k];
    }
    return v;
}

__global__ void ac2_src_gather_kernel(int nshots, int nsrc, long long plane, const long long *node_f,
                                      const float *s1, float *gw, int nt, int k, float scale)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nshots * nsrc) return;
    const int shot = i / nsrc;
    gw[(long long)i * nt + k] = scale * s1[(long long)shot * plane + node_f[i]];
}

void launch_ac2_src_gather(int nshots, int nsrc, long long plane, const long long *node_f, const float *s1,
                           float *gw, int nt, int k, float scale, hipStream_t s)
{
    const int n = nshots * nsrc;
    ac2_src_gather_kernel<<<(n + 255) / 256, 256, 0, s>>>(nshots, nsrc, plane, node_f, s1, gw, nt, k, scale);
}

// ------------------------------------------------------------ forward pass B
// A tile away from the layer (the interior update), u^k with a 4-cell halo in LDS.
template <bool SNAP, bool REC>
__device__ __forceinline__ void fwd_tile(const Ac2FwdArgs &a, float *su, int tile, int shot)
{
    constexpr int H = 4, W = TX + 2 * H;
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *u = a.u + so;
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int ix = x0 + lx;

    float uc[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j;
        uc[j] = u[fidx(g, z0 + r, ix)];
        su[(r + H) * W + lx + H] = uc[j];
    }
    load_halo(g, su, x0, z0, [&](long long f) { return u[f]; });
    __syncthreads();

    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const float *um = a.um + so;
    float *uo = a.un + so;
    const long long src = a.src_f[shot];
    const float sval = src_value(a.src_scale, a.wav[(long long)shot * a.nt + a.k]);
    float un[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        const long long f = fidx(g, iz, ix);
        float w = lap8(su + (r + H) * W + lx + H, W);
        un[j] = 0.f;
        if (iz < g.NZ && ix < g.NX) {
            // 2u - um + chat w = u + ((u - um) + chat w)
            float inc = fmaf(chat[f], w, uc[j] - __builtin_nontemporal_load(um + f));
            if (f == src) inc += sval;
            if (a.nsrc > 1) inc += node_sources(a, tile, shot, r * TX + lx);
            const float v = uc[j] + inc;
            __builtin_nontemporal_store(v, uo + f);
            un[j] = v;
            if constexpr (SNAP) __builtin_nontemporal_store(w, a.snap + so + f);
        }
    }

    if constexpr (REC) {
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int b = off[tile], e = off[tile + 1];
        if (b < e) {                      // uniform over the block
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RPT; ++j) su[(ly * RPT + j + H) * W + lx + H] = un[j];
            __syncthreads();
            for (int i = b + tid; i < e; i += NTH) {
                const int ent = a.rec_ent[i];
                const int cell = rec_cell(ent);
                const int r = cell / TX, c = cell - r * TX;
                a.seis[((long long)shot * a.nt + a.k) * a.nrec + rec_id(ent)] = su[(r + H) * W + c + H];
            }
        }
    }
}

// One forward step on a list of tiles away from the layer.
template <bool SNAP, bool REC>
__global__ __launch_bounds__(NTH) void ac2_fwd_kernel(Ac2FwdArgs a)
{
    __shared__ float su[(TZ + 8) * (TX + 8)];
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl;
    fwd_tile<SNAP, REC>(a, su, a.tiles[w - shot * a.ntl], shot);
}

// ------------------------------------------------------------ adjoint pass B
// A tile away from the layer, chat s^{k+2} with a 4-cell halo in LDS.
__device__ __forceinline__ void adj_tile(const Ac2AdjArgs &a, float *sc, int tile, int shot)
{
    constexpr int H = 4, W = TX + 2 * H;
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *s2 = a.s2 + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int ix = x0 + lx;

    float sc2[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j;
        const long long f = fidx(g, z0 + r, ix);
        sc2[j] = s2[f];
        sc[(r + H) * W + lx + H] = chat[f] * sc2[j];
    }
    load_halo(g, sc, x0, z0, [&](long long f) { return chat[f] * s2[f]; });
    __syncthreads();

    const float *s3 = a.s3 + so;
    float *s1o = a.s1 + so;
    float av[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        float v = lap8(sc + (r + H) * W + lx + H, W);
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fidx(g, iz, ix);
            v += sc2[j] + (sc2[j] - __builtin_nontemporal_load(s3 + f));
        }
        av[j] = v;
    }

    {   // receiver residual injection R^T dJ/dd^{k+1}, deterministic per cell
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int b = off[tile], e = off[tile + 1];
        if (b < e) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RPT; ++j) sc[(ly * RPT + j + H) * W + lx + H] = av[j];
            __syncthreads();
            const float *d = a.dJdd + ((long long)shot * a.nt + a.k) * a.nrec;
            for (int i = b + tid; i < e; i += NTH) {
                const int cell = rec_cell(a.rec_ent[i]);
                if (i > b && rec_cell(a.rec_ent[i - 1]) == cell) continue;  // not first of its cell
                float sum = 0.f;
                for (int m = i; m < e && rec_cell(a.rec_ent[m]) == cell; ++m) sum += d[rec_id(a.rec_ent[m])];
                const int r = cell / TX, c = cell - r * TX;
                sc[(r + H) * W + c + H] += sum;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RPT; ++j) av[j] = sc[(ly * RPT + j + H) * W + lx + H];
        }
    }

    const long long src = a.src_f[shot];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fidx(g, iz, ix);
            const float s1 = av[j];
            __builtin_nontemporal_store(s1, s1o + f);
            __builtin_nontemporal_store(fmaf(s1, __builtin_nontemporal_load(a.snap + so + f), __builtin_nontemporal_load(a.grad + so + f)), a.grad + so + f);
            if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k] = s1 * a.src_scale;
        }
    }
}

// (8 waves per SIMD: 64 VGPRs, no spill; measured 2 % faster than the
// compiler's choice of 70.  The forward's one-step variants are slower at 8.)
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(8))) void ac2_adj_kernel(Ac2AdjArgs a)
{
    __shared__ float sc[(TZ + 8) * (TX + 8)];
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl;
    adj_tile(a, sc, a.tiles[w - shot * a.ntl], shot);
}

// ---------------------------------------------------------- two-step kernels
// Blocked tiles: the tile and its 8-cell halo are physical cells, so pass A
// and every layer term vanish there and the forward update reduces to
// u^{k+1} = u^k + ((u^k - u^{k-1}) + chat w~^k) (+ source).  One launch
// forms u^{k+1} on the tile + 4 in LDS from u^k on the tile + 8, then
// u^{k+2} on the tile: two steps for one read of u^k, u^{k-1} and chat and
// one write of u^{k+1}, u^{k+2}.  Each value is computed with exactly the
// operations of the single-step kernel, so results agree bit for bit.
constexpr int H2 = 8;                       // u^k halo of a blocked tile
constexpr int W0 = TX + 2 * H2, R0 = TZ + 2 * H2;
constexpr int W1 = TX + 8, R1 = TZ + 8;
constexpr int NRING = R1 * W1 - TZ * TX;    // the 4-cell ring around the tile
// The forward blocked tiles take NTB threads (RB rows each): 8 waves per
// SIMD in 55 VGPRs against 5 at 256 threads (C2: 141 -> 136 us per launch).
// The adjoint keeps 256 threads (512 ran 2 % slower).
constexpr int RING_IT = (NRING + NTH - 1) / NTH;
constexpr int NTB = 512;
constexpr int RB = TZ * TX / NTB;
constexpr int RING_ITB = (NRING + NTB - 1) / NTB;
static_assert(RB * NTB == TZ * TX && NTB % TX == 0, "whole rows per thread");

// The tile + 8 of a field (rows start 32-byte aligned: x0 - 8 + OX is a
// multiple of 8) straight from global memory into LDS:
// 16 bytes per lane and load, item q into the 16-byte slot q (the LDS rows
// of W0 floats have no padding, so item order is slot order).  Every cell
// lies inside the zero frame.  The caller waits for the loads
// (s_waitcnt) before the barrier that publishes the tile.
template <int NT>
__device__ __forceinline__ void dma_tile8(const Grid2 &g, const float *u, float *lds, int x0, int z0)
{
    constexpr int Q = W0 / 4, N4 = R0 * Q;
#pragma unroll
    for (int it = 0; it < (N4 + NT - 1) / NT; ++it) {
        const int q = threadIdx.x + it * NT;
        if (q < N4) {
            const int r = q / Q, c = (q - r * Q) * 4;
            __builtin_amdgcn_global_load_lds((const void *)(u + fidx(g, z0 - H2 + r, x0 - H2 + c)),
                                             (void __attribute__((address_space(3))) *)(lds + (it * NT + (threadIdx.x & ~63)) * 4),
                                             16, 0, 0);
        }
    }
}

// The product chat * s on the tile + 8 in two phases: dma_product_load puts
// s straight into LDS (as dma_tile8) and chat of the same 16-byte items into
// registers; after the caller's wait and barrier, product_in_place multiplies
// each thread's items in LDS (one FP32 product per cell, chat times s).  The
// caller synchronises again before the tile is read.
template <int NT>
__device__ __forceinline__ void dma_product_load(const Grid2 &g, const float *s, const float *mul, float *lds,
                                                 int x0, int z0, float4 (&m)[(R0 * (W0 / 4) + NT - 1) / NT])
{
    constexpr int Q = W0 / 4, N4 = R0 * Q;
#pragma unroll
    for (int it = 0; it < (N4 + NT - 1) / NT; ++it) {
        const int q = threadIdx.x + it * NT;
        if (q < N4) {
            const int r = q / Q, c = (q - r * Q) * 4;
            const long long f = fidx(g, z0 - H2 + r, x0 - H2 + c);
            __builtin_amdgcn_global_load_lds((const void *)(s + f),
                                             (void __attribute__((address_space(3))) *)(lds + (it * NT + (threadIdx.x & ~63)) * 4),
                                             16, 0, 0);
            m[it] = *reinterpret_cast<const float4 *>(mul + f);
        }
    }
}

template <int NT>
__device__ __forceinline__ void product_in_place(float *lds, const float4 (&m)[(R0 * (W0 / 4) + NT - 1) / NT])
{
    constexpr int N4 = R0 * (W0 / 4);
#pragma unroll
    for (int it = 0; it < (N4 + NT - 1) / NT; ++it) {
        const int q = threadIdx.x + it * NT;
        if (q < N4) {
            float4 v = *reinterpret_cast<const float4 *>(lds + 4 * q);
            v.x = m[it].x * v.x; v.y = m[it].y * v.y; v.z = m[it].z * v.z; v.w = m[it].w * v.w;
            *reinterpret_cast<float4 *>(lds + 4 * q) = v;
        }
    }
}

// Cell i of the ring (rows 0-3 and 36-39 of the tile + 4, then columns 0-3
// and 68-71 of rows 4-35), as (row, column) of the tile + 4.
__device__ __forceinline__ void ring_cell(int i, int &r, int &c)
{
    if (i < 8 * W1) {
        const int rr = i / W1;
        r = rr < 4 ? rr : rr + TZ;
        c = i - rr * W1;
    } else {
        const int j = i - 8 * W1, cc = j & 7;
        r = 4 + (j >> 3);
        c = cc < 4 ? cc : cc + TX;
    }
}

// s0: u^k on the tile + 8 (R0 x W0), s1: u^{k+1} on the tile + 4 (R1 x W1)
__device__ __forceinline__ void fwd2_tile(const Ac2Fwd2Args &a, float *s0, float *s1, int tile, int shot)
{
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *um = a.um + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const long long src = a.src_f[shot];
    const float sv0 = src_value(a.src_scale, a.wav[(long long)shot * a.nt + a.k]);
    const float sv1 = src_value(a.src_scale, a.wav[(long long)shot * a.nt + a.k + 1]);
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;

    // own cells: column lx, rows ly*RB .. +RB-1; their chat and u^{k-1} first
    float ch[RB], pm[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        const long long f = fidx(g, z0 + ly * RB + j, x0 + lx);
        ch[j] = chat[f];
        pm[j] = um[f];
    }
    // ring cells of the tile + 4
    float rch[RING_ITB], rpm[RING_ITB];
    long long rf[RING_ITB];
#pragma unroll
    for (int it = 0; it < RING_ITB; ++it) {
        const int i = threadIdx.x + it * NTB;
        rf[it] = -1;
        if (i < NRING) {
            int r, c;
            ring_cell(i, r, c);
            rf[it] = fidx(g, z0 - 4 + r, x0 - 4 + c);
            rch[it] = chat[rf[it]];
            rpm[it] = um[rf[it]];
        }
    }
    dma_tile8<NTB>(g, a.u0 + so, s0, x0, z0);
    __builtin_amdgcn_s_waitcnt(0);       // the tile's direct loads have landed in LDS
    __syncthreads();

    // step k: u^{k+1} on the tile + 4 (own cells, then the ring)
    float uk[RB], u1[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        const int r = ly * RB + j;
        const long long f = fidx(g, z0 + r, x0 + lx);
        const float *cc = s0 + (r + H2) * W0 + lx + H2;
        const float wk = lap8(cc, W0);
        uk[j] = cc[0];
        float inc = fmaf(ch[j], wk, uk[j] - pm[j]);
        if (f == src) inc += sv0;
        u1[j] = uk[j] + inc;
        s1[(r + 4) * W1 + lx + 4] = u1[j];
        __builtin_nontemporal_store(u1[j], a.u1 + so + f);
        if (a.snap0) __builtin_nontemporal_store(wk, a.snap0 + so + f);
    }
#pragma unroll
    for (int it = 0; it < RING_ITB; ++it) {
        const int i = threadIdx.x + it * NTB;
        if (i < NRING) {
            int r, c;
            ring_cell(i, r, c);
            const float *cc = s0 + (r + 4) * W0 + c + 4;
            const float wk = lap8(cc, W0);
            const float u = cc[0];
            float inc = fmaf(rch[it], wk, u - rpm[it]);
            if (rf[it] == src) inc += sv0;
            s1[r * W1 + c] = u + inc;
        }
    }
    __syncthreads();

    // step k+1 on the tile
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        const int r = ly * RB + j;
        const long long f = fidx(g, z0 + r, x0 + lx);
        const float wk = lap8(s1 + (r + 4) * W1 + lx + 4, W1);
        float inc = fmaf(ch[j], wk, u1[j] - uk[j]);
        if (f == src) inc += sv1;
        __builtin_nontemporal_store(u1[j] + inc, a.u2 + so + f);
        if (a.snap1) __builtin_nontemporal_store(wk, a.snap1 + so + f);
    }
}

__global__ __launch_bounds__(NTB) void ac2_fwd2_kernel(Ac2Fwd2Args a)
{
    __shared__ __attribute__((aligned(16))) float s0[R0 * W0];
    __shared__ float s1[R1 * W1];
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl, tile = a.tiles[w - shot * a.ntl];
    fwd2_tile(a, s0, s1, tile, shot);
}

// Adjoint steps k and k-1 on blocked tiles (no receivers within 4 cells):
// s^{k+1} on the tile + 4 from chat s^{k+2} on the tile + 8, then s^k on
// the tile; the gradient gets s^{k+1} w~^k, then s^k w~^{k-1}, as in two
// single steps.
__global__ __launch_bounds__(NTH) void ac2_adj2_kernel(Ac2Adj2Args a)
{
    __shared__ __attribute__((aligned(16))) float p0[R0 * W0];   // chat s^{k+2} on the tile + 8
    __shared__ float p1[R1 * W1];   // chat s^{k+1} on the tile + 4
    const Grid2 &g = a.g;
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl, tile = a.tiles[w - shot * a.ntl];
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *s2 = a.s2 + so, *s3 = a.s3 + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const long long src = a.src_f[shot];
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;

    float ch[RPT], q2[RPT], q3[RPT], gr[RPT], w1[RPT], w0[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const long long f = fidx(g, z0 + ly * RPT + j, x0 + lx);
        ch[j] = chat[f];
        q2[j] = s2[f];
        q3[j] = s3[f];
        gr[j] = __builtin_nontemporal_load(a.grad + so + f);
        w1[j] = __builtin_nontemporal_load(a.snap1 + so + f);
        w0[j] = __builtin_nontemporal_load(a.snap0 + so + f);
    }
    float rch[RING_IT], rq2[RING_IT], rq3[RING_IT];
#pragma unroll
    for (int it = 0; it < RING_IT; ++it) {
        const int i = threadIdx.x + it * NTH;
        if (i < NRING) {
            int r, c;
            ring_cell(i, r, c);
            const long long f = fidx(g, z0 - 4 + r, x0 - 4 + c);
            rch[it] = chat[f];
            rq2[it] = s2[f];
            rq3[it] = s3[f];
        }
    }
    float4 cm[(R0 * (W0 / 4) + NTH - 1) / NTH];
    dma_product_load<NTH>(g, s2, chat, p0, x0, z0, cm);
    __builtin_amdgcn_s_waitcnt(0);       // the tile's direct loads have landed in LDS
    __syncthreads();
    product_in_place<NTH>(p0, cm);
    __syncthreads();

    // step k: s^{k+1} on the tile + 4
    float v1[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j;
        const long long f = fidx(g, z0 + r, x0 + lx);
        float v = lap8(p0 + (r + H2) * W0 + lx + H2, W0);
        v += q2[j] + (q2[j] - q3[j]);
        v1[j] = v;
        p1[(r + 4) * W1 + lx + 4] = ch[j] * v;
        __builtin_nontemporal_store(v, a.o1 + so + f);
        if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k] = v * a.src_scale;
    }
#pragma unroll
    for (int it = 0; it < RING_IT; ++it) {
        const int i = threadIdx.x + it * NTH;
        if (i < NRING) {
            int r, c;
            ring_cell(i, r, c);
            float v = lap8(p0 + (r + 4) * W0 + c + 4, W0);
            v += rq2[it] + (rq2[it] - rq3[it]);
            p1[r * W1 + c] = rch[it] * v;
        }
    }
    __syncthreads();

    // step k-1 on the tile
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j;
        const long long f = fidx(g, z0 + r, x0 + lx);
        float v = lap8(p1 + (r + 4) * W1 + lx + 4, W1);
        v += v1[j] + (v1[j] - q2[j]);
        __builtin_nontemporal_store(v, a.o0 + so + f);
        float t = fmaf(v1[j], w1[j], gr[j]);
        __builtin_nontemporal_store(fmaf(v, w0[j], t), a.grad + so + f);
        if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k - 1] = v * a.src_scale;
    }
}

// ---------------------------------------------------------------- near tiles
// The tiles within 4 cells of the layer, with pass A folded in.  LDS: the stepped field on
// the tile + 8 (as the blocked kernels stage it), the x auxiliary on the
// tile's rows x the tile + 4 columns, the z auxiliary on the tile + 4 rows x
// the tile's columns.
// Every value is formed by the same expression as in separate passes, so
// results do not depend on which tile computes a ring cell.  NTN threads per
// tile (RN rows each): the LDS arrays cap the workgroups per CU, so a
// larger workgroup keeps more waves resident.
constexpr int WPX = TX + 8;      // x auxiliary: columns x0 - 4 .. x0 + TX + 3
constexpr int RPZ = TZ + 8;      // z auxiliary: rows z0 - 4 .. z0 + TZ + 3
constexpr int NU = R0 * W0;      // the field on the tile + 8
constexpr int NTN = 512;         // threads of a near tile
constexpr int RN = TZ * TX / NTN;
static_assert(RN * NTN == TZ * TX && NTN % TX == 0, "whole rows per thread");

// Halo cells of the auxiliaries' LDS arrays: the 4 + 4 columns of the x
// array beside the tile (TZ x 8, one per thread) and the 4 + 4 rows of the z
// array above and below it (8 x TX, two per thread).
constexpr int NHX = TZ * 8, NHZ = 8 * TX;
constexpr int HXI = (NHX + NTN - 1) / NTN, HZI = (NHZ + NTN - 1) / NTN;   // halo cells per thread

__device__ __forceinline__ void halo_x_cell(int i, int &r, int &c)
{
    r = i >> 3;
    const int cc = i & 7;
    c = cc < 4 ? cc : cc + TX;           // column of the x array (x0 - 4 + c)
}

__device__ __forceinline__ void halo_z_cell(int i, int &r, int &c)
{
    const int rr = i / TX;
    c = i - rr * TX;
    r = rr < 4 ? rr : rr + TZ;           // row of the z array (z0 - 4 + r)
}

template <bool SNAP, bool REC>
__device__ __forceinline__ void fwd_near_tile(const Ac2FwdArgs &a, float *su, float *sx, float *sz, int tile,
                                              int shot)
{
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    // ly is uniform over a wavefront (TX lanes): rows and their tables in scalar registers
    const int tid = threadIdx.x, lx = tid % TX, ly = __builtin_amdgcn_readfirstlane(tid / TX);
    const int ix = x0 + lx;
    const bool inx = ix < g.NX;
    const float *__restrict__ chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const float *__restrict__ um = a.um + so;
    const float *__restrict__ phx0 = a.phx0 + so;
    const float *__restrict__ phz0 = a.phz0 + so;
    float *__restrict__ phx = a.phx + so;
    float *__restrict__ phz = a.phz + so;

    // operands of the own cells and of the halo cells first (none depends on LDS)
    const float hxc = inx ? a.hx[ix] : 0.f, pxc = inx ? a.px[ix] : 0.f, ihxc = inx ? a.ihx[ix] : 0.f;
    float ch[RN], pm[RN], hzr[RN], fx[RN], fz[RN], pzr[RN], ihzr[RN];
    unsigned lay = 0u;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int iz = z0 + ly * RN + j;
        const long long f = fidx(g, iz, ix);
        ch[j] = pm[j] = hzr[j] = fx[j] = fz[j] = 0.f;
        pzr[j] = iz < g.NZ ? a.pz[iz] : 0.f;
        ihzr[j] = iz < g.NZ ? a.ihz[iz] : 0.f;
        if (iz < g.NZ && inx) {
            ch[j] = chat[f];
            pm[j] = __builtin_nontemporal_load(um + f);
            hzr[j] = a.hz[iz];
            if (layer_cell_at(g, iz, ix)) {
                lay |= 1u << j;
                fx[j] = phx0[f];
                fz[j] = phz0[f];
            }
        }
    }
    // halo cells of the x and z arrays
    float xhx[HXI], xhz[HXI], xp[HXI], xih[HXI], xf[HXI];
    bool xl[HXI];
    int xr[HXI], xc[HXI];
#pragma unroll
    for (int it = 0; it < HXI; ++it) {
        const int i = tid + it * NTN;
        halo_x_cell(i < NHX ? i : 0, xr[it], xc[it]);
        const int iz = z0 + xr[it], jx = x0 - 4 + xc[it];
        xl[it] = i < NHX && iz < g.NZ && jx >= 0 && jx < g.NX && layer_cell_at(g, iz, jx);
        xhx[it] = xhz[it] = xp[it] = xih[it] = xf[it] = 0.f;
        if (xl[it]) {
            xhx[it] = a.hx[jx]; xhz[it] = a.hz[iz]; xp[it] = a.px[jx]; xih[it] = a.ihx[jx];
            xf[it] = phx0[fidx(g, iz, jx)];
        }
    }
    float zhx[HZI], zhz[HZI], zp[HZI], zih[HZI], zf[HZI];
    bool zl[HZI];
    int zr[HZI], zc[HZI];
#pragma unroll
    for (int it = 0; it < HZI; ++it) {
        const int i = tid + it * NTN;
        halo_z_cell(i < NHZ ? i : 0, zr[it], zc[it]);
        const int iz = z0 - 4 + zr[it], jx = x0 + zc[it];
        zl[it] = i < NHZ && iz >= 0 && iz < g.NZ && jx < g.NX && layer_cell_at(g, iz, jx);
        zhx[it] = zhz[it] = zp[it] = zih[it] = zf[it] = 0.f;
        if (zl[it]) {
            zhx[it] = a.hx[jx]; zhz[it] = a.hz[iz]; zp[it] = a.pz[iz]; zih[it] = a.ihz[iz];
            zf[it] = phz0[fidx(g, iz, jx)];
        }
    }
    dma_tile8<NTN>(g, a.u + so, su, x0, z0);               // u^k on the tile + 8
    const long long src = a.src_f[shot];
    const float sval = src_value(a.src_scale, a.wav[(long long)shot * a.nt + a.k]);
    __builtin_amdgcn_s_waitcnt(0);       // the tile's direct loads have landed in LDS
    __syncthreads();

    // pass A: phi~^k on the own layer cells (written out) and the halo cells
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int r = ly * RN + j;
        float vx = 0.f, vz = 0.f;
        if (lay >> j & 1u) {
            const int iz = z0 + r;
            const long long f = fidx(g, iz, ix);
            const float *cu = su + (r + H2) * W0 + lx + H2;
            const float qx = 2.f * (hzr[j] - hxc) * ihxc;
            const float qz = 2.f * (hxc - hzr[j]) * ihzr[j];
            vx = pxc * fx[j] + qx * d8(cu, 1);
            vz = pzr[j] * fz[j] + qz * d8(cu, (long long)W0);
            phx[f] = vx;
            phz[f] = vz;
        }
        sx[r * WPX + lx + 4] = vx;
        sz[(r + 4) * TX + lx] = vz;
    }
#pragma unroll
    for (int it = 0; it < HXI; ++it) {
        if (tid + it * NTN >= NHX) continue;
        float v = 0.f;
        if (xl[it]) {
            const float qx = 2.f * (xhz[it] - xhx[it]) * xih[it];
            v = xp[it] * xf[it] + qx * d8(su + (xr[it] + H2) * W0 + xc[it] + 4, 1);
        }
        sx[xr[it] * WPX + xc[it]] = v;
    }
#pragma unroll
    for (int it = 0; it < HZI; ++it) {
        if (tid + it * NTN >= NHZ) continue;
        float v = 0.f;
        if (zl[it]) {
            const float qz = 2.f * (zhx[it] - zhz[it]) * zih[it];
            v = zp[it] * zf[it] + qz * d8(su + (zr[it] + 4) * W0 + zc[it] + H2, (long long)W0);
        }
        sz[zr[it] * TX + zc[it]] = v;
    }
    __syncthreads();

    // pass B on the tile
    float *uo = a.un + so;
    float un[RN];
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int r = ly * RN + j, iz = z0 + r;
        const float *cu = su + (r + H2) * W0 + lx + H2;
        const float uc = cu[0];
        float w = lap8(cu, W0);
        un[j] = 0.f;
        if (iz < g.NZ && inx) {
            const long long f = fidx(g, iz, ix);
            w += d8(sx + r * WPX + lx + 4, 1) + d8(sz + (r + 4) * TX + lx, (long long)TX);
            const float hx = hxc, hz = hzr[j];
            // alpha (beta u - gamma um + chat w + src) with
            // beta u - gamma um = u + (u - um) + (hx + hz) um - 4 hx hz u
            const float alpha = 1.f / (1.f + hx + hz);
            const float umf = pm[j];
            float inc = (uc - umf) + ((hx + hz) * umf - 4.f * hx * hz * uc) + ch[j] * w;
            if (f == src) inc += sval;
            if (a.nsrc > 1) inc += node_sources(a, tile, shot, r * TX + lx);
            const float v = alpha * (uc + inc);
            __builtin_nontemporal_store(v, uo + f);
            un[j] = v;
            if constexpr (SNAP) __builtin_nontemporal_store(w, a.snap + so + f);
        }
    }

    if constexpr (REC) {
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int b = off[tile], e = off[tile + 1];
        if (b < e) {                      // uniform over the block
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RN; ++j) su[(ly * RN + j + H2) * W0 + lx + H2] = un[j];
            __syncthreads();
            for (int i = b + tid; i < e; i += NTN) {
                const int ent = a.rec_ent[i];
                const int cell = rec_cell(ent);
                const int r = cell / TX, c = cell - r * TX;
                a.seis[((long long)shot * a.nt + a.k) * a.nrec + rec_id(ent)] = su[(r + H2) * W0 + c + H2];
            }
        }
    }
}

// 34.8 KB of LDS per tile allow 4 tiles per CU: 8 waves per SIMD at 512
// threads, which the forward reaches in 56 VGPRs without spills (256-thread
// tiles held 4 waves per SIMD and ran the C2 near tiles 16 % slower).  The
// adjoint keeps 66 VGPRs and 7 waves: limited to 64 it spills and runs 4 %
// slower.  Taking the row index through readfirstlane puts the rows' z
// tables in scalar registers (forward 62 -> 56, adjoint 78 -> 66 VGPRs).
template <bool SNAP, bool REC>
__global__ __launch_bounds__(NTN) __attribute__((amdgpu_waves_per_eu(8))) void ac2_near_kernel(Ac2FwdArgs a)
{
    __shared__ __attribute__((aligned(16))) float su[NU];
    __shared__ float sx[TZ * WPX];
    __shared__ float sz[RPZ * TX];
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl, tile = a.tiles[w - shot * a.ntl];
    fwd_near_tile<SNAP, REC>(a, su, sx, sz, tile, shot);
}

// Step k of the tiles by the layer and steps k, k+1 of the blocked tiles in
// one launch.  The two read only u^k, u^{k-1} (and phi~^{k-1}) and write
// disjoint cells of u^{k+1} (and u^{k+2}, phi~^k, the seismograms), so they
// need no order; one grid lets the near tiles fill the blocked launch's last
// round instead of waiting for it.  The blocked tiles come first in the grid;
// the two share one LDS buffer.
constexpr int NPAIR_LDS = NU + TZ * WPX + RPZ * TX > R0 * W0 + R1 * W1 ? NU + TZ * WPX + RPZ * TX
                                                                      : R0 * W0 + R1 * W1;
static_assert(NTN == NTB, "one block size for the pair");
template <bool SNAP, bool REC>
__global__ __launch_bounds__(NTN) __attribute__((amdgpu_waves_per_eu(8)))
void ac2_fwd_pair_kernel(Ac2FwdArgs a, Ac2Fwd2Args b)
{
    __shared__ __attribute__((aligned(16))) float lds[NPAIR_LDS];
    const int nb = b.ntl * b.nshots;
    int w = xcd_work_id(nb + a.ntl * a.nshots);
    if (w < nb) {
        const int shot = w / b.ntl;
        fwd2_tile(b, lds, lds + R0 * W0, b.tiles[w - shot * b.ntl], shot);
    } else {
        w -= nb;
        const int shot = w / a.ntl;
        fwd_near_tile<SNAP, REC>(a, lds, lds + NU, lds + NU + TZ * WPX, a.tiles[w - shot * a.ntl], shot);
    }
}

__device__ __forceinline__ void adj_near_tile(const Ac2AdjArgs &a, float *sc, float *sx, float *sz, int tile,
                                              int shot)
{
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    // ly is uniform over a wavefront (TX lanes): rows and their tables in scalar registers
    const int tid = threadIdx.x, lx = tid % TX, ly = __builtin_amdgcn_readfirstlane(tid / TX);
    const int ix = x0 + lx;
    const bool inx = ix < g.NX;
    const float *__restrict__ s2 = a.s2 + so;
    const float *__restrict__ s3 = a.s3 + so;
    const float *__restrict__ chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const float *__restrict__ cx0 = a.cx0 + so;
    const float *__restrict__ cz0 = a.cz0 + so;
    float *__restrict__ cxo = a.cx + so;
    float *__restrict__ czo = a.cz + so;

    const float hxc = inx ? a.hx[ix] : 0.f, pxc = inx ? a.px[ix] : 0.f, ihxc = inx ? a.ihx[ix] : 0.f;
    float sc2[RN], q3[RN], hzr[RN], fx[RN], fz[RN], pzr[RN], ihzr[RN];
    unsigned lay = 0u;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int iz = z0 + ly * RN + j;
        const long long f = fidx(g, iz, ix);
        sc2[j] = s2[f];
        q3[j] = hzr[j] = fx[j] = fz[j] = 0.f;
        pzr[j] = iz < g.NZ ? a.pz[iz] : 0.f;
        ihzr[j] = iz < g.NZ ? a.ihz[iz] : 0.f;
        if (iz < g.NZ && inx) {
            q3[j] = __builtin_nontemporal_load(s3 + f);
            hzr[j] = a.hz[iz];
            if (layer_cell_at(g, iz, ix)) {
                lay |= 1u << j;
                fx[j] = cx0[f];
                fz[j] = cz0[f];
            }
        }
    }
    // halo cells of the x and z arrays
    float xhx[HXI], xhz[HXI], xp[HXI], xih[HXI], xf[HXI];
    bool xl[HXI];
    int xr[HXI], xc[HXI];
#pragma unroll
    for (int it = 0; it < HXI; ++it) {
        const int i = tid + it * NTN;
        halo_x_cell(i < NHX ? i : 0, xr[it], xc[it]);
        const int iz = z0 + xr[it], jx = x0 - 4 + xc[it];
        xl[it] = i < NHX && iz < g.NZ && jx >= 0 && jx < g.NX && layer_cell_at(g, iz, jx);
        xhx[it] = xhz[it] = xp[it] = xih[it] = xf[it] = 0.f;
        if (xl[it]) {
            xhx[it] = a.hx[jx]; xhz[it] = a.hz[iz]; xp[it] = a.px[jx]; xih[it] = a.ihx[jx];
            xf[it] = cx0[fidx(g, iz, jx)];
        }
    }
    float zhx[HZI], zhz[HZI], zp[HZI], zih[HZI], zf[HZI];
    bool zl[HZI];
    int zr[HZI], zc[HZI];
#pragma unroll
    for (int it = 0; it < HZI; ++it) {
        const int i = tid + it * NTN;
        halo_z_cell(i < NHZ ? i : 0, zr[it], zc[it]);
        const int iz = z0 - 4 + zr[it], jx = x0 + zc[it];
        zl[it] = i < NHZ && iz >= 0 && iz < g.NZ && jx < g.NX && layer_cell_at(g, iz, jx);
        zhx[it] = zhz[it] = zp[it] = zih[it] = zf[it] = 0.f;
        if (zl[it]) {
            zhx[it] = a.hx[jx]; zhz[it] = a.hz[iz]; zp[it] = a.pz[iz]; zih[it] = a.ihz[iz];
            zf[it] = cz0[fidx(g, iz, jx)];
        }
    }
    float4 cm[(R0 * (W0 / 4) + NTN - 1) / NTN];
    dma_product_load<NTN>(g, s2, chat, sc, x0, z0, cm);     // chat s^{k+2} on the tile + 8
    __builtin_amdgcn_s_waitcnt(0);       // the tile's direct loads have landed in LDS
    __syncthreads();
    product_in_place<NTN>(sc, cm);
    __syncthreads();

    // pass A: c^{k+1} on the own layer cells (written out) and the halo cells
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int r = ly * RN + j;
        float vx = 0.f, vz = 0.f;
        if (lay >> j & 1u) {
            const int iz = z0 + r;
            const long long f = fidx(g, iz, ix);
            const float *cc = sc + (r + H2) * W0 + lx + H2;
            const float qx = 2.f * (hzr[j] - hxc) * ihxc;
            const float qz = 2.f * (hxc - hzr[j]) * ihzr[j];
            vx = pxc * fx[j] - qx * d8(cc, 1);
            vz = pzr[j] * fz[j] - qz * d8(cc, (long long)W0);
            cxo[f] = vx;
            czo[f] = vz;
        }
        sx[r * WPX + lx + 4] = vx;
        sz[(r + 4) * TX + lx] = vz;
    }
#pragma unroll
    for (int it = 0; it < HXI; ++it) {
        if (tid + it * NTN >= NHX) continue;
        float v = 0.f;
        if (xl[it]) {
            const float qx = 2.f * (xhz[it] - xhx[it]) * xih[it];
            v = xp[it] * xf[it] - qx * d8(sc + (xr[it] + H2) * W0 + xc[it] + 4, 1);
        }
        sx[xr[it] * WPX + xc[it]] = v;
    }
#pragma unroll
    for (int it = 0; it < HZI; ++it) {
        if (tid + it * NTN >= NHZ) continue;
        float v = 0.f;
        if (zl[it]) {
            const float qz = 2.f * (zhx[it] - zhz[it]) * zih[it];
            v = zp[it] * zf[it] - qz * d8(sc + (zr[it] + 4) * W0 + zc[it] + H2, (long long)W0);
        }
        sz[zr[it] * TX + zc[it]] = v;
    }
    __syncthreads();

    // the snapshot and the gradient accumulator of the own cells, loaded
    // here so that their latency overlaps pass B (loaded with the other
    // operands before pass A, they would spill)
    float snv[RN], grv[RN];
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int iz = z0 + ly * RN + j;
        snv[j] = grv[j] = 0.f;
        if (iz < g.NZ && inx) {
            const long long f = fidx(g, iz, ix);
            snv[j] = __builtin_nontemporal_load(a.snap + so + f);
            grv[j] = __builtin_nontemporal_load(a.grad + so + f);
        }
    }

    // pass B on the tile
    float *s1o = a.s1 + so;
    float av[RN];
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int r = ly * RN + j, iz = z0 + r;
        float v = lap8(sc + (r + H2) * W0 + lx + H2, W0);
        if (iz < g.NZ && inx) {
            v -= d8(sx + r * WPX + lx + 4, 1) + d8(sz + (r + 4) * TX + lx, (long long)TX);
            const float hx = hxc, hz = hzr[j];
            const float s3f = q3[j];
            v += sc2[j] + ((sc2[j] - s3f) + ((hx + hz) * s3f - 4.f * hx * hz * sc2[j]));
        }
        av[j] = v;
    }

    {   // receiver residual injection R^T dJ/dd^{k+1}, deterministic per cell
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int b = off[tile], e = off[tile + 1];
        if (b < e) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RN; ++j) sc[(ly * RN + j + H2) * W0 + lx + H2] = av[j];
            __syncthreads();
            const float *d = a.dJdd + ((long long)shot * a.nt + a.k) * a.nrec;
            for (int i = b + tid; i < e; i += NTN) {
                const int cell = rec_cell(a.rec_ent[i]);
                if (i > b && rec_cell(a.rec_ent[i - 1]) == cell) continue;  // not first of its cell
                float sum = 0.f;
                for (int m = i; m < e && rec_cell(a.rec_ent[m]) == cell; ++m) sum += d[rec_id(a.rec_ent[m])];
                const int r = cell / TX, c = cell - r * TX;
                sc[(r + H2) * W0 + c + H2] += sum;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RN; ++j) av[j] = sc[(ly * RN + j + H2) * W0 + lx + H2];
        }
    }

    const long long src = a.src_f[shot];
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int r = ly * RN + j, iz = z0 + r;
        if (iz < g.NZ && inx) {
            const long long f = fidx(g, iz, ix);
            const float s1 = av[j] / (1.f + hxc + hzr[j]);
            __builtin_nontemporal_store(s1, s1o + f);
            __builtin_nontemporal_store(fmaf(s1, snv[j], grv[j]), a.grad + so + f);
            if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k] = s1 * a.src_scale;
        }
    }
}

__global__ __launch_bounds__(NTN) __attribute__((amdgpu_waves_per_eu(6))) void ac2_adj_near_kernel(Ac2AdjArgs a)
{
    __shared__ __attribute__((aligned(16))) float sc[NU];
    __shared__ float sx[TZ * WPX];
    __shared__ float sz[RPZ * TX];
    const int w = xcd_work_id(a.ntl * a.nshots);
    const int shot = w / a.ntl, tile = a.tiles[w - shot * a.ntl];
    adj_near_tile(a, sc, sx, sz, tile, shot);
}

// ------------------------------------------------------------------ launchers
void launch_ac2_fwd2(const Ac2Fwd2Args &a, hipStream_t s)
{
    const int nb = a.ntl * a.nshots;
    if (nb == 0) return;
    ac2_fwd2_kernel<<<nb, NTB, 0, s>>>(a);
}

void launch_ac2_adj2(const Ac2Adj2Args &a, hipStream_t s)
{
    const int nb = a.ntl * a.nshots;
    if (nb == 0) return;
    ac2_adj2_kernel<<<nb, NTH, 0, s>>>(a);
}

void launch_ac2_fwd_pair(const Ac2FwdArgs &a, const Ac2Fwd2Args &b, hipStream_t s)
{
    const int nb = a.ntl * a.nshots + b.ntl * b.nshots;
    if (nb == 0) return;
    if (a.seis) { ac2_fwd_pair_kernel<false, true><<<nb, NTN, 0, s>>>(a, b); return; }
    if (a.snap) ac2_fwd_pair_kernel<true, false><<<nb, NTN, 0, s>>>(a, b);
    else ac2_fwd_pair_kernel<false, false><<<nb, NTN, 0, s>>>(a, b);
}

void launch_ac2_fwd(const Ac2FwdArgs &a, bool near, hipStream_t s)
{
    const int nb = a.ntl * a.nshots;
    if (nb == 0) return;
    const bool snap = a.snap != nullptr, rec = a.seis != nullptr;
    if (near) {
        if (snap) { if (rec) ac2_near_kernel<true, true><<<nb, NTN, 0, s>>>(a); else ac2_near_kernel<true, false><<<nb, NTN, 0, s>>>(a); }
        else      { if (rec) ac2_near_kernel<false, true><<<nb, NTN, 0, s>>>(a); else ac2_near_kernel<false, false><<<nb, NTN, 0, s>>>(a); }
    } else {
        if (snap) { if (rec) ac2_fwd_kernel<true, true><<<nb, NTH, 0, s>>>(a); else ac2_fwd_kernel<true, false><<<nb, NTH, 0, s>>>(a); }
        else      { if (rec) ac2_fwd_kernel<false, true><<<nb, NTH, 0, s>>>(a); else ac2_fwd_kernel<false, false><<<nb, NTH, 0, s>>>(a); }
    }
}

void launch_ac2_adj(const Ac2AdjArgs &a, bool near, hipStream_t s)
{
    const int nb = a.ntl * a.nshots;
    if (nb == 0) return;
    if (near) ac2_adj_near_kernel<<<nb, NTN, 0, s>>>(a);
    else      ac2_adj_kernel<<<nb, NTH, 0, s>>>(a);
}

// ---------------------------------------------------------------- model prep
// chat = dt^2 c^2 / dx^2 and the padded velocity on the frame (edge
// replication of the physical model; zero outside the padded grid).
__global__ void ac2_prep_kernel(Grid2 g, int nmodels, const float *vp, double dt, double dx,
                                float *chat, float *cpad)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        const int fz = (int)(f / g.SX), fx = (int)(f - (long long)fz * g.SX);
        const int iz = fz - OZ, ix = fx - OX;
        float c = 0.f, ch = 0.f;
        if (iz >= 0 && iz < g.NZ && ix >= 0 && ix < g.NX) {
            const int pz = min(max(iz - g.P, 0), g.nz - 1), px = min(max(ix - g.P, 0), g.nx - 1);
            c = vp[(m * g.nz + pz) * g.nx + px];
            const double cd = c;
            ch = (float)(dt * dt * cd * cd / (dx * dx));
        }
        chat[i] = ch;
        cpad[i] = c;
    }
}

void launch_ac2_prep(const Grid2 &g, int nmodels, const float *vp, double dt, double dx,
                     float *chat, float *cpad, hipStream_t s)
{
    const long long n = (long long)nmodels * g.plane;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac2_prep_kernel<<<blocks, 256, 0, s>>>(g, nmodels, vp, dt, dx, chat, cpad);
}

// ------------------------------------------------------------ grad finalize
// Pass 1: per padded cell, sum dJ/dchat over the model's shots in shot order
// (coalesced over cells).  Pass 2: per physical cell, sum the padded cells
// that replicate it and apply the chain rule dchat/dc = 2 dt^2 c / dx^2.
__global__ void ac2_sum_shots_kernel(Grid2 g, int nmodels, int spm, const float *grad, float *acc)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        float v = 0.f;
        for (int s = 0; s < spm; ++s) v += grad[(m * spm + s) * g.plane + f];
        acc[i] = v;
    }
}

__global__ void ac2_finalize_kernel(Grid2 g, int nmodels, const float *acc, const float *cpad,
                                    double dt, double dx, float *g_vp)
{
    const long long n = (long long)nmodels * g.nz * g.nx;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / ((long long)g.nz * g.nx);
        const long long rem = i - m * g.nz * g.nx;
        const int iz = (int)(rem / g.nx), ix = (int)(rem - (long long)iz * g.nx);
        const int zlo = iz == 0 ? 0 : iz + g.P, zhi = iz == g.nz - 1 ? g.NZ - 1 : iz + g.P;
        const int xlo = ix == 0 ? 0 : ix + g.P, xhi = ix == g.nx - 1 ? g.NX - 1 : ix + g.P;
        const float *am = acc + m * g.plane;
        float v = 0.f;
        for (int pz = zlo; pz <= zhi; ++pz)
            for (int px = xlo; px <= xhi; ++px)
                v += am[(long long)(pz + OZ) * g.SX + px + OX];
        const double c = cpad[m * g.plane + (long long)(iz + g.P + OZ) * g.SX + ix + g.P + OX];
        g_vp[i] = (float)(2.0 * dt * dt * c / (dx * dx)) * v;
    }
}

void launch_ac2_finalize(const Grid2 &g, int nmodels, int spm, const float *grad, float *acc,
                         const float *cpad, double dt, double dx, float *g_vp, hipStream_t s)
{
    long long n = (long long)nmodels * g.plane;
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac2_sum_shots_kernel<<<blocks, 256, 0, s>>>(g, nmodels, spm, grad, acc);
    n = (long long)nmodels * g.nz * g.nx;
    blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac2_finalize_kernel<<<blocks, 256, 0, s>>>(g, nmodels, acc, cpad, dt, dx, g_vp);
}

} // namespace sg
