// ad2.hip -- gfx950 kernels of the 2-D acoustic equation in divergence form,
// u_tt = div(c^2 grad u) + f (Eq. (12) as printed), on a staggered grid with
// a convolutional PML, and its adjoint (Eqs. (4)-(5)).
//
// Scaled variables: chat = dt^2 c^2 / dx^2 at the nodes, khat = (chat_i +
// chat_{i+1}) / 2 at the half nodes (a neighbour beyond the padded grid takes
// the edge value, so chat is replicated one node beyond it), differences
// without the 1/dx factor,
//   Dp' u (i + 1/2) = 9/8 (u_{i+1} - u_i) - 1/24 (u_{i+2} - u_{i-1}),
//   Dm' q (i)       = 9/8 (q_i - q_{i-1}) - 1/24 (q_{i+1} - q_{i-2}),
// psi' = dx psi and xi' = dt^2 xi for the layer memories.  Forward step k,
// one launch over (tile, shot):
//   G' = Dp' u^k;   psi'^{k+1} = bh psi'^k + ah G';   S' = G' + psi'^{k+1}
//   q' = khat S';   H' = Dm' q';   xi'^{k+1} = b xi'^k + a H'
//   u^{k+1} = 2 u^k - u^{k-1} + H'x + xi'x + H'z + xi'z + dt^2/(dx dz) sum_j r_j(t_k)
// Half-node values exist on [0, NX) x [0, NZ) only (zero beyond), so that
// Dm'^T = -Dp'.  psi' is read in the halo and written by its owner, so it
// alternates between two buffers; xi' is read only at its own node and is
// updated in place.
//
// Adjoint launch k computes lambda^k = dJ/du^k.  The layer adjoints are
// kept multiplied by their constant coefficients, Y = a dJ/dxi' (nodes) and
// Z = ah dJ/dpsi' (half nodes), so they vanish outside the layer:
//   Y^{k+1} = a lambda^{k+1} + b Y^{k+2};   Hb = lambda^{k+1} + Y^{k+1}
//   qb = -Dp' Hb;  Sb = khat qb;  Z^{k+1} = ah Sb + bh Z^{k+2};  Gb = Sb + Z^{k+1}
//   lambda^k = 2 lambda^{k+1} - lambda^{k+2} - Dm' Gbx - Dm' Gbz + R^T dJ/dd_{k-1}
//   dJ/dchat_i += 1/2 (qb S' at the two half nodes beside node i, per axis),
//   S' of forward step k being a snapshot
// Y and Z alternate between two buffers like psi'.
// Cache policy: u^{k-1} (lambda^{k+2}) and its overwrite, the xi' memories,
// the snapshot stores and the gradient accumulator are streamed
// (non-temporal); the
// snapshot loads of the adjoint stay cached, since the half-node averages
// read each of them from two rows (streaming them cost 16 % of the adjoint).
#include <algorithm>
#include "ad2_internal.h"

namespace sg {
namespace {

// 512 threads per 64 x 32 tile, 4 rows each: 8 waves per SIMD, against 5
// with 256 threads of 8 rows (C2 grid: forward 391 -> 347 us, adjoint 480 ->
// 450 us per step).  A thread's rows are uniform over its wavefront (TX
// lanes); taken through readfirstlane, they put the z tables in scalar
// registers (46-62 VGPRs against 61-65, with a spill, before), which leaves
// room to load the adjoint's gradient accumulator with the other operands
// before the first barrier (adjoint 457 -> 413 us per step).
constexpr int NTA = 512;
constexpr int RPA = TZ * TX / NTA;
static_assert(RPA * NTA == TZ * TX && NTA % TX == 0, "whole rows per thread");
constexpr int AH = 3;              // halo of the composite stencil Dm' khat Dp'
constexpr int AW = TX + 2 * AH;    // node tile with halo: AR rows of AW
constexpr int AR = TZ + 2 * AH;
constexpr int QXW = TX + 3;        // x half nodes x0-2 .. x0+TX on each row of the tile
constexpr float S1 = (float)(9.0 / 8.0);
constexpr float S2 = (float)(-1.0 / 24.0);

__device__ __forceinline__ long long fr(const Grid2 &g, int iz, int ix)
{
    return (long long)(iz + OZ) * g.SX + ix + OX;
}

// 9/8 (c - b) - 1/24 (d - a) of four consecutive values: Dp' at i + 1/2
// from (u_{i-1}, u_i, u_{i+1}, u_{i+2}), Dm' at i from (q_{i-2}, .., q_{i+1}).
__device__ __forceinline__ float d4(float a, float b, float c, float d)
{
    return fmaf(S1, c - b, S2 * (d - a));
}

// Consecutive work ids on one XCD (workgroups are dealt to the 8 XCDs
// round-robin), so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_id(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, j = b / NXCD;
    return x * per + min(x, rem) + j;
}

// Does the tile or its 3-node halo reach the absorbing layer or the edge of
// the grid (layer memories, masks of the half-node range)?
__device__ __forceinline__ bool near_edge(const Grid2 &g, int x0, int z0)
{
    return x0 - AH < g.P || x0 + TX + AH > g.P + g.nx || z0 - AH < g.P || z0 + TZ + AH > g.P + g.nz;
}

// acc[cell] = sum of val(entry) over the tile's entries [b, e) of each local
// cell (acc: TX*TZ floats, zeroed here).  Entries are sorted by cell; the
// first entry of each cell sums its run in entry order, so duplicates add up
// deterministically.  Every thread of the block must call this.
template <class CellOf, class ValOf>
__device__ __forceinline__ void gather_entries(float *acc, const int *ent, int b, int e, CellOf cell_of, ValOf val_of)
{
    for (int i = threadIdx.x; i < TX * TZ; i += NTA) acc[i] = 0.f;
    __syncthreads();
    for (int i = b + (int)threadIdx.x; i < e; i += NTA) {
        const int c = cell_of(ent[i]);
        if (i > b && cell_of(ent[i - 1]) == c) continue;
        float v = 0.f;
        for (int j = i; j < e && cell_of(ent[j]) == c; ++j) v += val_of(ent[j]);
        acc[c] = v;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ forward
// Work split of a tile: thread (lx, ly) owns column x0 + lx and rows
// r0 = ly*RPA .. r0+RPA-1.  The z fluxes of its column (its own half rows and
// the three around them that its Dm' needs) are computed in registers from
// its column of the u tile; the x fluxes go through LDS (own half column by
// every thread, the three extra columns x0-2, x0-1, x0+TX by the first 3*TZ
// threads).  chat of the own column is read once per thread; the right
// neighbour's comes from the next lane (one wavefront = one tile row).  The
// z part runs first so that only Hz and u^k of the own rows stay live.
template <bool NEAR, bool SNAP>
__device__ __forceinline__ float fwd_xflux(const Ad2FwdArgs &a, const float *su, long long so, int x0, int z0, int r,
                                           int h, float c0, float c1)
{
    const Grid2 &g = a.g;
    const int iz = z0 + r, ix = x0 - 2 + h;
    const float *s = su + (r + AH) * AW + h;
    const float G = d4(s[0], s[1], s[2], s[3]);
    float q = 0.f;
    if (!NEAR || (ix >= 0 && ix < g.NX)) {
        const long long f = fr(g, iz, ix);
        const bool own = h >= 2 && h < TX + 2 && iz < g.NZ;
        float S = G;
        if constexpr (NEAR) {
            const float p = fmaf(a.t.bhx[ix], a.psx[so + f], a.t.ahx[ix] * G);
            S = G + p;
            if (own) a.psxn[so + f] = p;
        }
        if constexpr (SNAP) {
            if (own) __builtin_nontemporal_store(S, a.snx + so + f);
        }
        q = 0.5f * (c0 + c1) * S;
    }
    return q;
}

template <bool NEAR, bool SNAP, bool REC>
__device__ __forceinline__ void fwd_tile(const Ad2FwdArgs &a, float *su, float *qx, int tile, int shot)
{
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *u = a.u + so;
    const float *ch = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const int tid = threadIdx.x, lx = tid % TX, ly = __builtin_amdgcn_readfirstlane(tid / TX), r0 = ly * RPA, ix = x0 + lx;

    // u^k on the tile + 3 straight from global memory into LDS: 4 bytes per
    // lane and load into consecutive LDS words (item order is the row-major
    // order of su); every cell lies inside the zero frame
    {
        constexpr int NV = AR * AW, K = (NV + NTA - 1) / NTA;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = tid + k * NTA;
            if (i < NV) {
                const int r = i / AW, c = i - r * AW;
                __builtin_amdgcn_global_load_lds((const void *)(u + fr(g, z0 - AH + r, x0 - AH + c)),
                                                 (void __attribute__((address_space(3))) *)(su + k * NTA + (tid & ~63)),
                                                 4, 0, 0);
            }
        }
    }
    float cz[RPA + 4];                    // chat of rows z0+r0-2 .. z0+r0+RPA+1
#pragma unroll
    for (int m = 0; m < RPA + 4; ++m) cz[m] = ch[fr(g, z0 + r0 - 2 + m, ix)];
    float um[RPA];                        // u^{k-1} of the own rows, loaded early
#pragma unroll
    for (int j = 0; j < RPA; ++j) um[j] = __builtin_nontemporal_load(a.um + so + fr(g, z0 + r0 + j, ix));
    __builtin_amdgcn_s_waitcnt(0);       // the tile's direct loads have landed in LDS
    __syncthreads();

    // z fluxes of the own column at half rows z0+r0-2+m, m = 0 .. RPA+2
    float uc[RPA], hz[RPA];
    {
        float uz[RPA + 6];
#pragma unroll
        for (int m = 0; m < RPA + 6; ++m) uz[m] = su[(r0 + m) * AW + lx + AH];
        float qz[RPA + 3];
#pragma unroll
        for (int m = 0; m < RPA + 3; ++m) {
            const int iz = z0 + r0 - 2 + m;
            const float G = d4(uz[m], uz[m + 1], uz[m + 2], uz[m + 3]);
            float q = 0.f;
            if (!NEAR || (iz >= 0 && iz < g.NZ)) {
                const long long f = fr(g, iz, ix);
                const bool own = m >= 2 && m < RPA + 2 && ix < g.NX;
                float S = G;
                if constexpr (NEAR) {
                    const float p = fmaf(a.t.bhz[iz], a.psz[so + f], a.t.ahz[iz] * G);
                    S = G + p;
                    if (own) a.pszn[so + f] = p;
                }
                if constexpr (SNAP) {
                    if (own) __builtin_nontemporal_store(S, a.snz + so + f);
                }
                q = 0.5f * (cz[m] + cz[m + 1]) * S;
            }
            qz[m] = q;
        }
#pragma unroll
        for (int j = 0; j < RPA; ++j) {
            uc[j] = uz[j + 3];
            hz[j] = d4(qz[j], qz[j + 1], qz[j + 2], qz[j + 3]);
        }
    }
#pragma unroll
    for (int j = 0; j < RPA; ++j) {
        const float c0 = cz[j + 2];
        float c1 = __shfl_down(c0, 1, TX);
        if (lx == TX - 1) c1 = ch[fr(g, z0 + r0 + j, ix + 1)];
        qx[(r0 + j) * QXW + lx + 2] = fwd_xflux<NEAR, SNAP>(a, su, so, x0, z0, r0 + j, lx + 2, c0, c1);
    }
    if (tid < 3 * TZ) {
        const int r = tid / 3, e = tid - 3 * r, h = e == 2 ? TX + 2 : e;
        const long long f = fr(g, z0 + r, x0 - 2 + h);
        qx[r * QXW + h] = fwd_xflux<NEAR, SNAP>(a, su, so, x0, z0, r, h, ch[f], ch[f + 1]);
    }
    __syncthreads();                      // qx complete; su no longer read

    const int ntiles = g.ntx * g.ntz;
    const int *soff = a.src_off + (long long)shot * (ntiles + 1);
    const int sb = soff[tile], se = soff[tile + 1];
    if (sb < se) {                        // uniform over the block
        const float *w = a.wav + (long long)shot * a.nsrc * a.nt + a.k;
        gather_entries(su, a.src_ent, sb, se, [](int e) { return src_cell(e); },
                       [&](int e) { return a.src_scale * w[(long long)src_node(e) * a.nt]; });
    }
    float un[RPA];
#pragma unroll
    for (int j = 0; j < RPA; ++j) {
        const int r = r0 + j, iz = z0 + r;
        const float *qa = qx + r * QXW + lx;
        const float Hx = d4(qa[0], qa[1], qa[2], qa[3]);
        un[j] = 0.f;
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fr(g, iz, ix);
            float inc = Hx + hz[j];
            if constexpr (NEAR) {
                const float xx = fmaf(a.t.b0x[ix], __builtin_nontemporal_load(a.xix + so + f), a.t.a0x[ix] * Hx);
                const float xz = fmaf(a.t.b0z[iz], __builtin_nontemporal_load(a.xiz + so + f), a.t.a0z[iz] * hz[j]);
                __builtin_nontemporal_store(xx, a.xix + so + f);
                __builtin_nontemporal_store(xz, a.xiz + so + f);
                inc += xx + xz;
            }
            inc += uc[j] - um[j];
            if (sb < se) inc += su[r * TX + lx];
            const float v = uc[j] + inc;
            __builtin_nontemporal_store(v, a.un + so + f);
            un[j] = v;
        }
    }
    if constexpr (REC) {
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int b = off[tile], e = off[tile + 1];
        if (b < e) {                      // uniform over the block
            __syncthreads();
#pragma unroll
            for (int j = 0; j < RPA; ++j) su[(r0 + j) * TX + lx] = un[j];
            __syncthreads();
            for (int i = b + tid; i < e; i += NTA) {
                const int ent = a.rec_ent[i];
                a.seis[((long long)shot * a.nt + a.k) * a.nrec + rec_id(ent)] = su[rec_cell(ent)];
            }
        }
    }
}

template <bool SNAP, bool REC>
__global__ __launch_bounds__(NTA) __attribute__((amdgpu_waves_per_eu(8))) void ad2_fwd_kernel(Ad2FwdArgs a)
{
    __shared__ float su[AR * AW];
    __shared__ float qx[TZ * QXW];
    const int ntl = a.g.ntx * a.g.ntz;
    const int w = xcd_id(ntl * a.nshots);
    const int shot = w / ntl, tile = w - shot * ntl;
    const int tz = tile / a.g.ntx, tx = tile - tz * a.g.ntx;
    if (near_edge(a.g, tx * TX, tz * TZ)) fwd_tile<true, SNAP, REC>(a, su, qx, tile, shot);
    else                                  fwd_tile<false, SNAP, REC>(a, su, qx, tile, shot);
}

// ------------------------------------------------------------------ adjoint
// Gradient per node: khat at a half node feeds its two nodes with weight
// 1/2 each, so dJ/dchat_i = 1/2 (p at i-1/2 + p at i+1/2) per axis, with
// p = qb S' the half-node product; the node at the far edge of each axis
// also takes the other half of its right half node (the chat beyond the
// grid is its replica).  The x product of the half node left of a thread's
// node comes from the neighbouring lane (lane 0: from the extra column).
template <bool NEAR, bool GRAD>
__device__ __forceinline__ float adj_xflux(const Ad2AdjArgs &a, const float *hx, long long so, int x0, int z0, int r,
                                           int h, float c0, float c1, bool want_p, float &p)
{
    const Grid2 &g = a.g;
    const int iz = z0 + r, ix = x0 - 2 + h;
    const float *s = hx + (r + AH) * AW + h;
    const float qb = -d4(s[0], s[1], s[2], s[3]);
    float Gb = 0.f;
    p = 0.f;
    if (!NEAR || (ix >= 0 && ix < g.NX)) {
        const long long f = fr(g, iz, ix);
        const bool own = h >= 2 && h < TX + 2 && iz < g.NZ;
        const float Sb = 0.5f * (c0 + c1) * qb;
        Gb = Sb;
        if constexpr (NEAR) {
            const float z = fmaf(a.t.ahx[ix], Sb, a.t.bhx[ix] * a.zx[so + f]);
            Gb = Sb + z;
            if (own) a.zxn[so + f] = z;
        }
        if constexpr (GRAD) {
            if (want_p && iz < g.NZ) p = qb * a.snx[so + f];
        }
    }
    return Gb;
}

template <bool NEAR, bool GRAD>
__device__ __forceinline__ void adj_tile(const Ad2AdjArgs &a, float *hx, float *hz, float *qx, float *pl, int tile,
                                         int shot)
{
    const Grid2 &g = a.g;
    const int tz = tile / g.ntx, tx = tile - tz * g.ntx;
    const int x0 = tx * TX, z0 = tz * TZ;
    const long long so = (long long)shot * g.plane;
    const float *l1 = a.l1 + so;
    const float *ch = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const int tid = threadIdx.x, lx = tid % TX, ly = __builtin_amdgcn_readfirstlane(tid / TX), r0 = ly * RPA, ix = x0 + lx;

    // Hb = lambda^{k+1} + Y^{k+1} per axis on the tile and its halo
    if constexpr (!NEAR) {
        // away from the layer the x and z arrays are both lambda^{k+1} itself:
        // straight from global memory into LDS (4 bytes per lane and load,
        // item order = the row-major order of hx; every cell inside the frame)
        constexpr int NV = AR * AW, K = (NV + NTA - 1) / NTA;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = tid + k * NTA;
            if (i < NV) {
                const int r = i / AW, c = i - r * AW;
                __builtin_amdgcn_global_load_lds((const void *)(l1 + fr(g, z0 - AH + r, x0 - AH + c)),
                                                 (void __attribute__((address_space(3))) *)(hx + k * NTA + (tid & ~63)),
                                                 4, 0, 0);
            }
        }
    }
    for (int i = tid; NEAR && i < AR * AW; i += NTA) {
        const int r = i / AW, c = i - r * AW;
        const int iz = z0 - AH + r, jx = x0 - AH + c;
        const long long f = fr(g, iz, jx);
        const float l = l1[f];
        if constexpr (NEAR) {
            float bx = l, bz = l;
            if (iz >= 0 && iz < g.NZ && jx >= 0 && jx < g.NX) {
                const float yx = fmaf(a.t.a0x[jx], l, a.t.b0x[jx] * a.yx[so + f]);
                const float yz = fmaf(a.t.a0z[iz], l, a.t.b0z[iz] * a.yz[so + f]);
                if (r >= AH && r < AH + TZ && c >= AH && c < AH + TX) {
                    a.yxn[so + f] = yx;
                    a.yzn[so + f] = yz;
                }
                bx = l + yx;
                bz = l + yz;
            }
            hx[i] = bx;
            hz[i] = bz;
        }
    }
    float cz[RPA + 4];
#pragma unroll
    for (int m = 0; m < RPA + 4; ++m) cz[m] = ch[fr(g, z0 + r0 - 2 + m, ix)];
    float l2[RPA];                        // lambda^{k+2} of the own rows, loaded early
#pragma unroll
    for (int j = 0; j < RPA; ++j) l2[j] = __builtin_nontemporal_load(a.l2 + so + fr(g, z0 + r0 + j, ix));
    float gacc[RPA];                      // the gradient accumulator of the own rows, loaded early
    if constexpr (GRAD) {
#pragma unroll
        for (int j = 0; j < RPA; ++j) {
            const int iz = z0 + r0 + j;
            gacc[j] = iz < g.NZ && ix < g.NX ? __builtin_nontemporal_load(a.gn + so + fr(g, iz, ix)) : 0.f;
        }
    }
    if constexpr (!NEAR) __builtin_amdgcn_s_waitcnt(0);   // the tile's direct loads have landed in LDS
    __syncthreads();
    const float *hzz = NEAR ? hz : hx;

    float lam[RPA], dz[RPA], gnz[RPA];   // lambda^{k+1}, Dm' Gb_z and the z gradient of the own rows
    {
        float hc[RPA + 6];
#pragma unroll
        for (int m = 0; m < RPA + 6; ++m) hc[m] = hzz[(r0 + m) * AW + lx + AH];
        float gz[RPA + 3], pz[RPA + 3];
#pragma unroll
        for (int m = 0; m < RPA + 3; ++m) {
            const int iz = z0 + r0 - 2 + m;
            const float qb = -d4(hc[m], hc[m + 1], hc[m + 2], hc[m + 3]);
            float Gb = 0.f;
            pz[m] = 0.f;
            if (!NEAR || (iz >= 0 && iz < g.NZ)) {
                const long long f = fr(g, iz, ix);
                const bool own = m >= 2 && m < RPA + 2 && ix < g.NX;
                const float Sb = 0.5f * (cz[m] + cz[m + 1]) * qb;
                Gb = Sb;
                if constexpr (NEAR) {
                    const float z = fmaf(a.t.ahz[iz], Sb, a.t.bhz[iz] * a.zz[so + f]);
                    Gb = Sb + z;
                    if (own) a.zzn[so + f] = z;
                }
                if constexpr (GRAD) {
                    if (m >= 1 && m < RPA + 2) pz[m] = qb * a.snz[so + f];
                }
            }
            gz[m] = Gb;
        }
#pragma unroll
        for (int j = 0; j < RPA; ++j) {
            const int iz = z0 + r0 + j;
            lam[j] = NEAR ? 0.f : hc[j + 3];
            dz[j] = d4(gz[j], gz[j + 1], gz[j + 2], gz[j + 3]);
            gnz[j] = 0.5f * (pz[j + 1] + pz[j + 2]);
            if (iz == g.NZ - 1) gnz[j] += 0.5f * pz[j + 2];
        }
    }
    float px[RPA];                        // x products at the own half column
#pragma unroll
    for (int j = 0; j < RPA; ++j) {
        const float c0 = cz[j + 2];
        float c1 = __shfl_down(c0, 1, TX);
        if (lx == TX - 1) c1 = ch[fr(g, z0 + r0 + j, ix + 1)];
        float pj;
        qx[(r0 + j) * QXW + lx + 2] = adj_xflux<NEAR, GRAD>(a, hx, so, x0, z0, r0 + j, lx + 2, c0, c1, true, pj);
        px[j] = pj;
    }
    if (tid < 3 * TZ) {
        const int r = tid / 3, e = tid - 3 * r, h = e == 2 ? TX + 2 : e;
        const long long f = fr(g, z0 + r, x0 - 2 + h);
        float p = 0.f;
        qx[r * QXW + h] = adj_xflux<NEAR, GRAD>(a, hx, so, x0, z0, r, h, ch[f], ch[f + 1], h == 1, p);
        if (GRAD && h == 1) pl[r] = p;    // the half node left of the tile's first column
    }
    __syncthreads();                      // qx, pl complete; hx, hz no longer read

    const int ntiles = g.ntx * g.ntz;
    const int *off = a.rec_off + (long long)shot * (ntiles + 1);
    const int b = off[tile], e = off[tile + 1];
    const bool inj = a.k >= 1 && b < e;   // uniform over the block
    if (inj) {
        const float *d = a.dJdd + ((long long)shot * a.nt + (a.k - 1)) * a.nrec;
        gather_entries(hx, a.rec_ent, b, e, [](int en) { return rec_cell(en); },
                       [&](int en) { return d[rec_id(en)]; });
    }
#pragma unroll
    for (int j = 0; j < RPA; ++j) {
        const int r = r0 + j, iz = z0 + r;
        const float *ga = qx + r * QXW + lx;
        const float Dx = d4(ga[0], ga[1], ga[2], ga[3]);
        float gn = 0.f;
        if constexpr (GRAD) {
            float left = __shfl_up(px[j], 1, TX);
            if (lx == 0) left = pl[r];
            gn = 0.5f * (left + px[j]) + gnz[j];
            if (ix == g.NX - 1) gn += 0.5f * px[j];
        }
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fr(g, iz, ix);
            const float lc = NEAR ? l1[f] : lam[j];
            float v = lc + ((lc - l2[j]) - (Dx + dz[j]));
            if (inj) v += hx[r * TX + lx];
            __builtin_nontemporal_store(v, a.l0 + so + f);
            if constexpr (GRAD) __builtin_nontemporal_store(gacc[j] + gn, a.gn + so + f);
        }
    }
}

template <bool GRAD>
__global__ __launch_bounds__(NTA) __attribute__((amdgpu_waves_per_eu(8))) void ad2_adj_kernel(Ad2AdjArgs a)
{
    __shared__ float hx[AR * AW];
    __shared__ float hz[AR * AW];
    __shared__ float qx[TZ * QXW];
    __shared__ float pl[TZ];
    const int ntl = a.g.ntx * a.g.ntz;
    const int w = xcd_id(ntl * a.nshots);
    const int shot = w / ntl, tile = w - shot * ntl;
    const int tz = tile / a.g.ntx, tx = tile - tz * a.g.ntx;
    if (near_edge(a.g, tx * TX, tz * TZ)) adj_tile<true, GRAD>(a, hx, hz, qx, pl, tile, shot);
    else                                  adj_tile<false, GRAD>(a, hx, hz, qx, pl, tile, shot);
}

// ------------------------------------------------------------------ model and gradient
__global__ void ad2_prep_kernel(Grid2 g, int nmodels, const float *vp, double dt, double dx, float *chat, float *cpad)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        const int iz = (int)(f / g.SX) - OZ, ix = (int)(f - (f / g.SX) * g.SX) - OX;
        const bool in = iz >= 0 && iz < g.NZ && ix >= 0 && ix < g.NX;
        const bool rep = (ix == g.NX && iz >= 0 && iz < g.NZ) || (iz == g.NZ && ix >= 0 && ix < g.NX);
        float c = 0.f, ch = 0.f;
        if (in || rep) {
            const int pz = min(max(min(iz, g.NZ - 1) - g.P, 0), g.nz - 1);
            const int px = min(max(min(ix, g.NX - 1) - g.P, 0), g.nx - 1);
            c = vp[(m * g.nz + pz) * g.nx + px];
            const double cd = c;
            ch = (float)(dt * dt * cd * cd / (dx * dx));
        }
        chat[i] = ch;
        cpad[i] = in ? c : 0.f;
    }
}

// dJ/dchat per padded node, summed over the model's shots in shot order.
__global__ void ad2_sum_shots_kernel(Grid2 g, int nmodels, int spm, const float *gn, float *acc)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        float v = 0.f;
        for (int s = 0; s < spm; ++s) v += gn[(m * spm + s) * g.plane + f];
        acc[i] = v;
    }
}

// dJ/dc per physical cell: the padded nodes replicating it, times
// dchat/dc = 2 dt^2 c / dx^2.
__global__ void ad2_fold_kernel(Grid2 g, int nmodels, const float *acc, const float *cpad, double dt, double dx,
                                float *g_vp)
{
    const long long n = (long long)nmodels * g.nz * g.nx;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / ((long long)g.nz * g.nx);
        const long long rem = i - m * g.nz * g.nx;
        const int iz = (int)(rem / g.nx), ix = (int)(rem - (long long)iz * g.nx);
        const int zlo = iz == 0 ? 0 : iz + g.P, zhi = iz == g.nz - 1 ? g.NZ - 1 : iz + g.P;
        const int xlo = ix == 0 ? 0 : ix + g.P, xhi = ix == g.nx - 1 ? g.NX - 1 : ix + g.P;
        const float *am = acc + m * g.plane;
        float v = 0.f;
        for (int pz = zlo; pz <= zhi; ++pz)
            for (int px = xlo; px <= xhi; ++px) v += am[fr(g, pz, px)];
        const double c = cpad[m * g.plane + fr(g, iz + g.P, ix + g.P)];
        g_vp[i] = (float)(2.0 * dt * dt * c / (dx * dx)) * v;
    }
}

int blocks_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 65536); }

} // namespace

void launch_ad2_fwd(const Ad2FwdArgs &a, hipStream_t s)
{
    const int n = a.g.ntx * a.g.ntz * a.nshots;
    const bool rec = a.seis && a.nrec > 0;
    if (a.snx) {
        if (rec) ad2_fwd_kernel<true, true><<<n, NTA, 0, s>>>(a);
        else     ad2_fwd_kernel<true, false><<<n, NTA, 0, s>>>(a);
    } else {
        if (rec) ad2_fwd_kernel<false, true><<<n, NTA, 0, s>>>(a);
        else     ad2_fwd_kernel<false, false><<<n, NTA, 0, s>>>(a);
    }
}

void launch_ad2_adj(const Ad2AdjArgs &a, hipStream_t s)
{
    const int n = a.g.ntx * a.g.ntz * a.nshots;
    if (a.snx) ad2_adj_kernel<true><<<n, NTA, 0, s>>>(a);
    else       ad2_adj_kernel<false><<<n, NTA, 0, s>>>(a);
}

void launch_ad2_prep(const Grid2 &g, int nmodels, const float *vp, double dt, double dx, float *chat, float *cpad,
                     hipStream_t s)
{
    ad2_prep_kernel<<<blocks_for((long long)nmodels * g.plane), 256, 0, s>>>(g, nmodels, vp, dt, dx, chat, cpad);
}

void launch_ad2_finalize(const Grid2 &g, int nmodels, int spm, const float *gn, float *acc, const float *cpad,
                         double dt, double dx, float *g_vp, hipStream_t s)
{
    ad2_sum_shots_kernel<<<blocks_for((long long)nmodels * g.plane), 256, 0, s>>>(g, nmodels, spm, gn, acc);
    ad2_fold_kernel<<<blocks_for((long long)nmodels * g.nz * g.nx), 256, 0, s>>>(g, nmodels, acc, cpad, dt, dx, g_vp);
}

} // namespace sg
