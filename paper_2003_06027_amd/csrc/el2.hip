// el2.hip -- gfx950 kernels of the 2-D elastic velocity-stress scheme
// (paper: Implementation, Eq. (13), with the explicit recursion Eq. (1)) and
// its exact adjoint (Eqs. (4)-(5)), gradients with respect to vp, vs, rho.
//
// Staggered grid, all fields [iz][ix] on the padded grid, the index naming
// the node below-left of the field's position: sxx, szz at (ix, iz); vx at
// (ix+1/2, iz); vz at (ix, iz+1/2); sxz at (ix+1/2, iz+1/2).  4th-order
// staggered differences without the 1/dx factor (kap = dt/dx carries it):
//     Dp f[i] = 9/8 (f[i+1] - f[i]) - 1/24 (f[i+2] - f[i-1])
//     Dm f[i] = 9/8 (f[i] - f[i-1]) - 1/24 (f[i+1] - f[i-2])
// zero beyond the padded grid, so Dm^T = -Dp.  Forward step n:
//   velocity:  m = b m + a D(sigma) on the CPML cells, then
//     vx += kap bx (Dxp sxx + Dzm sxz + m_sxx_x + m_sxz_z)
//     vz += kap bz (Dxm sxz + Dzp szz + m_sxz_x + m_szz_z)
//   stress:    m = b m + a D(v), Exx = Dxm vx + m, Ezz = Dzm vz + m,
//     Exz = Dzp vx + m + Dxp vz + m
//     sxx += kap ((lam+2mu) Exx + lam Ezz), szz += kap (lam Exx + (lam+2mu) Ezz),
//     sxz += kap muxz Exz, plus dt M r(t_n)/(dx dz) at the source node.
// Adjoint step n (reverse): pass 1 forms the adjoints e1..e4 of the four
// velocity differences from the stress adjoints (and the lam/mu/muxz
// gradients from the stored strains); pass 2 applies their transposes to the
// velocity adjoints, then forms the adjoints d1..d4 of the stress
// differences (and the bx/bz gradients from the stored divergences); pass 3
// applies those transposes to the stress adjoints.
// Cache policy: the snapshots, the gradient accumulators and the adjoint CPML
// memories, which only their own cell touches, are loaded and stored
// non-temporally; the fields that the stencils share stay cached.  (The
// forward CPML memories stay cached: streaming them slowed the forward.)
#include "el2_internal.h"

namespace sg {
namespace {

constexpr float C1 = (float)(9.0 / 8.0);
constexpr float C2 = (float)(-1.0 / 24.0);
// Cell blocks of 256 threads, EBX x (256 / EBX) cells: 32 x 8 in both
// passes, the forward's in XCD order, the adjoint's in the hardware order
// (they ran slower in XCD order with every block shape). Each is the
// measured best of 16 x 16 (forward), 32 x 8, 64 x 4, 128 x 2 and 256 x 1.
constexpr bool XCD_FWD = true, XCD_ADJ = false;

__device__ __forceinline__ float Dp(const float *f, long long i, long long s)
{
    return C1 * (f[i + s] - f[i]) + C2 * (f[i + 2 * s] - f[i - s]);
}
__device__ __forceinline__ float Dm(const float *f, long long i, long long s)
{
    return C1 * (f[i] - f[i - s]) + C2 * (f[i + s] - f[i - 2 * s]);
}

// gradient accumulator += v, streamed (non-temporal): read and written once per step
__device__ __forceinline__ void gacc(float *p, float v)
{
    __builtin_nontemporal_store(__builtin_nontemporal_load(p) + v, p);
}

// Is (ix, iz) a CPML cell? (The cells that update memory variables; frame
// padding beyond the grid counts as layer when there is a layer.)
__device__ __forceinline__ bool in_layer(const Grid2 &g, int ix, int iz)
{
    return g.P > 0 && (ix < g.P || ix >= g.P + g.nx - 1 || iz < g.P || iz >= g.P + g.nz - 1);
}

// Staggered differences of a field that the adjoint passes store in two
// arrays: `lay` holds it on CPML cells, `inn` elsewhere, where it equals the
// field `inn` holds. Point k of the stencil along axis AX (0: x, 1: z) reads
// the array its cell belongs to.
template <int AX>
__device__ __forceinline__ float at_sel(const Grid2 &g, const float *lay, const float *inn, long long i, long long s,
                                        int ix, int iz, int k)
{
    const bool l = AX == 0 ? in_layer(g, ix + k, iz) : in_layer(g, ix, iz + k);
    return (l ? lay : inn)[i + k * s];
}
template <int AX>
__device__ __forceinline__ float Dp_sel(const Grid2 &g, const float *lay, const float *inn, long long i, long long s,
                                        int ix, int iz)
{
    return C1 * (at_sel<AX>(g, lay, inn, i, s, ix, iz, 1) - at_sel<AX>(g, lay, inn, i, s, ix, iz, 0)) +
           C2 * (at_sel<AX>(g, lay, inn, i, s, ix, iz, 2) - at_sel<AX>(g, lay, inn, i, s, ix, iz, -1));
}
template <int AX>
__device__ __forceinline__ float Dm_sel(const Grid2 &g, const float *lay, const float *inn, long long i, long long s,
                                        int ix, int iz)
{
    return C1 * (at_sel<AX>(g, lay, inn, i, s, ix, iz, 0) - at_sel<AX>(g, lay, inn, i, s, ix, iz, -1)) +
           C2 * (at_sel<AX>(g, lay, inn, i, s, ix, iz, 1) - at_sel<AX>(g, lay, inn, i, s, ix, iz, -2));
}

struct Cell {
    int ix, iz, shot;
    bool valid, layer;
    long long f, so, mo;   // frame index, shot and model offsets
};

// Work id of this workgroup with consecutive ids on one XCD: the hardware
// hands workgroups to the 8 XCDs round-robin, so id b runs on XCD b % 8; the
// remap gives each XCD a contiguous range of (block, shot) work, so the rows
// that a block's z stencil shares with the blocks above and below it are
// fetched into one L2.
__device__ __forceinline__ int xcd_work_id(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, j = b / NXCD;
    return x * per + min(x, rem) + j;
}

// Cell of this thread in a grid of EBX x (256 / EBX) cell blocks. XCD =
// true: a 1-D grid over (block, shot) taken in xcd_work_id order; false: a
// 2-D grid, blockIdx.y the shot.
template <int EBX, bool XCD>
__device__ __forceinline__ Cell cell_of(const Grid2 &g, int spm)
{
    constexpr int EBZ = 256 / EBX;
    Cell c;
    const int ntxe = (g.NX + EBX - 1) / EBX, nblk = ntxe * ((g.NZ + EBZ - 1) / EBZ);
    int r;
    if (XCD) {
        const int w = xcd_work_id((int)gridDim.x);
        c.shot = w / nblk;
        r = w - c.shot * nblk;
    } else {
        c.shot = blockIdx.y;
        r = blockIdx.x;
    }
    const int bz = r / ntxe, bx = r - bz * ntxe;
    c.ix = bx * EBX + (int)(threadIdx.x % EBX);
    c.iz = bz * EBZ + (int)(threadIdx.x / EBX);
    c.valid = c.ix < g.NX && c.iz < g.NZ;
    c.layer = in_layer(g, c.ix, c.iz);
    c.f = (long long)(c.iz + OZ) * g.SX + c.ix + OX;
    c.so = (long long)c.shot * g.plane;
    c.mo = (long long)(c.shot / spm) * g.plane;
    return c;
}

template <int EBX, bool XCD>
dim3 cell_grid(const Grid2 &g, int nshots)
{
    constexpr int EBZ = 256 / EBX;
    const int nblk = ((g.NX + EBX - 1) / EBX) * ((g.NZ + EBZ - 1) / EBZ);
    return XCD ? dim3(nblk * nshots) : dim3(nblk, nshots);
}

// Shots per thread in the step passes: the shots of a group belong to one
// model, so a thread reads the model fields once per group. The adjoint
// passes that accumulate gradients also add the group's summed contribution
// to one accumulator slot per group (slots [group][plane]), where one slot
// per shot would cost a read and a write of each accumulator per shot.

template <int GSH, int EBX>
__global__ __launch_bounds__(256) void el2_vel_kernel(El2Args a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_FWD>(g, a.shots_per_model / GSH);   // c.shot: the group
    if (!c.valid) return;
    const long long SX = g.SX;
    const float kbx = a.kap * a.m[M_BX][c.mo + c.f], kbz = a.kap * a.m[M_BZ][c.mo + c.f];
#pragma unroll
    for (int j = 0; j < GSH; ++j) {
        const long long f = (long long)(c.shot * GSH + j) * g.plane + c.f;
        float d1 = Dp(a.f[E_SXX], f, 1), d2 = Dm(a.f[E_SXZ], f, SX);
        float d3 = Dm(a.f[E_SXZ], f, 1), d4 = Dp(a.f[E_SZZ], f, SX);
        if (c.layer) {
            float m;
            m = a.t.bx[1][c.ix] * a.f[E_MSXXX][f] + a.t.ax[1][c.ix] * d1; a.f[E_MSXXX][f] = m; d1 += m;
            m = a.t.bz[0][c.iz] * a.f[E_MSXZZ][f] + a.t.az[0][c.iz] * d2; a.f[E_MSXZZ][f] = m; d2 += m;
            m = a.t.bx[0][c.ix] * a.f[E_MSXZX][f] + a.t.ax[0][c.ix] * d3; a.f[E_MSXZX][f] = m; d3 += m;
            m = a.t.bz[1][c.iz] * a.f[E_MSZZZ][f] + a.t.az[1][c.iz] * d4; a.f[E_MSZZZ][f] = m; d4 += m;
        }
        const float fx = d1 + d2, fz = d3 + d4;
        a.f[E_VX][f] += kbx * fx;
        a.f[E_VZ][f] += kbz * fz;
        if (a.snap) {
            __builtin_nontemporal_store(fx, a.snap + 3 * a.snap_stride + f);
            __builtin_nontemporal_store(fz, a.snap + 4 * a.snap_stride + f);
        }
    }
}

template <int GSH, int EBX>
__global__ __launch_bounds__(256) void el2_str_kernel(El2Args a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_FWD>(g, a.shots_per_model / GSH);   // c.shot: the group
    if (!c.valid) return;
    const long long SX = g.SX;
    const float lam = a.m[M_LAM][c.mo + c.f], mu = a.m[M_MU][c.mo + c.f], muxz = a.m[M_MUXZ][c.mo + c.f];
#pragma unroll
    for (int j = 0; j < GSH; ++j) {
        const int shot = c.shot * GSH + j;
        const long long f = (long long)shot * g.plane + c.f;
        float e1 = Dm(a.f[E_VX], f, 1), e2 = Dm(a.f[E_VZ], f, SX);
        float e3 = Dp(a.f[E_VX], f, SX), e4 = Dp(a.f[E_VZ], f, 1);
        if (c.layer) {
            float m;
            m = a.t.bx[0][c.ix] * a.f[E_MVXX][f] + a.t.ax[0][c.ix] * e1; a.f[E_MVXX][f] = m; e1 += m;
            m = a.t.bz[0][c.iz] * a.f[E_MVZZ][f] + a.t.az[0][c.iz] * e2; a.f[E_MVZZ][f] = m; e2 += m;
            m = a.t.bz[1][c.iz] * a.f[E_MVXZ][f] + a.t.az[1][c.iz] * e3; a.f[E_MVXZ][f] = m; e3 += m;
            m = a.t.bx[1][c.ix] * a.f[E_MVZX][f] + a.t.ax[1][c.ix] * e4; a.f[E_MVZX][f] = m; e4 += m;
        }
        const float exz = e3 + e4;
        float sxx = a.f[E_SXX][f] + a.kap * ((lam + 2.f * mu) * e1 + lam * e2);
        float szz = a.f[E_SZZ][f] + a.kap * (lam * e1 + (lam + 2.f * mu) * e2);
        float sxz = a.f[E_SXZ][f] + a.kap * muxz * exz;
        if (c.f == a.src_f[shot]) {
            const float s = a.src_scale * a.wav[(long long)shot * a.nt + a.k];
            sxx += s * a.mt[3 * shot];
            szz += s * a.mt[3 * shot + 1];
            sxz += s * a.mt[3 * shot + 2];
        }
        a.f[E_SXX][f] = sxx;
        a.f[E_SZZ][f] = szz;
        a.f[E_SXZ][f] = sxz;
        if (a.snap) {
            __builtin_nontemporal_store(e1, a.snap + f);
            __builtin_nontemporal_store(e2, a.snap + a.snap_stride + f);
            __builtin_nontemporal_store(exz, a.snap + 2 * a.snap_stride + f);
        }
    }
}

__global__ void el2_record_kernel(El2RecArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nshots * a.nrec) return;
    const int shot = i / a.nrec, r = i - shot * a.nrec;
    const long long f = (long long)shot * a.plane + a.rec_f[i];
    a.seis[((long long)(shot * 2) * a.nt + a.k) * a.nrec + r] = a.vx[f];
    a.seis[((long long)(shot * 2 + 1) * a.nt + a.k) * a.nrec + r] = a.vz[f];
}

// R^T dJ/dd of sample k into the velocity adjoints: one thread per unique
// receiver cell, summing its receivers in a fixed order.
__global__ void el2_inject_kernel(El2RecArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nshots * a.nuniq_max) return;
    const int shot = i / a.nuniq_max, u = i - shot * a.nuniq_max;
    const int *off = a.uoff + (long long)shot * (a.nuniq_max + 1);
    const int b = off[u], e = off[u + 1];
    if (b >= e) return;
    const float *dx = a.dJdd + ((long long)(shot * 2) * a.nt + a.k) * a.nrec;
    const float *dz = a.dJdd + ((long long)(shot * 2 + 1) * a.nt + a.k) * a.nrec;
    float sx = 0.f, sz = 0.f;
    for (int j = b; j < e; ++j) {
        sx += dx[a.uid[j]];
        sz += dz[a.uid[j]];
    }
    const long long f = (long long)shot * a.plane + a.rec_f[(long long)shot * a.nrec + a.uid[b]];
    a.ax[f] += sx;
    a.az[f] += sz;
}


// Pass 1 at one cell of one shot, from its stress adjoints sxx, szz, sxz:
// the adjoints e1..e4 of the velocity differences (with the CPML memories),
// the lam/mu/muxz gradient terms (added to g0..g2) and the source gradient.
__device__ __forceinline__ void adj1_cell(const El2AdjArgs &a, const Cell &c, int shot, long long f, float sxx,
                                          float szz, float sxz, float lam, float mu, float muxz, float &g0,
                                          float &g1, float &g2)
{
    {
        const float txx = a.kap * ((lam + 2.f * mu) * sxx + lam * szz);
        const float tzz = a.kap * (lam * sxx + (lam + 2.f * mu) * szz);
        const float txz = a.kap * muxz * sxz;
        const float exx = __builtin_nontemporal_load(a.snap + f),
                    ezz = __builtin_nontemporal_load(a.snap + a.snap_stride + f),
                    exz = __builtin_nontemporal_load(a.snap + 2 * a.snap_stride + f);
        g0 += a.kap * (exx + ezz) * (sxx + szz);
        g1 += 2.f * a.kap * (exx * sxx + ezz * szz);
        g2 += a.kap * exz * sxz;
        float e1 = txx, e2 = tzz, e3 = txz, e4 = txz;
        if (c.layer) {
            float q;
            q = txx + __builtin_nontemporal_load(a.a[E_MVXX] + f); __builtin_nontemporal_store(a.t.bx[0][c.ix] * q, a.a[E_MVXX] + f); e1 = txx + a.t.ax[0][c.ix] * q;
            q = tzz + __builtin_nontemporal_load(a.a[E_MVZZ] + f); __builtin_nontemporal_store(a.t.bz[0][c.iz] * q, a.a[E_MVZZ] + f); e2 = tzz + a.t.az[0][c.iz] * q;
            q = txz + __builtin_nontemporal_load(a.a[E_MVXZ] + f); __builtin_nontemporal_store(a.t.bz[1][c.iz] * q, a.a[E_MVXZ] + f); e3 = txz + a.t.az[1][c.iz] * q;
            q = txz + __builtin_nontemporal_load(a.a[E_MVZX] + f); __builtin_nontemporal_store(a.t.bx[1][c.ix] * q, a.a[E_MVZX] + f); e4 = txz + a.t.ax[1][c.ix] * q;
        }
        a.tmp[0][f] = e1;
        a.tmp[1][f] = e2;
        a.tmp[2][f] = e3;
        if (c.layer) a.tmp[3][f] = e4;   // e4 = e3 off the layer
        if (a.gwav && c.f == a.src_f[shot])
            a.gwav[(long long)shot * a.nt + a.k] =
                a.src_scale * (a.mt[3 * shot] * sxx + a.mt[3 * shot + 1] * szz + a.mt[3 * shot + 2] * sxz);
    }
}

// Pass 3 at one cell of one shot: the stress adjoints minus the transposed
// differences of d1..d4; returns them through sxx, szz, sxz (stored).
__device__ __forceinline__ void adj3_cell(const El2AdjArgs &a, const Grid2 &g, long long f, int ix, int iz,
                                          float &sxx, float &szz, float &sxz)
{
    const long long SX = g.SX;
    sxx = a.a[E_SXX][f] - Dm(a.tmp[4], f, 1);
    sxz = a.a[E_SXZ][f] - (Dp_sel<1>(g, a.tmp[5], a.tmp[4], f, SX, ix, iz) + Dp(a.tmp[6], f, 1));
    szz = a.a[E_SZZ][f] - Dm_sel<1>(g, a.tmp[7], a.tmp[6], f, SX, ix, iz);
    a.a[E_SXX][f] = sxx;
    a.a[E_SXZ][f] = sxz;
    a.a[E_SZZ][f] = szz;
}

template <int GSH, int EBX>
__global__ __launch_bounds__(256) void el2_adj1_kernel(El2AdjArgs a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_ADJ>(g, a.shots_per_model / GSH);   // c.shot: the group
    if (!c.valid) return;
    const float lam = a.m[M_LAM][c.mo + c.f], mu = a.m[M_MU][c.mo + c.f], muxz = a.m[M_MUXZ][c.mo + c.f];
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int j = 0; j < GSH; ++j) {
        const int shot = c.shot * GSH + j;
        const long long f = (long long)shot * g.plane + c.f;
        adj1_cell(a, c, shot, f, a.a[E_SXX][f], a.a[E_SZZ][f], a.a[E_SXZ][f], lam, mu, muxz, g0, g1, g2);
    }
    const long long gf = c.so + c.f;
    gacc(a.grad + gf, g0);
    gacc(a.grad + a.grad_stride + gf, g1);
    gacc(a.grad + 2 * a.grad_stride + gf, g2);
}

// Pass 3 of step k and pass 1 of step k - 1 in one launch (a: the arguments
// of step k - 1): pass 1 reads the stress adjoints of its own cell only,
// which pass 3 has just formed there, so one read and write of them serve
// both.
template <int GSH, int EBX>
__global__ __launch_bounds__(256) void el2_adj31_kernel(El2AdjArgs a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_ADJ>(g, a.shots_per_model / GSH);   // c.shot: the group
    if (!c.valid) return;
    const float lam = a.m[M_LAM][c.mo + c.f], mu = a.m[M_MU][c.mo + c.f], muxz = a.m[M_MUXZ][c.mo + c.f];
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int j = 0; j < GSH; ++j) {
        const int shot = c.shot * GSH + j;
        const long long f = (long long)shot * g.plane + c.f;
        float sxx, szz, sxz;
        adj3_cell(a, g, f, c.ix, c.iz, sxx, szz, sxz);
        adj1_cell(a, c, shot, f, sxx, szz, sxz, lam, mu, muxz, g0, g1, g2);
    }
    const long long gf = c.so + c.f;
    gacc(a.grad + gf, g0);
    gacc(a.grad + a.grad_stride + gf, g1);
    gacc(a.grad + 2 * a.grad_stride + gf, g2);
}

template <int GSH, int EBX>
__global__ __launch_bounds__(256) void el2_adj2_kernel(El2AdjArgs a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_ADJ>(g, a.shots_per_model / GSH);   // c.shot: the group
    if (!c.valid) return;
    const long long SX = g.SX;
    const float bxm = a.m[M_BX][c.mo + c.f], bzm = a.m[M_BZ][c.mo + c.f];
    float g3 = 0.f, g4 = 0.f;
#pragma unroll
    for (int j = 0; j < GSH; ++j) {
        const long long f = (long long)(c.shot * GSH + j) * g.plane + c.f;
        // transposes of the velocity differences: Dm^T = -Dp, Dp^T = -Dm
        const float vx = a.a[E_VX][f] - (Dp(a.tmp[0], f, 1) + Dm(a.tmp[2], f, SX));
        const float vz = a.a[E_VZ][f] - (Dp(a.tmp[1], f, SX) + Dm_sel<0>(g, a.tmp[3], a.tmp[2], f, 1, c.ix, c.iz));
        a.a[E_VX][f] = vx;
        a.a[E_VZ][f] = vz;
        const float fxb = a.kap * bxm * vx;
        const float fzb = a.kap * bzm * vz;
        g3 += a.kap * __builtin_nontemporal_load(a.snap + 3 * a.snap_stride + f) * vx;
        g4 += a.kap * __builtin_nontemporal_load(a.snap + 4 * a.snap_stride + f) * vz;
        float d1 = fxb, d2 = fxb, d3 = fzb, d4 = fzb;
        if (c.layer) {
            float q;
            q = fxb + __builtin_nontemporal_load(a.a[E_MSXXX] + f); __builtin_nontemporal_store(a.t.bx[1][c.ix] * q, a.a[E_MSXXX] + f); d1 = fxb + a.t.ax[1][c.ix] * q;
            q = fxb + __builtin_nontemporal_load(a.a[E_MSXZZ] + f); __builtin_nontemporal_store(a.t.bz[0][c.iz] * q, a.a[E_MSXZZ] + f); d2 = fxb + a.t.az[0][c.iz] * q;
            q = fzb + __builtin_nontemporal_load(a.a[E_MSXZX] + f); __builtin_nontemporal_store(a.t.bx[0][c.ix] * q, a.a[E_MSXZX] + f); d3 = fzb + a.t.ax[0][c.ix] * q;
            q = fzb + __builtin_nontemporal_load(a.a[E_MSZZZ] + f); __builtin_nontemporal_store(a.t.bz[1][c.iz] * q, a.a[E_MSZZZ] + f); d4 = fzb + a.t.az[1][c.iz] * q;
        }
        a.tmp[4][f] = d1;
        a.tmp[6][f] = d3;
        if (c.layer) {   // d2 = d1 and d4 = d3 off the layer
            a.tmp[5][f] = d2;
            a.tmp[7][f] = d4;
        }
    }
    const long long gf = c.so + c.f;
    gacc(a.grad + 3 * a.grad_stride + gf, g3);
    gacc(a.grad + 4 * a.grad_stride + gf, g4);
}

template <int EBX>
__global__ __launch_bounds__(256) void el2_adj3_kernel(El2AdjArgs a)
{
    const Grid2 &g = a.g;
    const Cell c = cell_of<EBX, XCD_ADJ>(g, a.shots_per_model);
    if (!c.valid) return;
    float sxx, szz, sxz;
    adj3_cell(a, g, c.so + c.f, c.ix, c.iz, sxx, szz, sxz);
}

// Model fields on the frame (FP64 arithmetic, rounded once) and padded
// copies of vp, vs, rho for the chain rule.
__global__ void el2_prep_kernel(Grid2 g, int nmodels, const float *vp, const float *vs, const float *rho,
                                float *lam, float *mu, float *muxz, float *bx, float *bz,
                                float *pvp, float *pvs, float *prho)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        const int fz = (int)(f / g.SX), fx = (int)(f - (long long)fz * g.SX);
        const int iz = fz - OZ, ix = fx - OX;
        float o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (iz >= 0 && iz < g.NZ && ix >= 0 && ix < g.NX) {
            auto at = [&](const float *p, int z, int x) -> double {
                z = min(max(z, 0), g.NZ - 1);
                x = min(max(x, 0), g.NX - 1);
                const int pz = min(max(z - g.P, 0), g.nz - 1), px = min(max(x - g.P, 0), g.nx - 1);
                return p[(m * g.nz + pz) * g.nx + px];
            };
            auto mu_at = [&](int z, int x) { const double b = at(vs, z, x); return at(rho, z, x) * b * b; };
            const double a = at(vp, iz, ix), b = at(vs, iz, ix), r = at(rho, iz, ix);
            o[0] = (float)(r * (a * a - 2.0 * b * b));
            o[1] = (float)(r * b * b);
            o[2] = (float)(4.0 / (1.0 / mu_at(iz, ix) + 1.0 / mu_at(iz, ix + 1) + 1.0 / mu_at(iz + 1, ix) +
                                  1.0 / mu_at(iz + 1, ix + 1)));
            o[3] = (float)(2.0 / (r + at(rho, iz, ix + 1)));
            o[4] = (float)(2.0 / (r + at(rho, iz + 1, ix)));
            o[5] = (float)a;
            o[6] = (float)b;
            o[7] = (float)r;
        }
        lam[i] = o[0]; mu[i] = o[1]; muxz[i] = o[2]; bx[i] = o[3]; bz[i] = o[4];
        pvp[i] = o[5]; pvs[i] = o[6]; prho[i] = o[7];
    }
}

// Sum of the accumulator slots (shot groups) of each model, in slot order.
__global__ void el2_sum_shots_kernel(Grid2 g, int nmodels, int slots, const float *grad, long long gs, float *acc)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        for (int q = 0; q < 5; ++q) {
            float v = 0.f;
            for (int s = 0; s < slots; ++s) v += grad[q * gs + (m * slots + s) * g.plane + f];
            acc[q * n + i] = v;
        }
    }
}

// Per padded cell: dJ/d(vp, vs, rho) of the padded model through
// lam = rho (vp^2 - 2 vs^2), mu = rho vs^2, the harmonic mu average and the
// arithmetic density averages (neighbours clamped to the padded grid, the
// clamped references counted with multiplicity).
__global__ void el2_chain_kernel(Grid2 g, int nmodels, const float *acc, const float *muxz,
                                 const float *mu, const float *bx, const float *bz,
                                 const float *pvp, const float *pvs, const float *prho, float *out)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        const int fz = (int)(f / g.SX), fx = (int)(f - (long long)fz * g.SX);
        const int iz = fz - OZ, ix = fx - OX;
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (iz >= 0 && iz < g.NZ && ix >= 0 && ix < g.NX) {
            const long long mb = m * g.plane;
            auto fr = [&](int z, int x) { return mb + (long long)(z + OZ) * g.SX + x + OX; };
            double glam = acc[i], gmu = acc[n + i], grho = 0.0;
            const double mui = mu[i];
            for (int dz = 0; dz <= 1; ++dz)
                for (int dx = 0; dx <= 1; ++dx) {
                    const int jz = iz - dz, jx = ix - dx;
                    if (jz < 0 || jx < 0) continue;
                    int cnt = 0;
                    for (int a2 = 0; a2 <= 1; ++a2)
                        for (int b2 = 0; b2 <= 1; ++b2)
                            cnt += (min(jz + a2, g.NZ - 1) == iz && min(jx + b2, g.NX - 1) == ix);
                    if (!cnt) continue;
                    const double mx = muxz[fr(jz, jx)];
                    gmu += cnt * acc[2 * n + fr(jz, jx)] * mx * mx / (4.0 * mui * mui);
                }
            for (int d = 0; d <= 1; ++d) {
                if (ix - d >= 0) {
                    const int cnt = (ix - d == ix) + (min(ix - d + 1, g.NX - 1) == ix);
                    const double b = bx[fr(iz, ix - d)];
                    grho += cnt * acc[3 * n + fr(iz, ix - d)] * (-0.5 * b * b);
                }
                if (iz - d >= 0) {
                    const int cnt = (iz - d == iz) + (min(iz - d + 1, g.NZ - 1) == iz);
                    const double b = bz[fr(iz - d, ix)];
                    grho += cnt * acc[4 * n + fr(iz - d, ix)] * (-0.5 * b * b);
                }
            }
            const double a = pvp[i], b = pvs[i], r = prho[i];
            r0 = (float)(glam * 2.0 * r * a);
            r1 = (float)(2.0 * r * b * (gmu - 2.0 * glam));
            r2 = (float)(grho + (a * a - 2.0 * b * b) * glam + b * b * gmu);
        }
        out[i] = r0;
        out[n + i] = r1;
        out[2 * n + i] = r2;
    }
}

__global__ void el2_fold_kernel(Grid2 g, int nmodels, const float *pad, float *g_vp, float *g_vs, float *g_rho)
{
    const long long np = (long long)nmodels * g.plane;
    const long long n = (long long)nmodels * g.nz * g.nx;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / ((long long)g.nz * g.nx);
        const long long rem = i - m * g.nz * g.nx;
        const int iz = (int)(rem / g.nx), ix = (int)(rem - (long long)iz * g.nx);
        const int zlo = iz == 0 ? 0 : iz + g.P, zhi = iz == g.nz - 1 ? g.NZ - 1 : iz + g.P;
        const int xlo = ix == 0 ? 0 : ix + g.P, xhi = ix == g.nx - 1 ? g.NX - 1 : ix + g.P;
        float v0 = 0.f, v1 = 0.f, v2 = 0.f;
        for (int pz = zlo; pz <= zhi; ++pz)
            for (int px = xlo; px <= xhi; ++px) {
                const long long q = m * g.plane + (long long)(pz + OZ) * g.SX + px + OX;
                v0 += pad[q];
                v1 += pad[np + q];
                v2 += pad[2 * np + q];
            }
        g_vp[i] = v0;
        g_vs[i] = v1;
        g_rho[i] = v2;
    }
}

int blocks_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 65536); }

} // namespace

// Launch kernel K<GSH, EBX> for the args' group size and block width.
#define EL2_DISPATCH(K, a, XCD, s)                                                                    \
    do {                                                                                              \
        const int gs_ = (a).gs, n_ = (a).nshots / gs_;                                                \
        if ((a).ebx == 64) {                                                                          \
            const dim3 grid_ = cell_grid<64, XCD>((a).g, n_);                                         \
            if (gs_ == 4) K<4, 64><<<grid_, 256, 0, s>>>(a);                                          \
            else if (gs_ == 2) K<2, 64><<<grid_, 256, 0, s>>>(a);                                     \
            else K<1, 64><<<grid_, 256, 0, s>>>(a);                                                   \
        } else {                                                                                      \
            const dim3 grid_ = cell_grid<32, XCD>((a).g, n_);                                         \
            if (gs_ == 4) K<4, 32><<<grid_, 256, 0, s>>>(a);                                          \
            else if (gs_ == 2) K<2, 32><<<grid_, 256, 0, s>>>(a);                                     \
            else K<1, 32><<<grid_, 256, 0, s>>>(a);                                                   \
        }                                                                                             \
    } while (0)

void launch_el2_vel(const El2Args &a, hipStream_t s) { EL2_DISPATCH(el2_vel_kernel, a, XCD_FWD, s); }
void launch_el2_str(const El2Args &a, hipStream_t s) { EL2_DISPATCH(el2_str_kernel, a, XCD_FWD, s); }
void launch_el2_adj1(const El2AdjArgs &a, hipStream_t s) { EL2_DISPATCH(el2_adj1_kernel, a, XCD_ADJ, s); }
void launch_el2_adj2(const El2AdjArgs &a, hipStream_t s) { EL2_DISPATCH(el2_adj2_kernel, a, XCD_ADJ, s); }
void launch_el2_adj31(const El2AdjArgs &a, hipStream_t s) { EL2_DISPATCH(el2_adj31_kernel, a, XCD_ADJ, s); }
void launch_el2_adj3(const El2AdjArgs &a, hipStream_t s)
{
    if (a.ebx == 64) el2_adj3_kernel<64><<<cell_grid<64, XCD_ADJ>(a.g, a.nshots), 256, 0, s>>>(a);
    else el2_adj3_kernel<32><<<cell_grid<32, XCD_ADJ>(a.g, a.nshots), 256, 0, s>>>(a);
}
#undef EL2_DISPATCH

void launch_el2_record(const El2RecArgs &a, hipStream_t s)
{
    const int n = a.nshots * a.nrec;
    if (n > 0) el2_record_kernel<<<(n + 255) / 256, 256, 0, s>>>(a);
}

void launch_el2_inject(const El2RecArgs &a, hipStream_t s)
{
    const int n = a.nshots * a.nuniq_max;
    if (n > 0) el2_inject_kernel<<<(n + 255) / 256, 256, 0, s>>>(a);
}

void launch_el2_prep(const Grid2 &g, int nmodels, const float *vp, const float *vs, const float *rho,
                     float *const *model, float *const *phys_pad, hipStream_t s)
{
    el2_prep_kernel<<<blocks_for((long long)nmodels * g.plane), 256, 0, s>>>(
        g, nmodels, vp, vs, rho, model[0], model[1], model[2], model[3], model[4], phys_pad[0], phys_pad[1],
        phys_pad[2]);
}

void launch_el2_finalize(const Grid2 &g, int nmodels, int spm, int gs, const float *grad, long long grad_stride,
                         float *acc, const float *const *model, const float *const *phys_pad,
                         float *g_vp, float *g_vs, float *g_rho, hipStream_t s)
{
    const long long n = (long long)nmodels * g.plane;
    float *pad = acc + 5 * n;
    // one accumulator slot per shot group
    el2_sum_shots_kernel<<<blocks_for(n), 256, 0, s>>>(g, nmodels, spm / gs, grad, grad_stride, acc);
    el2_chain_kernel<<<blocks_for(n), 256, 0, s>>>(g, nmodels, acc, model[2], model[1], model[3], model[4],
                                                    phys_pad[0], phys_pad[1], phys_pad[2], pad);
    el2_fold_kernel<<<blocks_for((long long)nmodels * g.nz * g.nx), 256, 0, s>>>(g, nmodels, pad, g_vp, g_vs,
                                                                                 g_rho);
}

} // namespace sg
