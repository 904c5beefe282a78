// ac3.hip -- gfx950 kernels of the 3-D acoustic recursion and its adjoint.
//
// Paper: U_{k+1} = A(theta) U_k + F_k (Eq. (1)), PDE Eq. (11) in the
// constant-density form u_tt = c^2 lap(u) + f, adjoint Eqs. (4)-(5).  The
// absorbing layer is the auxiliary-field form obtained by complex coordinate
// stretching, with psi = integral of u in time:
//   u_tt + s1 u_t + s2 u + s3 psi = c^2 (lap u + div phi) + f
//   phij_t = -zj phij + (sum_{i!=j} zi - zj) d_j u + (prod_{i!=j} zi) d_j psi
// Scaled variables as in 2-D (chat = dt^2 c^2 / dx^2, phi~ = dx phi,
// h = zeta dt / 2).  Forward step k:
//   pass A (layer cells):  phi~_j^k = p_j phi~_j^{k-1} + q_j D~_j u^k + r_j D~_j psi^k
//       p_j = (1-h_j)/(1+h_j), q_j = 2(hsum - 2 h_j)/(1+h_j), r_j = (4/dt) h_a h_b/(1+h_j)
//   pass B (all cells, z-marching):
//       w~^k = L~ u^k + sum_j D~_j phi~_j^k
//       u^{k+1} = alpha (beta u^k - gamma u^{k-1} - dt^2 s3 psi^k + chat w~^k + src)
//       psi^{k+1} = psi^k + dt u^{k+1}          (layer cells)
//   alpha = 1/(1+hsum), beta = 2 - 4(hx hy + hy hz + hz hx), gamma = 1 - hsum,
//   dt^2 s3 = 8 hx hy hz / dt.
// Adjoint step k (s = alpha dJ/du, b_j = dJ/dphi~_j, e = dJ/dpsi):
//   pass A':  b_j^{k+1} = p_j b_j^{k+2} - D~_j(chat s^{k+2})
//   pass B':  e^{k+1} = e^{k+2} - dt^2 s3 s^{k+2} - sum_j D~_j(r_j b_j^{k+1})
//             a^{k+1} = R^T dJ/dd^{k+1} + dt e^{k+1} - sum_j D~_j(q_j b_j^{k+1})
//                       + L~(chat s^{k+2}) + beta s^{k+2} - gamma s^{k+3}
//             s^{k+1} = alpha a^{k+1};  dJ/dchat += s^{k+1} w~^k
#include "sg_internal.h"

namespace sg {
namespace {

constexpr float A1 = (float)(8.0 / 5.0);
constexpr float A2 = (float)(-1.0 / 5.0);
constexpr float A3 = (float)(8.0 / 315.0);
constexpr float A4 = (float)(-1.0 / 560.0);
constexpr float D1 = (float)(4.0 / 5.0);
constexpr float D2 = (float)(-1.0 / 5.0);
constexpr float D3 = (float)(4.0 / 105.0);
constexpr float D4 = (float)(-1.0 / 280.0);

__device__ __forceinline__ float dcoef(int m) { return m == 1 ? D1 : m == 2 ? D2 : m == 3 ? D3 : D4; }

__device__ __forceinline__ long long f3(const Grid3 &g, int iz, int iy, int ix)
{
    return (long long)(iz + OZ3) * g.sz + (long long)(iy + OY3) * g.sy + ix + OX3;
}

template <class T>
__device__ __forceinline__ float d8(const T *c, long long s)
{
    return D1 * (c[s] - c[-s]) + D2 * (c[2 * s] - c[-2 * s])
         + D3 * (c[3 * s] - c[-3 * s]) + D4 * (c[4 * s] - c[-4 * s]);
}

// 8th-order Laplacian (times dx^2) at the centre of the LDS plane cc (row
// stride W) and of the z window q (q[4] the centre): per distance m the six
// neighbours, weighted by a_m, plus 3 a_0 times the centre.  (The 2-D kernels
// sum neighbour differences instead, which halves the rounding error; here
// the direct sum saves a third of the stencil's VALU work, and the error stays
// far below the parity bound.)
constexpr float A0X3 = (float)(3.0 * -205.0 / 72.0);
__device__ __forceinline__ float lap3(const float *cc, int W, const float *q)
{
    float s = A4 * ((cc[4] + cc[-4]) + (cc[4 * W] + cc[-4 * W]) + (q[8] + q[0]));
    s = fmaf(A3, (cc[3] + cc[-3]) + (cc[3 * W] + cc[-3 * W]) + (q[7] + q[1]), s);
    s = fmaf(A2, (cc[2] + cc[-2]) + (cc[2 * W] + cc[-2 * W]) + (q[6] + q[2]), s);
    s = fmaf(A1, (cc[1] + cc[-1]) + (cc[W] + cc[-W]) + (q[5] + q[3]), s);
    return fmaf(A0X3, q[4], s);
}

__device__ __forceinline__ int xcd_work_id(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / NXCD, rem = nblocks % NXCD;
    const int x = b % NXCD, j = b / NXCD;
    return x * per + min(x, rem) + j;
}

__device__ __forceinline__ bool tile_near_xy(const Grid3 &g, int x0, int y0)
{
    return g.P > 0 && (x0 - 4 < g.P || x0 + TX3 + 4 > g.P + g.nx || y0 - 4 < g.P || y0 + TY3 + 4 > g.P + g.ny);
}

__device__ __forceinline__ bool plane_near_z(const Grid3 &g, int z)
{
    return g.P > 0 && (z - 4 < g.P || z + 4 >= g.P + g.nz);
}

// Halo ring of a (TY3+8) x (TX3+8) plane tile: rows 0-3 and TY3+4.. full
// width, then 4 + 4 columns of the middle rows.
__device__ __forceinline__ void ring_rc(int i, int &r, int &c)
{
    constexpr int W = TX3 + 8;
    if (i < 8 * W) {
        const int s = i / W;
        c = i - s * W;
        r = s < 4 ? s : s + TY3;
    } else {
        const int j = i - 8 * W;
        const int rr = j / 8, cc = j - rr * 8;
        r = 4 + rr;
        c = cc < 4 ? cc : cc + TX3;
    }
}
constexpr int RING3 = 8 * (TX3 + 8) + 8 * TY3;

// ------------------------------------------------------------ forward pass A
// z-marching over the layer work items (every plane of the tiles that touch
// the layer in x or y, the z slabs of the others), like pass B: u^k and
// psi^k planes with a 4-cell ring in LDS, 9-plane register windows along z,
// the next plane's values loaded one plane ahead.  phi is updated at the
// layer cells only.
__device__ __forceinline__ bool layer3(const Grid3 &g, int ix, int iy, int iz)
{
    return ix < g.P || ix >= g.P + g.nx || iy < g.P || iy >= g.P + g.ny || iz < g.P || iz >= g.P + g.nz;
}

__device__ __forceinline__ float d8w(const float *q)
{
    return D1 * (q[5] - q[3]) + D2 * (q[6] - q[2]) + D3 * (q[7] - q[1]) + D4 * (q[8] - q[0]);
}

__global__ __launch_bounds__(NTH3) void ac3_phi_kernel(Ac3PhiArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pu[2][(TY3 + 8) * W];
    __shared__ float pp[2][(TY3 + 8) * W];
    const Grid3 &g = a.g;
    const int w = xcd_work_id((int)gridDim.x);
    const int shot = w / a.nitems;
    const int4 it = a.items[w - shot * a.nitems];
    const int ty = it.x / g.ntx, tx = it.x - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = it.y, z1 = it.z;
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const long long so = (long long)shot * g.plane;
    const float *u = a.u + so, *psi = a.psi + so;
    const long long col = f3(g, 0, iy, ix);
    float qu[9], qp[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const long long o = col + (long long)(z0 - 4 + m) * g.sz;
        qu[m] = u[o];
        qp[m] = psi[o];
    }
    int rs[2];
    long long ro[2];
    float ru[2], rp[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int i = tid + e * NTH3;
        int r = 0, c = 0;
        if (i < RING3) ring_rc(i, r, c);
        rs[e] = i < RING3 ? r * W + c : -1;
        ro[e] = f3(g, 0, y0 - 4 + r, x0 - 4 + c);
        const long long o = ro[e] + (long long)z0 * g.sz;
        ru[e] = rs[e] >= 0 ? u[o] : 0.f;
        rp[e] = rs[e] >= 0 ? psi[o] : 0.f;
    }
    const float hx = valid_xy ? a.t.h[0][ix] : 0.f, hy = valid_xy ? a.t.h[1][iy] : 0.f;
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        float *P = pu[z & 1], *Q = pp[z & 1];
        const int ctr = (ly + 4) * W + lx + 4;
        P[ctr] = qu[4];
        Q[ctr] = qp[4];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (rs[e] >= 0) {
                P[rs[e]] = ru[e];
                Q[rs[e]] = rp[e];
            }
        __syncthreads();
        float nu = 0.f, np = 0.f;
        if (z + 1 < z1) {
            const long long o = col + (long long)(z + 5) * g.sz;
            nu = u[o];
            np = psi[o];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (rs[e] >= 0) {
                    const long long oe = ro[e] + (long long)(z + 1) * g.sz;
                    ru[e] = u[oe];
                    rp[e] = psi[oe];
                }
        }
        if (valid_xy && layer3(g, ix, iy, z)) {
            const long long f = so + col + (long long)z * g.sz;
            const float h[3] = {hx, hy, a.t.h[2][z]};
            const int id[3] = {ix, iy, z};
            const float hs = h[0] + h[1] + h[2];
            const float du[3] = {d8(P + ctr, 1), d8(P + ctr, W), d8w(qu)};
            const float dp[3] = {d8(Q + ctr, 1), d8(Q + ctr, W), d8w(qp)};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float ih = a.t.ih[j][id[j]];
                const float q = 2.f * (hs - 2.f * h[j]) * ih;
                const float r = 4.f * a.inv_dt * h[(j + 1) % 3] * h[(j + 2) % 3] * ih;
                float *ph = a.ph[j];
                ph[f] = a.t.p[j][id[j]] * ph[f] + q * du[j] + r * dp[j];
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            qu[m] = qu[m + 1];
            qp[m] = qp[m + 1];
        }
        qu[8] = nu;
        qp[8] = np;
    }
}

// ------------------------------------------------------------ forward pass B
template <bool SNAP, bool REC>
__global__ __launch_bounds__(NTH3) void ac3_fwd_kernel(Ac3FwdArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pl[2][(TY3 + 8) * W];
    __shared__ float xch[REC ? TX3 * TY3 : 1];
    const Grid3 &g = a.g;
    const int nxy = g.ntx * g.nty;
    const int w = xcd_work_id(nxy * g.nzc * a.nshots);
    const int shot = w / (nxy * g.nzc);
    const int rem = w - shot * nxy * g.nzc;
    const int zc = rem / nxy, tile = rem - zc * nxy;
    const int ty = tile / g.ntx, tx = tile - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = zc * TZC, z1 = min(z0 + TZC, g.NZ);
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const bool near_xy = tile_near_xy(g, x0, y0);
    const long long so = (long long)shot * g.plane;
    const float *u = a.u + so;
    float *um = a.um + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const long long src = a.src_f[shot];
    const float sval = a.src_scale * a.wav[(long long)shot * a.nt + a.k];

    int rb = 0, re = 0;
    if constexpr (REC) {
        const int *off = a.rec_off + (long long)shot * (nxy + 1);
        rb = off[tile];
        re = off[tile + 1];
        while (rb < re && (a.rec_ent[rb].x >> CELL3_BITS) < z0) ++rb;
    }

    float q[9];
    const long long col = f3(g, 0, iy, ix);
#pragma unroll
    for (int m = 0; m < 9; ++m) q[m] = u[col + (long long)(z0 - 4 + m) * g.sz];
    // this thread's (at most two) halo-ring cells of every plane: LDS slot and
    // plane-0 frame offset, and their values for the current plane, loaded
    // one plane ahead so that the loads overlap the previous plane's work
    int rs[2];
    long long ro[2];
    float rv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int i = tid + e * NTH3;
        int r = 0, c = 0;
        if (i < RING3) ring_rc(i, r, c);
        rs[e] = i < RING3 ? r * W + c : -1;
        ro[e] = f3(g, 0, y0 - 4 + r, x0 - 4 + c);
        rv[e] = rs[e] >= 0 ? u[ro[e] + (long long)z0 * g.sz] : 0.f;
    }

#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        float *P = pl[z & 1];
        P[(ly + 4) * W + lx + 4] = q[4];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (rs[e] >= 0) P[rs[e]] = rv[e];
        const long long f = col + (long long)z * g.sz;
        const float umf = valid_xy ? um[f] : 0.f;
        const float chf = valid_xy ? chat[f] : 0.f;
        __syncthreads();
        // next plane: the window's new value and the ring
        float qn = 0.f;
        if (z + 1 < z1) {
            qn = u[col + (long long)(z + 5) * g.sz];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (rs[e] >= 0) rv[e] = u[ro[e] + (long long)(z + 1) * g.sz];
        }
        const float *cc = P + (ly + 4) * W + lx + 4;
        const float c0 = q[4];
        float wv = lap3(cc, W, q);
        float un = 0.f;
        if (valid_xy) {
            if (near_xy || plane_near_z(g, z)) {
                wv += d8(a.ph[0] + so + f, 1) + d8(a.ph[1] + so + f, g.sy) + d8(a.ph[2] + so + f, g.sz);
                const float hx = a.t.h[0][ix], hy = a.t.h[1][iy], hz = a.t.h[2][z];
                const float hs = hx + hy + hz;
                float inc = (c0 - umf) + (hs * umf - 4.f * (hx * hy + hy * hz + hz * hx) * c0) + chf * wv;
                float ps = 0.f;
                if (hs > 0.f) {
                    ps = a.psi[so + f];
                    inc -= 8.f * hx * hy * hz * a.inv_dt * ps;
                }
                if (f == src) inc += sval;
                un = (c0 + inc) / (1.f + hs);
                if (hs > 0.f) a.psi[so + f] = ps + a.dt * un;
            } else {
                float inc = (c0 - umf) + chf * wv;
                if (f == src) inc += sval;
                un = c0 + inc;
            }
            um[f] = un;
            if constexpr (SNAP) a.snap[so + f] = wv;
        }
        if constexpr (REC) {
            int pe = rb;
            while (pe < re && (a.rec_ent[pe].x >> CELL3_BITS) == z) ++pe;
            if (pe > rb) {                         // uniform over the block
                xch[tid] = un;
                __syncthreads();
                for (int i = rb + tid; i < pe; i += NTH3) {
                    const int2 en = a.rec_ent[i];
                    a.seis[((long long)shot * a.nt + a.k) * a.nrec + en.y] = xch[en.x & ((1 << CELL3_BITS) - 1)];
                }
                __syncthreads();
                rb = pe;
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) q[m] = q[m + 1];
        q[8] = qn;
        __builtin_amdgcn_sched_barrier(0);   // keep each plane's loads in its own iteration
    }
}

// ------------------------------------------------------------ adjoint pass A
// Same work items and marching, on chat s^{k+2}.
__global__ __launch_bounds__(NTH3) void ac3_phi_adj_kernel(Ac3PhiAdjArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pc[2][(TY3 + 8) * W];
    const Grid3 &g = a.g;
    const int w = xcd_work_id((int)gridDim.x);
    const int shot = w / a.nitems;
    const int4 it = a.items[w - shot * a.nitems];
    const int ty = it.x / g.ntx, tx = it.x - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = it.y, z1 = it.z;
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const long long so = (long long)shot * g.plane;
    const float *s2 = a.s2 + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const long long col = f3(g, 0, iy, ix);
    float q[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const long long o = col + (long long)(z0 - 4 + m) * g.sz;
        q[m] = chat[o] * s2[o];
    }
    int rs[2];
    long long ro[2];
    float rv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int i = tid + e * NTH3;
        int r = 0, c = 0;
        if (i < RING3) ring_rc(i, r, c);
        rs[e] = i < RING3 ? r * W + c : -1;
        ro[e] = f3(g, 0, y0 - 4 + r, x0 - 4 + c);
        const long long o = ro[e] + (long long)z0 * g.sz;
        rv[e] = rs[e] >= 0 ? chat[o] * s2[o] : 0.f;
    }
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        float *P = pc[z & 1];
        const int ctr = (ly + 4) * W + lx + 4;
        P[ctr] = q[4];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (rs[e] >= 0) P[rs[e]] = rv[e];
        __syncthreads();
        float nq = 0.f;
        if (z + 1 < z1) {
            const long long o = col + (long long)(z + 5) * g.sz;
            nq = chat[o] * s2[o];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (rs[e] >= 0) {
                    const long long oe = ro[e] + (long long)(z + 1) * g.sz;
                    rv[e] = chat[oe] * s2[oe];
                }
        }
        if (valid_xy && layer3(g, ix, iy, z)) {
            const long long f = so + col + (long long)z * g.sz;
            const int id[3] = {ix, iy, z};
            const float d[3] = {d8(P + ctr, 1), d8(P + ctr, W), d8w(q)};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float *b = a.b[j];
                b[f] = a.t.p[j][id[j]] * b[f] - d[j];
            }
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) q[m] = q[m + 1];
        q[8] = nq;
    }
}

// ------------------------------------------------------------ adjoint pass B
__global__ __launch_bounds__(NTH3) void ac3_adj_kernel(Ac3AdjArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pl[2][(TY3 + 8) * W];
    __shared__ float xch[TX3 * TY3];
    const Grid3 &g = a.g;
    const int nxy = g.ntx * g.nty;
    const int w = xcd_work_id(nxy * g.nzc * a.nshots);
    const int shot = w / (nxy * g.nzc);
    const int rem = w - shot * nxy * g.nzc;
    const int zc = rem / nxy, tile = rem - zc * nxy;
    const int ty = tile / g.ntx, tx = tile - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = zc * TZC, z1 = min(z0 + TZC, g.NZ);
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const bool near_xy = tile_near_xy(g, x0, y0);
    const long long so = (long long)shot * g.plane;
    const float *s2 = a.s2 + so;
    float *s3 = a.s3 + so;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    const long long src = a.src_f[shot];

    const int *off = a.rec_off + (long long)shot * (nxy + 1);
    int rb = off[tile], re = off[tile + 1];
    while (rb < re && (a.rec_ent[rb].x >> CELL3_BITS) < z0) ++rb;
    const float *dd = a.dJdd + ((long long)shot * a.nt + a.k) * a.nrec;

    float q[9];        // chat s^{k+2}, z-4 .. z+4 of the own column
    float sraw;        // s^{k+2} at (z, own column)
    const long long col = f3(g, 0, iy, ix);
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const long long o = col + (long long)(z0 - 4 + m) * g.sz;
        q[m] = chat[o] * s2[o];
    }
    // halo-ring cells of this thread, loaded one plane ahead (as in the forward)
    int rs[2];
    long long ro[2];
    float rv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int i = tid + e * NTH3;
        int r = 0, c = 0;
        if (i < RING3) ring_rc(i, r, c);
        rs[e] = i < RING3 ? r * W + c : -1;
        ro[e] = f3(g, 0, y0 - 4 + r, x0 - 4 + c);
        const long long o = ro[e] + (long long)z0 * g.sz;
        rv[e] = rs[e] >= 0 ? chat[o] * s2[o] : 0.f;
    }
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        const long long f = col + (long long)z * g.sz;
        sraw = s2[f];
        float *P = pl[z & 1];
        P[(ly + 4) * W + lx + 4] = q[4];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (rs[e] >= 0) P[rs[e]] = rv[e];
        const float s3f = valid_xy ? s3[f] : 0.f;
        const float snf = valid_xy ? a.snap[so + f] : 0.f;
        __syncthreads();
        float qn = 0.f;
        if (z + 1 < z1) {
            const long long o = col + (long long)(z + 5) * g.sz;
            qn = chat[o] * s2[o];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                if (rs[e] >= 0) {
                    const long long oe = ro[e] + (long long)(z + 1) * g.sz;
                    rv[e] = chat[oe] * s2[oe];
                }
        }
        const float *cc = P + (ly + 4) * W + lx + 4;
        float v = lap3(cc, W, q);
        bool nearz = false;
        float hs = 0.f;
        if (valid_xy) {
            nearz = near_xy || plane_near_z(g, z);
            if (nearz) {
                const int id[3] = {ix, iy, z};
                const float h[3] = {a.t.h[0][ix], a.t.h[1][iy], a.t.h[2][z]};
                hs = h[0] + h[1] + h[2];
                const long long st[3] = {1, g.sy, g.sz};
                float de = 0.f;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float ha = h[(j + 1) % 3], hb = h[(j + 2) % 3];
                    const float *tj = a.t.h[j], *ij = a.t.ih[j];
                    const float *b = a.b[j] + so + f;
                    float dq = 0.f, dr = 0.f;
#pragma unroll
                    for (int m = 1; m <= 4; ++m) {
                        const long long o = m * st[j];
                        const float bp = b[o], bm = b[-o];
                        const float ip = ij[id[j] + m], im = ij[id[j] - m];
                        dq += dcoef(m) * (2.f * (ha + hb - tj[id[j] + m]) * ip * bp
                                          - 2.f * (ha + hb - tj[id[j] - m]) * im * bm);
                        dr += dcoef(m) * (ip * bp - im * bm);
                    }
                    v -= dq;
                    de += 4.f * a.inv_dt * ha * hb * dr;
                }
                if (hs > 0.f) {
                    const float en = a.e[so + f] - 8.f * h[0] * h[1] * h[2] * a.inv_dt * sraw - de;
                    a.e[so + f] = en;
                    v += a.dt * en;
                }
                v += sraw + ((sraw - s3f) + (hs * s3f - 4.f * (h[0] * h[1] + h[1] * h[2] + h[2] * h[0]) * sraw));
            } else {
                v += sraw + (sraw - s3f);
            }
        }
        // receiver residual injection (deterministic per cell)
        int pe = rb;
        while (pe < re && (a.rec_ent[pe].x >> CELL3_BITS) == z) ++pe;
        if (pe > rb) {                              // uniform over the block
            xch[tid] = v;
            __syncthreads();
            for (int i = rb + tid; i < pe; i += NTH3) {
                const int cell = a.rec_ent[i].x & ((1 << CELL3_BITS) - 1);
                if (i > rb && (a.rec_ent[i - 1].x & ((1 << CELL3_BITS) - 1)) == cell) continue;
                float sum = 0.f;
                for (int m = i; m < pe && (a.rec_ent[m].x & ((1 << CELL3_BITS) - 1)) == cell; ++m)
                    sum += dd[a.rec_ent[m].y];
                xch[cell] += sum;
            }
            __syncthreads();
            v = xch[tid];
            __syncthreads();
            rb = pe;
        }
        if (valid_xy) {
            const float s1 = nearz ? v / (1.f + hs) : v;
            s3[f] = s1;
            a.grad[so + f] += s1 * snf;
            if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k] = s1 * a.src_scale;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) q[m] = q[m + 1];
        q[8] = qn;
        __builtin_amdgcn_sched_barrier(0);
    }
}

__global__ void ac3_prep_kernel(Grid3 g, int nmodels, const float *vp, double dt, double dx,
                                float *chat, float *cpad)
{
    const long long n = (long long)nmodels * g.plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / g.plane, f = i - m * g.plane;
        const int fz = (int)(f / g.sz);
        const long long r = f - fz * g.sz;
        const int fy = (int)(r / g.sy), fx = (int)(r - fy * g.sy);
        const int iz = fz - OZ3, iy = fy - OY3, ix = fx - OX3;
        float c = 0.f, ch = 0.f;
        if (iz >= 0 && iz < g.NZ && iy >= 0 && iy < g.NY && ix >= 0 && ix < g.NX) {
            const int pz = min(max(iz - g.P, 0), g.nz - 1), py = min(max(iy - g.P, 0), g.ny - 1),
                      px = min(max(ix - g.P, 0), g.nx - 1);
            c = vp[((m * g.nz + pz) * g.ny + py) * g.nx + px];
            const double cd = c;
            ch = (float)(dt * dt * cd * cd / (dx * dx));
        }
        chat[i] = ch;
        cpad[i] = c;
    }
}

__global__ void ac3_sum_shots_kernel(Grid3 g, int nmodels, int spm, const float *grad, float *acc)
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

// Fold the padded cells onto the physical cells they replicate, then the
// chain rule dchat/dc = 2 dt^2 c / dx^2.
__global__ void ac3_finalize_kernel(Grid3 g, int nmodels, const float *acc, const float *cpad,
                                    double dt, double dx, float *g_vp)
{
    const long long nphys = (long long)g.nx * g.ny * g.nz;
    const long long n = (long long)nmodels * nphys;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / nphys, rem = i - m * nphys;
        const int iz = (int)(rem / ((long long)g.nx * g.ny));
        const long long r2 = rem - (long long)iz * g.nx * g.ny;
        const int iy = (int)(r2 / g.nx), ix = (int)(r2 - (long long)iy * g.nx);
        const int zlo = iz == 0 ? 0 : iz + g.P, zhi = iz == g.nz - 1 ? g.NZ - 1 : iz + g.P;
        const int ylo = iy == 0 ? 0 : iy + g.P, yhi = iy == g.ny - 1 ? g.NY - 1 : iy + g.P;
        const int xlo = ix == 0 ? 0 : ix + g.P, xhi = ix == g.nx - 1 ? g.NX - 1 : ix + g.P;
        const float *am = acc + m * g.plane;
        float v = 0.f;
        for (int pz = zlo; pz <= zhi; ++pz)
            for (int py = ylo; py <= yhi; ++py)
                for (int px = xlo; px <= xhi; ++px) v += am[f3(g, pz, py, px)];
        const double c = cpad[m * g.plane + f3(g, iz + g.P, iy + g.P, ix + g.P)];
        g_vp[i] = (float)(2.0 * dt * dt * c / (dx * dx)) * v;
    }
}

} // namespace

void launch_ac3_phi(const Ac3PhiArgs &a, int nshots, hipStream_t s)
{
    if (a.g.P == 0 || nshots == 0 || a.nitems == 0) return;
    ac3_phi_kernel<<<a.nitems * nshots, NTH3, 0, s>>>(a);
}

void launch_ac3_phi_adj(const Ac3PhiAdjArgs &a, int nshots, hipStream_t s)
{
    if (a.g.P == 0 || nshots == 0 || a.nitems == 0) return;
    ac3_phi_adj_kernel<<<a.nitems * nshots, NTH3, 0, s>>>(a);
}

void launch_ac3_fwd(const Ac3FwdArgs &a, hipStream_t s)
{
    const int nb = a.g.ntx * a.g.nty * a.g.nzc * a.nshots;
    if (nb == 0) return;
    const bool snap = a.snap != nullptr, rec = a.seis != nullptr;
    if (snap) { if (rec) ac3_fwd_kernel<true, true><<<nb, NTH3, 0, s>>>(a); else ac3_fwd_kernel<true, false><<<nb, NTH3, 0, s>>>(a); }
    else      { if (rec) ac3_fwd_kernel<false, true><<<nb, NTH3, 0, s>>>(a); else ac3_fwd_kernel<false, false><<<nb, NTH3, 0, s>>>(a); }
}

void launch_ac3_adj(const Ac3AdjArgs &a, hipStream_t s)
{
    const int nb = a.g.ntx * a.g.nty * a.g.nzc * a.nshots;
    if (nb == 0) return;
    ac3_adj_kernel<<<nb, NTH3, 0, s>>>(a);
}

void launch_ac3_prep(const Grid3 &g, int nmodels, const float *vp, double dt, double dx,
                     float *chat, float *cpad, hipStream_t s)
{
    const long long n = (long long)nmodels * g.plane;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac3_prep_kernel<<<blocks, 256, 0, s>>>(g, nmodels, vp, dt, dx, chat, cpad);
}

void launch_ac3_finalize(const Grid3 &g, int nmodels, int spm, const float *grad, float *acc,
                         const float *cpad, double dt, double dx, float *g_vp, hipStream_t s)
{
    long long n = (long long)nmodels * g.plane;
    int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac3_sum_shots_kernel<<<blocks, 256, 0, s>>>(g, nmodels, spm, grad, acc);
    n = (long long)nmodels * g.nx * g.ny * g.nz;
    blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac3_finalize_kernel<<<blocks, 256, 0, s>>>(g, nmodels, acc, cpad, dt, dx, g_vp);
}

} // namespace sg
