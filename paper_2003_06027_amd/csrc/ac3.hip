// ac3.hip -- gfx950 kernels of the 3-D acoustic recursion and its adjoint.
//
// Paper: U_{k+1} = A(theta) U_k + F_k (Eq. (1)), PDE Eq. (12) in the
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
#include "ac3_internal.h"

#include <climits>
#include <type_traits>

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

// Work item of this workgroup: the hardware order, which deals consecutive
// items to the 8 XCDs in turn, so that all XCDs march the same chunks at
// once.  Giving each XCD a contiguous range of items instead, as the 2-D
// kernels do, was measured slower at 448^3: interior forward 465 -> 359 us,
// interior adjoint 736 -> 669 us, forward step 1088 -> 963 us in hardware
// order.
__device__ __forceinline__ int work_id()
{
    return (int)blockIdx.x;
}

// Work item of a tile pass over a list of ntl xy tiles: the (shot, z chunk)
// pair cs and the tile's position t in the list.  Workgroups still go to
// the XCDs in turn and all XCDs march the same chunk, but each XCD takes a
// contiguous run of the list (whole rows of tiles), so the halo rings a tile
// reads were mostly brought into the same XCD's L2 by its neighbours.  The
// grid holds band_blocks(ntl) workgroups per (shot, chunk); those past the
// list return at once.
__host__ __device__ __forceinline__ int band_per(int ntl) { return (ntl + NXCD - 1) / NXCD; }
__device__ __forceinline__ bool band_item(int ntl, int &cs, int &t)
{
    const int per = band_per(ntl);
    const int b = (int)blockIdx.x, x = b % NXCD, s = b / NXCD;
    cs = s / per;
    t = x * per + (s - cs * per);
    return t < ntl;
}

__device__ __forceinline__ bool plane_near_z(const Grid3 &g, int z)
{
    return g.P > 0 && (z - 4 < g.P || z + 4 >= g.P + g.nz);
}

// psi (forward) and its adjoint e enter the recursion only through terms
// with the damping of two or three axes (s3 psi; h_a h_b D~_j psi, whose
// stencil along j stays on cells with the same two damped axes), so they are
// kept only on cells with at least two damped axes: elsewhere they stay
// zero, and a tile plane without such cells reads them from one shared zero
// line of the frame instead of its columns.  Planes of a tile that may hold
// such cells: every plane if the tile meets the layer in x and in y, the z
// slabs if it meets it in x or in y.
struct TwoAxis {
    bool xy, any;
    __device__ bool plane(const Grid3 &g, int z) const { return xy || (any && (z < g.P || z >= g.P + g.nz)); }
};
__device__ __forceinline__ TwoAxis two_axis_tile(const Grid3 &g, int x0, int y0)
{
    const bool tx = x0 < g.P || x0 + TX3 > g.P + g.nx, ty = y0 < g.P || y0 + TY3 > g.P + g.ny;
    return TwoAxis{tx && ty, tx || ty};
}
__device__ __forceinline__ bool two_axis_cell(float hx, float hy, float hz)
{
    return (hx > 0.f) + (hy > 0.f) + (hz > 0.f) >= 2;
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

__device__ __forceinline__ float d8w(const float *q)
{
    return D1 * (q[5] - q[3]) + D2 * (q[6] - q[2]) + D3 * (q[7] - q[1]) + D4 * (q[8] - q[0]);
}

// ------------------------------------------------------------ marching scheme
// Every per-plane operand is loaded PD planes ahead into registers that the
// planes in between do not use: the z windows are rings of ZR registers (9
// in use, the next PD receiving planes z + 5 ..), the other operands rings of
// NB = PD + 1, and the z loop is unrolled by ZR so that ring positions are
// compile-time constants.  The prefetch loads are unconditional (addresses
// stay inside the frame; unused values are dropped) and so are the stores
// that follow them, so that the memory counter waits are exact and do not
// wait for the loads just issued; a conditional store of a plane (psi, phi,
// e on layer cells) is issued at the start of the next one, before its
// prefetch.  Streaming operands use non-temporal loads and stores.  Addresses are
// 32-bit byte offsets from per-block bases at the chunk's first window plane
// (the host bounds (TZC + 8) planes below 4 GiB).
constexpr int PD = 1, NB = PD + 1, ZR = 10;
static_assert(ZR % NB == 0 && 8 + PD < ZR, "ring sizes");
static_assert(RING3 <= NTH3, "one halo-ring cell per thread");

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>)
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

__device__ __forceinline__ void tab_at(const float *h, const float *ih, int i, int n, float &hv, float &ihv)
{
    const bool in = i >= -4 && i < n + 4;     // the tables' extent
    hv = in ? h[i] : 0.f;
    ihv = in ? ih[i] : 1.f;
}

__device__ __forceinline__ float ldb(const float *b, unsigned o)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(b) + o);
}
__device__ __forceinline__ void stb(float *b, unsigned o, float v)
{
    *reinterpret_cast<float *>(reinterpret_cast<char *>(b) + o) = v;
}
// streaming operands (read or written once per step, no neighbour reuse):
// non-temporal, so that they do not displace the reused planes from L2
__device__ __forceinline__ float ldn(const float *b, unsigned o)
{
    return __builtin_nontemporal_load(reinterpret_cast<const float *>(reinterpret_cast<const char *>(b) + o));
}
__device__ __forceinline__ void stn(float *b, unsigned o, float v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<float *>(reinterpret_cast<char *>(b) + o));
}
// d8 at byte offset o with byte stride sb
__device__ __forceinline__ float d8b(const float *b, unsigned o, unsigned sb)
{
    return D1 * (ldb(b, o + sb) - ldb(b, o - sb)) + D2 * (ldb(b, o + 2 * sb) - ldb(b, o - 2 * sb))
         + D3 * (ldb(b, o + 3 * sb) - ldb(b, o - 3 * sb)) + D4 * (ldb(b, o + 4 * sb) - ldb(b, o - 4 * sb));
}

// ------------------------------------------------------------ forward pass A
// z-marching over the layer work items (every plane of the tiles that touch
// the layer in x or y, the z slabs of the others), like pass B: u^k and
// psi^k planes with a 4-cell ring in LDS, register windows along z, the
// operands of the next plane loaded one plane ahead into rings (the marching
// scheme above).  phi is updated at the layer cells only, and loaded only
// there (elsewhere every lane reads one shared line).  The psi terms of
// axis j carry the damping of the other two axes, h_a h_b: items where no
// cell has two axes in the layer (PSI = false: a tile in the layer in x or
// y only, off the z slabs; the z slabs of the other tiles) leave psi out,
// which adds an exact zero in the other items.
constexpr int LPD = 1, LNB = LPD + 1, LZR = 10;
static_assert(LZR % LNB == 0 && 8 + LPD < LZR, "ring sizes");

template <bool PSI>
__global__ __launch_bounds__(NTH3) __attribute__((amdgpu_waves_per_eu(8)))
void ac3_phi_kernel(Ac3PhiArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pu[2][(TY3 + 8) * W];
    __shared__ float pp[PSI ? 2 : 1][PSI ? (TY3 + 8) * W : 1];
    const Grid3 &g = a.g;
    const int w = work_id();
    const int shot = w / a.nitems;
    const int4 it = a.items[w - shot * a.nitems];
    if (it.x < 0) return;                  // padding of the launch order
    const int ty = it.x / g.ntx, tx = it.x - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = it.y, z1 = it.z;
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const bool layer_xy = ix < g.P || ix >= g.P + g.nx || iy < g.P || iy >= g.P + g.ny;
    const long long zb0 = (long long)shot * g.plane + (long long)(z0 + OZ3 - 4) * g.sz;
    const float *u = a.u + zb0, *psi = a.psi + zb0;
    float *ph0 = a.ph[0] + zb0, *ph1 = a.ph[1] + zb0, *ph2 = a.ph[2] + zb0;
    const unsigned SZB = (unsigned)g.sz * 4u;
    auto pb = [&](int z) { return (unsigned)(z - z0 + 4) * SZB; };
    auto pbc = [&](int z) { return pb(min(z, g.NZ + 3)); };
    const unsigned colb = (unsigned)((iy + OY3) * g.sy + ix + OX3) * 4u;
    int rs;
    unsigned rob;
    {
        int r = 0, c = 0;
        if (tid < RING3) ring_rc(tid, r, c);
        rs = tid < RING3 ? r * W + c : -1;
        rob = (unsigned)((y0 - 4 + r + OY3) * g.sy + x0 - 4 + c + OX3) * 4u;
    }
    float qu[LZR], qp[PSI ? LZR : 1], ru[LNB], rp[PSI ? LNB : 1], f0[LNB], f1[LNB], f2[LNB];
#pragma unroll
    for (int m = 0; m < 8 + LPD; ++m) {
        const unsigned o = colb + pbc(z0 - 4 + m);
        qu[m] = ldb(u, o);
        if constexpr (PSI) qp[m] = ldb(psi, o);
    }
#pragma unroll
    for (int d = 0; d < LPD; ++d) {
        const unsigned o = pbc(z0 + d);
        ru[d] = ldb(u, rob + o);
        if constexpr (PSI) rp[d] = ldb(psi, rob + o);
        f0[d] = ldb(ph0, colb + o);
        f1[d] = ldb(ph1, colb + o);
        f2[d] = ldb(ph2, colb + o);
    }
    // per-column coefficients of x and y
    float hx = 0.f, hy = 0.f, ihx = 1.f, ihy = 1.f, px = 1.f, py = 1.f;
    if (valid_xy) {
        hx = a.t.h[0][ix]; ihx = a.t.ih[0][ix]; px = a.t.p[0][ix];
        hy = a.t.h[1][iy]; ihy = a.t.ih[1][iy]; py = a.t.p[1][iy];
    }
    // phi of the previous plane, stored at the start of the next
    bool fw = false;
    float fn0 = 0.f, fn1 = 0.f, fn2 = 0.f;
    unsigned ff = 0;

#pragma unroll 1
    for (int zb = z0; zb < z1; zb += LZR) {
        const int zbo = __builtin_amdgcn_readfirstlane(zb);
        static_for<LZR>([&](auto R) __attribute__((always_inline)) {
            constexpr int r = decltype(R)::value;
            constexpr int c = r % LNB, n = (r + LPD) % LNB;
            const int z = zbo + r;
            if (z >= z1) return;
            if (fw) {
                stb(ph0, ff, fn0);
                stb(ph1, ff, fn1);
                stb(ph2, ff, fn2);
            }
            fw = false;
            float *P = pu[z & 1], *Q = pp[PSI ? (z & 1) : 0];
            const int ctr = (ly + 4) * W + lx + 4;
            P[ctr] = qu[(r + 4) % LZR];
            if constexpr (PSI) Q[ctr] = qp[(r + 4) % LZR];
            if (rs >= 0) {
                P[rs] = ru[c];
                if constexpr (PSI) Q[rs] = rp[c];
            }
            const unsigned fb = colb + pb(z);
            __syncthreads();
            {
                const unsigned d1 = pbc(z + LPD), dw = colb + pbc(z + 4 + LPD);
                ru[n] = ldb(u, rob + d1);
                if constexpr (PSI) rp[n] = ldb(psi, rob + d1);
                qu[(r + 8 + LPD) % LZR] = ldb(u, dw);
                if constexpr (PSI) qp[(r + 8 + LPD) % LZR] = ldb(psi, dw);
                // phi only where it is updated; elsewhere one shared line
                const unsigned fo = layer_xy || z + LPD < g.P || z + LPD >= g.P + g.nz ? colb + d1 : 0u;
                f0[n] = ldb(ph0, fo);
                f1[n] = ldb(ph1, fo);
                f2[n] = ldb(ph2, fo);
            }
            if (valid_xy && (layer_xy || z < g.P || z >= g.P + g.nz)) {
                float wu[9], wp[9];
#pragma unroll
                for (int m = 0; m < 9; ++m) {
                    wu[m] = qu[(r + m) % LZR];
                    if constexpr (PSI) wp[m] = qp[(r + m) % LZR];
                }
                const float hz = a.t.h[2][z], ihz = a.t.ih[2][z], pz = a.t.p[2][z];
                const float hs = hx + hy + hz;
                fn0 = px * f0[c] + 2.f * (hs - 2.f * hx) * ihx * d8(P + ctr, 1);
                fn1 = py * f1[c] + 2.f * (hs - 2.f * hy) * ihy * d8(P + ctr, W);
                fn2 = pz * f2[c] + 2.f * (hs - 2.f * hz) * ihz * d8w(wu);
                if constexpr (PSI) {
                    const float k4 = 4.f * a.inv_dt;
                    fn0 += k4 * hy * hz * ihx * d8(Q + ctr, 1);
                    fn1 += k4 * hz * hx * ihy * d8(Q + ctr, W);
                    fn2 += k4 * hx * hy * ihz * d8w(wp);
                }
                fw = true;
                ff = fb;
            }
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    if (fw) {
        stb(ph0, ff, fn0);
        stb(ph1, ff, fn1);
        stb(ph2, ff, fn2);
    }
}

// ------------------------------------------------------------ forward pass B
// Two launches over (xy tile, z chunk, shot): the tiles within 4 cells of the
// layer in x or y (LAYER: every plane takes the layer terms) and the others
// (only the z slabs do; their cells are interior in x and y, hx = hy = 0).
// In LAYER tiles the layer auxiliaries are staged like u: phi_x with its x
// halo and phi_y with its y halo in LDS planes, phi_z in a register window;
// the other tiles read the few stencil points of their slab planes directly.
template <bool SNAP, bool REC, bool LAYER>
__global__ __launch_bounds__(NTH3) __attribute__((amdgpu_waves_per_eu(LAYER ? 4 : 8)))
void ac3_fwd_kernel(Ac3FwdArgs a)
{
    constexpr int W = TX3 + 8;
    constexpr int WX = TX3 + 8, WY = TX3;      // phi_x plane: TY3 rows of WX; phi_y: TY3 + 8 rows of WY
    __shared__ float pl[2][(TY3 + 8) * W];
    __shared__ float sphx[LAYER ? 2 * TY3 * WX : 1];
    __shared__ float sphy[LAYER ? 2 * (TY3 + 8) * WY : 1];
    __shared__ float xch[REC ? TX3 * TY3 : 1];
    const Grid3 &g = a.g;
    const int nzf = (g.NZ + g.zcf - 1) / g.zcf;
    int cs, ti;
    if (!band_item(a.ntl, cs, ti)) return;
    const int shot = cs / nzf, zc = cs - shot * nzf, tile = a.tiles[a.t0 + ti];
    const int nxy = g.ntx * g.nty;
    const int ty = tile / g.ntx, tx = tile - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = zc * g.zcf, z1 = min(z0 + g.zcf, g.NZ);
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    // bases at plane z0 - 4 of this shot; plane z at byte offset pb(z)
    const long long zoff = (long long)(z0 + OZ3 - 4) * g.sz;
    const long long zb0 = (long long)shot * g.plane + zoff;
    const float *u = a.u + zb0;
    float *um = a.um + zb0;
    float *psi = a.psi + zb0;
    float *snap = a.snap + zb0;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane + zoff;
    const float *phx = a.ph[0] + zb0, *phy = a.ph[1] + zb0, *phz = a.ph[2] + zb0;
    const unsigned SZB = (unsigned)g.sz * 4u, SYB = (unsigned)g.sy * 4u;
    auto pb = [&](int z) { return (unsigned)(z - z0 + 4) * SZB; };
    auto pbc = [&](int z) { return pb(min(z, g.NZ + 3)); };
    const unsigned colb = (unsigned)((iy + OY3) * g.sy + ix + OX3) * 4u;
    // the source cell as (plane, in-plane byte offset)
    const long long src = a.src_f[shot];
    const int srcp = (int)(src / g.sz) - OZ3;
    const unsigned srcc = (unsigned)(src - (long long)(srcp + OZ3) * g.sz) * 4u;
    const float sval = a.src_scale * a.wav[(long long)shot * a.nt + a.k];

    // receivers of this tile and chunk, by plane; zr = plane of the next one
    int rb = 0, re = 0, zr = INT_MAX;
    if constexpr (REC) {
        const int *off = a.rec_off + (long long)shot * (nxy + 1);
        rb = off[tile];
        re = off[tile + 1];
        while (rb < re && (a.rec_ent[rb].x >> CELL3_BITS) < z0) ++rb;
        if (rb < re) zr = a.rec_ent[rb].x >> CELL3_BITS;
    }

    // window: planes z0 - 4 .. z0 + 3 + PD; the rings: planes z0 .. z0 + PD - 1
    float q[ZR];
#pragma unroll
    for (int m = 0; m < 8 + PD; ++m) q[m] = ldb(u, colb + pbc(z0 - 4 + m));
    // this thread's halo-ring cell of every plane (if any): LDS slot and
    // in-plane byte offset (a cell of the ring's row 0 for threads without)
    int rs;
    unsigned rob;
    float rv[NB], umv[NB], chv[NB];
    {
        int r = 0, c = 0;
        if (tid < RING3) ring_rc(tid, r, c);
        rs = tid < RING3 ? r * W + c : -1;
        rob = (unsigned)((y0 - 4 + r + OY3) * g.sy + x0 - 4 + c + OX3) * 4u;
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        rv[d] = ldb(u, rob + pbc(z0 + d));
        umv[d] = ldn(um, colb + pbc(z0 + d));
        chv[d] = ldn(chat, colb + pbc(z0 + d));
    }
    // LAYER: the phi_z window, this column's phi_x, phi_y and psi, and one
    // halo cell: of phi_x (the first 8 TY3 threads) or of phi_y (the next 8 TX3)
    float pz[LAYER ? ZR : 1], pxv[NB], pyv[NB], hvv[NB], psv[NB];
    const TwoAxis two = two_axis_tile(g, x0, y0);
    int hslot = -1;
    const float *hsrc = phx;
    unsigned hob = colb;
    float hx = 0.f, hy = 0.f;
    if constexpr (LAYER) {
#pragma unroll
        for (int m = 0; m < 8 + PD; ++m) pz[m] = ldb(phz, colb + pbc(z0 - 4 + m));
        if (tid < 8 * TY3) {
            const int r = tid / 8, c = tid % 8, cx = c < 4 ? c : c + TX3;
            hslot = r * WX + cx;
            hob = (unsigned)((y0 + r + OY3) * g.sy + x0 - 4 + cx + OX3) * 4u;
        } else if (tid < 8 * TY3 + 8 * TX3) {
            const int i = tid - 8 * TY3, r = i / TX3, c = i % TX3, ry = r < 4 ? r : r + TY3;
            hslot = TY3 * WX + ry * WY + c;    // past the phi_x plane: one index space for both
            hsrc = phy;
            hob = (unsigned)((y0 - 4 + ry + OY3) * g.sy + x0 + c + OX3) * 4u;
        }
#pragma unroll
        for (int d = 0; d < PD; ++d) {
            const unsigned o = pbc(z0 + d);
            pxv[d] = ldb(phx, colb + o);
            pyv[d] = ldb(phy, colb + o);
            psv[d] = ldb(psi, two.plane(g, z0 + d) ? colb + o : 0u);
            hvv[d] = ldb(hsrc, hob + o);
        }
        if (valid_xy) {
            hx = a.t.h[0][ix];
            hy = a.t.h[1][iy];
        }
    }
    // psi^{k+1} of the previous plane, stored at the start of the next
    bool psw = false;
    float psn = 0.f;
    unsigned psf = 0;

#pragma unroll 1
    for (int zb = z0; zb < z1; zb += ZR) {
        // an opaque copy of the chunk's plane: addresses are formed afresh in
        // every pass rather than carried as strength-reduced pointers
        const int zbo = __builtin_amdgcn_readfirstlane(zb);
        static_for<ZR>([&](auto R) __attribute__((always_inline)) {
            constexpr int r = decltype(R)::value;
            constexpr int c = r % NB, n = (r + PD) % NB;
            const int z = zbo + r;
            if (z >= z1) return;
            if (psw) stb(psi, psf, psn);
            psw = false;
            float *P = pl[z & 1];
            P[(ly + 4) * W + lx + 4] = q[(r + 4) % ZR];
            if (rs >= 0) P[rs] = rv[c];
            float *PX = sphx + (LAYER ? (z & 1) * TY3 * WX : 0);
            float *PY = sphy + (LAYER ? (z & 1) * (TY3 + 8) * WY : 0);
            if constexpr (LAYER) {
                PX[ly * WX + lx + 4] = pxv[c];
                PY[(ly + 4) * WY + lx] = pyv[c];
                if (hslot >= 0) {
                    if (hslot < TY3 * WX) PX[hslot] = hvv[c];
                    else PY[hslot - TY3 * WX] = hvv[c];
                }
            }
            const unsigned fb = colb + pb(z);
            __syncthreads();
            // plane z + PD (the windows: plane z + 4 + PD), kept inside the frame
            {
                const unsigned d1 = pbc(z + PD), dw = pbc(z + 4 + PD);
                rv[n] = ldb(u, rob + d1);
                if constexpr (LAYER) {
                    pxv[n] = ldb(phx, colb + d1);
                    pyv[n] = ldb(phy, colb + d1);
                    hvv[n] = ldb(hsrc, hob + d1);
                }
                q[(r + 8 + PD) % ZR] = ldb(u, colb + dw);
                umv[n] = ldn(um, colb + d1);
                chv[n] = ldn(chat, colb + d1);
                if constexpr (LAYER) {
                    pz[(r + 8 + PD) % ZR] = ldb(phz, colb + dw);
                    psv[n] = ldb(psi, two.plane(g, z + PD) ? colb + d1 : 0u);
                }
            }
            float qw[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) qw[m] = q[(r + m) % ZR];
            const float *cc = P + (ly + 4) * W + lx + 4;
            const float c0 = qw[4], umf = umv[c], chf = chv[c];
            float wv = lap3(cc, W, qw);
            float un = 0.f;
            const bool at_src = z == srcp && colb == srcc;
            if (valid_xy) {
                if (LAYER || plane_near_z(g, z)) {
                    float ps;
                    if constexpr (LAYER) {
                        float pw[9];
#pragma unroll
                        for (int m = 0; m < 9; ++m) pw[m] = pz[(r + m) % ZR];
                        wv += d8(PX + ly * WX + lx + 4, 1) + d8(PY + (ly + 4) * WY + lx, (long long)WY) + d8w(pw);
                        ps = psv[c];
                    } else {
                        // slab planes only: the offset comes from an opaque
                        // copy of z (no strength-reduced stencil addresses)
                        const unsigned fo = colb + pb(__builtin_amdgcn_readfirstlane(z));
                        wv += d8b(phx, fo, 4u) + d8b(phy, fo, SYB) + d8b(phz, fo, SZB);
                        ps = 0.f;                  // only z damped here: psi is not kept
                    }
                    const float hz = a.t.h[2][z];
                    const float hs = hx + hy + hz;
                    float inc = (c0 - umf) + (hs * umf - 4.f * (hx * hy + hy * hz + hz * hx) * c0) + chf * wv;
                    if (hs > 0.f) inc -= 8.f * hx * hy * hz * a.inv_dt * ps;
                    if (at_src) inc += sval;
                    un = (c0 + inc) / (1.f + hs);
                    if (two_axis_cell(hx, hy, hz)) {
                        psw = true;
                        psn = ps + a.dt * un;
                        psf = fb;
                    }
                } else {
                    float inc = (c0 - umf) + chf * wv;
                    if (at_src) inc += sval;
                    un = c0 + inc;
                }
            }
            stn(um, fb, un);                       // 0 outside the grid, as the frame holds
            if constexpr (SNAP) stn(snap, fb, valid_xy ? wv : 0.f);
            if constexpr (REC) {
                if (z == zr) {                     // uniform over the block
                    int pe = rb;
                    while (pe < re && (a.rec_ent[pe].x >> CELL3_BITS) == z) ++pe;
                    xch[tid] = un;
                    __syncthreads();
                    for (int i = rb + tid; i < pe; i += NTH3) {
                        const int2 en = a.rec_ent[i];
                        a.seis[((long long)shot * a.nt + a.k) * a.nrec + en.y] = xch[en.x & ((1 << CELL3_BITS) - 1)];
                    }
                    __syncthreads();
                    rb = pe;
                    zr = rb < re ? a.rec_ent[rb].x >> CELL3_BITS : INT_MAX;
                }
            }
            __builtin_amdgcn_sched_barrier(0);   // keep each plane's loads in its own step
        });
    }
    if (psw) stb(psi, psf, psn);
}

// ------------------------------------------------------------ adjoint pass A
// Same work items and marching, on chat s^{k+2} (its factors one plane ahead).
__global__ __launch_bounds__(NTH3) __attribute__((amdgpu_waves_per_eu(8)))
void ac3_phi_adj_kernel(Ac3PhiAdjArgs a)
{
    constexpr int W = TX3 + 8;
    __shared__ float pc[2][(TY3 + 8) * W];
    const Grid3 &g = a.g;
    const int w = work_id();
    const int shot = w / a.nitems;
    const int4 it = a.items[w - shot * a.nitems];
    if (it.x < 0) return;                  // padding of the launch order
    const int ty = it.x / g.ntx, tx = it.x - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = it.y, z1 = it.z;
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    const bool layer_xy = ix < g.P || ix >= g.P + g.nx || iy < g.P || iy >= g.P + g.ny;
    const long long zoff = (long long)(z0 + OZ3 - 4) * g.sz;
    const long long zb0 = (long long)shot * g.plane + zoff;
    const float *s2 = a.s2 + zb0;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane + zoff;
    float *b0 = a.b[0] + zb0, *b1 = a.b[1] + zb0, *b2 = a.b[2] + zb0;
    const unsigned SZB = (unsigned)g.sz * 4u;
    auto pb = [&](int z) { return (unsigned)(z - z0 + 4) * SZB; };
    auto pbc = [&](int z) { return pb(min(z, g.NZ + 3)); };
    const unsigned colb = (unsigned)((iy + OY3) * g.sy + ix + OX3) * 4u;
    int rs;
    unsigned rob;
    {
        int r = 0, c = 0;
        if (tid < RING3) ring_rc(tid, r, c);
        rs = tid < RING3 ? r * W + c : -1;
        rob = (unsigned)((y0 - 4 + r + OY3) * g.sy + x0 - 4 + c + OX3) * 4u;
    }
    float q[LZR], wc[LNB], ws[LNB], rc[LNB], rsv[LNB], e0[LNB], e1[LNB], e2[LNB];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const unsigned o = colb + pbc(z0 - 4 + m);
        q[m] = ldb(chat, o) * ldb(s2, o);
    }
#pragma unroll
    for (int d = 0; d < LPD; ++d) {
        const unsigned o = pbc(z0 + d), ow = colb + pbc(z0 + d + 4);
        wc[d] = ldb(chat, ow);
        ws[d] = ldb(s2, ow);
        rc[d] = ldb(chat, rob + o);
        rsv[d] = ldb(s2, rob + o);
        e0[d] = ldb(b0, colb + o);
        e1[d] = ldb(b1, colb + o);
        e2[d] = ldb(b2, colb + o);
    }
    const float px = valid_xy ? a.t.p[0][ix] : 1.f, py = valid_xy ? a.t.p[1][iy] : 1.f;
    bool fw = false;
    float fn0 = 0.f, fn1 = 0.f, fn2 = 0.f;
    unsigned ff = 0;

#pragma unroll 1
    for (int zb = z0; zb < z1; zb += LZR) {
        const int zbo = __builtin_amdgcn_readfirstlane(zb);
        static_for<LZR>([&](auto R) __attribute__((always_inline)) {
            constexpr int r = decltype(R)::value;
            constexpr int c = r % LNB, n = (r + LPD) % LNB;
            const int z = zbo + r;
            if (z >= z1) return;
            if (fw) {
                stb(b0, ff, fn0);
                stb(b1, ff, fn1);
                stb(b2, ff, fn2);
            }
            fw = false;
            q[(r + 8) % LZR] = wc[c] * ws[c];
            float *P = pc[z & 1];
            const int ctr = (ly + 4) * W + lx + 4;
            P[ctr] = q[(r + 4) % LZR];
            if (rs >= 0) P[rs] = rc[c] * rsv[c];
            const unsigned fb = colb + pb(z);
            __syncthreads();
            {
                const unsigned d1 = pbc(z + LPD), dw = colb + pbc(z + 4 + LPD);
                rc[n] = ldb(chat, rob + d1);
                rsv[n] = ldb(s2, rob + d1);
                wc[n] = ldb(chat, dw);
                ws[n] = ldb(s2, dw);
                const unsigned fo = layer_xy || z + LPD < g.P || z + LPD >= g.P + g.nz ? colb + d1 : 0u;
                e0[n] = ldb(b0, fo);
                e1[n] = ldb(b1, fo);
                e2[n] = ldb(b2, fo);
            }
            if (valid_xy && (layer_xy || z < g.P || z >= g.P + g.nz)) {
                float wq[9];
#pragma unroll
                for (int m = 0; m < 9; ++m) wq[m] = q[(r + m) % LZR];
                fn0 = px * e0[c] - d8(P + ctr, 1);
                fn1 = py * e1[c] - d8(P + ctr, W);
                fn2 = a.t.p[2][z] * e2[c] - d8w(wq);
                fw = true;
                ff = fb;
            }
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    if (fw) {
        stb(b0, ff, fn0);
        stb(b1, ff, fn1);
        stb(b2, ff, fn2);
    }
}

// ------------------------------------------------------------ adjoint pass B
// Two launches as in the forward: LAYER tiles take the layer terms on every
// plane; in the others only the z slabs do, with hx = hy = 0 (their x and y
// neighbours are interior too: h = 0, 1/(1+h) = 1), where e is constant.
// The layer terms of axis j need D~_j of r_j = b_j / (1 + h_j) and of
// t_j = h_j r_j:
//   sum_m d_m (2 (ha + hb - h_j) r_j)|_{+m} - (..)|_{-m} = 2 (ha + hb) D~_j r_j - 2 D~_j t_j.
// In LAYER tiles r and t of x (y) are staged in LDS planes with their x (y)
// halo, b_z in a register window whose r and t are formed with the scalar z
// tables.  Operands are prefetched one plane ahead into rings as in the
// forward; chat s^{k+2} enters the window as a product formed one step after
// its two factors arrive.  Addresses are 32-bit byte offsets from per-block
// bases at the chunk's first window plane.
constexpr int APD = 1, ANB = APD + 1, AZR = 10;
static_assert(AZR % ANB == 0 && 8 + APD < AZR, "ring sizes");

template <bool LAYER>
__global__ __launch_bounds__(NTH3) __attribute__((amdgpu_waves_per_eu(LAYER ? 4 : 8)))
void ac3_adj_kernel(Ac3AdjArgs a)
{
    constexpr int W = TX3 + 8;
    constexpr int WX = TX3 + 8, WY = TX3;
    constexpr int NPX = TY3 * WX, NPY = (TY3 + 8) * WY;
    __shared__ float pl[2][(TY3 + 8) * W];
    // per buffer: r_x, t_x (NPX each), r_y, t_y (NPY each)
    __shared__ float sb[LAYER ? 2 * 2 * (NPX + NPY) : 1];
    __shared__ float xch[TX3 * TY3];
    const Grid3 &g = a.g;
    const int nxy = g.ntx * g.nty;
    int cs, ti;
    if (!band_item(a.ntl, cs, ti)) return;
    const int shot = cs / g.nzc, zc = cs - shot * g.nzc, tile = a.tiles[a.t0 + ti];
    const int ty = tile / g.ntx, tx = tile - ty * g.ntx;
    const int x0 = tx * TX3, y0 = ty * TY3, z0 = zc * g.zca, z1 = min(z0 + g.zca, g.NZ);
    const int tid = threadIdx.x, lx = tid % TX3, ly = tid / TX3;
    const int ix = x0 + lx, iy = y0 + ly;
    const bool valid_xy = ix < g.NX && iy < g.NY;
    // bases at plane z0 - 4 of this shot; plane z at byte offset pb(z)
    const long long zb0 = (long long)shot * g.plane + (long long)(z0 + OZ3 - 4) * g.sz;
    const float *s2 = a.s2 + zb0;
    float *s3 = a.s3 + zb0;
    float *ee = a.e + zb0;
    float *grad = a.grad + zb0;
    const float *snap = a.snap + zb0;
    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane + (long long)(z0 + OZ3 - 4) * g.sz;
    const float *bxp = a.b[0] + zb0, *byp = a.b[1] + zb0, *bzp = a.b[2] + zb0;
    const unsigned SZB = (unsigned)g.sz * 4u, SYB = (unsigned)g.sy * 4u;
    auto pb = [&](int z) { return (unsigned)(z - z0 + 4) * SZB; };
    auto pbc = [&](int z) { return pb(min(z, g.NZ + 3)); };
    const unsigned colb = (unsigned)((iy + OY3) * g.sy + ix + OX3) * 4u;
    // the source cell as (plane, in-plane byte offset)
    const long long src = a.src_f[shot];
    const int srcp = (int)(src / g.sz) - OZ3;
    const unsigned srcc = (unsigned)(src - (long long)(srcp + OZ3) * g.sz) * 4u;

    const int *off = a.rec_off + (long long)shot * (nxy + 1);
    int rb = off[tile], re = off[tile + 1], zr = INT_MAX;
    while (rb < re && (a.rec_ent[rb].x >> CELL3_BITS) < z0) ++rb;
    if (rb < re) zr = a.rec_ent[rb].x >> CELL3_BITS;
    const float *dd = a.dJdd + ((long long)shot * a.nt + a.k) * a.nrec;

    int rs;
    unsigned rob;
    {
        int r = 0, c = 0;
        if (tid < RING3) ring_rc(tid, r, c);
        rs = tid < RING3 ? r * W + c : -1;
        rob = (unsigned)((y0 - 4 + r + OY3) * g.sy + x0 - 4 + c + OX3) * 4u;
    }
    // q: chat s^{k+2} of planes z - 4 .. z + 4 (ring); wc, ws: the factors
    // of plane z + 4 + APD; the other rings: planes z .. z + APD.  The
    // pointwise terms need s^{k+2} at the centre: interior tiles keep it in a
    // window beside q (sw), layer tiles, short of registers, load it again (srv).
    constexpr bool SWIN = !LAYER;
    float q[AZR], sw[SWIN ? AZR : 1], srv[SWIN ? 1 : ANB];
    float wc[ANB], ws[ANB], rc[ANB], rsv[ANB], s3v[ANB], snv[ANB], gv[ANB];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const unsigned o = colb + pbc(z0 - 4 + m);
        const float sv = ldb(s2, o);
        q[m] = ldb(chat, o) * sv;
        if constexpr (SWIN) sw[m] = sv;
    }
#pragma unroll
    for (int d = 0; d < APD; ++d) {
        const unsigned o = pbc(z0 + d), ow = colb + pbc(z0 + d + 4);
        wc[d] = ldb(chat, ow);
        ws[d] = ldb(s2, ow);
        rc[d] = ldb(chat, rob + o);
        rsv[d] = ldb(s2, rob + o);
        if constexpr (!SWIN) srv[d] = ldb(s2, colb + o);
        s3v[d] = ldn(s3, colb + o);
        snv[d] = ldn(snap, colb + o);
        gv[d] = ldn(grad, colb + o);
    }
    // LAYER: b_z window, own b_x, b_y, e, one halo cell of b_x or b_y, and
    // the tables at the own column, row and halo cell
    float bzw[LAYER ? AZR : 1], bxv[ANB], byv[ANB], hbv[ANB], ev[ANB];
    const TwoAxis two = two_axis_tile(g, x0, y0);
    float hxo = 0.f, ihxo = 1.f, hyo = 0.f, ihyo = 1.f, hho = 0.f, ihho = 1.f;
    int hslot = -1;
    const float *hsrc = bxp;
    unsigned hob = colb;
    if constexpr (LAYER) {
#pragma unroll
        for (int m = 0; m < 8 + APD; ++m) bzw[m] = ldb(bzp, colb + pbc(z0 - 4 + m));
        if (tid < 8 * TY3) {
            const int r = tid / 8, c = tid % 8, cx = c < 4 ? c : c + TX3;
            hslot = r * WX + cx;
            hob = (unsigned)((y0 + r + OY3) * g.sy + x0 - 4 + cx + OX3) * 4u;
            tab_at(a.t.h[0], a.t.ih[0], x0 - 4 + cx, g.NX, hho, ihho);
        } else if (tid < 8 * TY3 + 8 * TX3) {
            const int i = tid - 8 * TY3, r = i / TX3, c = i % TX3, ry = r < 4 ? r : r + TY3;
            hslot = 2 * NPX + ry * WY + c;     // r_y plane; t_y follows at + NPY
            hsrc = byp;
            hob = (unsigned)((y0 - 4 + ry + OY3) * g.sy + x0 + c + OX3) * 4u;
            tab_at(a.t.h[1], a.t.ih[1], y0 - 4 + ry, g.NY, hho, ihho);
        }
        tab_at(a.t.h[0], a.t.ih[0], ix, g.NX, hxo, ihxo);
        tab_at(a.t.h[1], a.t.ih[1], iy, g.NY, hyo, ihyo);
#pragma unroll
        for (int d = 0; d < APD; ++d) {
            const unsigned o = pbc(z0 + d);
            bxv[d] = ldb(bxp, colb + o);
            byv[d] = ldb(byp, colb + o);
            hbv[d] = ldb(hsrc, hob + o);
            ev[d] = ldb(ee, two.plane(g, z0 + d) ? colb + o : 0u);
        }
    }
    const float *tz = a.t.h[2], *iz = a.t.ih[2];
    // e^{k+1} of the previous plane, stored at the start of the next
    bool esw = false;
    float esn = 0.f;
    unsigned esf = 0;

#pragma unroll 1
    for (int zb = z0; zb < z1; zb += AZR) {
        const int zbo = __builtin_amdgcn_readfirstlane(zb);
        static_for<AZR>([&](auto R) __attribute__((always_inline)) {
            constexpr int r = decltype(R)::value;
            constexpr int c = r % ANB, n = (r + APD) % ANB;
            const int z = zbo + r;
            if (z >= z1) return;
            if (esw) stb(ee, esf, esn);
            esw = false;
            q[(r + 8) % AZR] = wc[c] * ws[c];
            if constexpr (SWIN) sw[(r + 8) % AZR] = ws[c];
            float *P = pl[z & 1];
            P[(ly + 4) * W + lx + 4] = q[(r + 4) % AZR];
            if (rs >= 0) P[rs] = rc[c] * rsv[c];
            float *SB = sb + (LAYER ? (z & 1) * 2 * (NPX + NPY) : 0);
            if constexpr (LAYER) {
                const float rx = ihxo * bxv[c], ry = ihyo * byv[c], rh = ihho * hbv[c];
                SB[ly * WX + lx + 4] = rx;
                SB[NPX + ly * WX + lx + 4] = hxo * rx;
                SB[2 * NPX + (ly + 4) * WY + lx] = ry;
                SB[2 * NPX + NPY + (ly + 4) * WY + lx] = hyo * ry;
                if (hslot >= 0) {
                    const int o2 = hslot < NPX ? NPX : NPY;
                    SB[hslot] = rh;
                    SB[hslot + o2] = hho * rh;
                }
            }
            const unsigned fb = colb + pb(z);
            __syncthreads();
            {
                const unsigned d1 = pbc(z + APD), dw = pbc(z + 4 + APD);
                rc[n] = ldb(chat, rob + d1);
                rsv[n] = ldb(s2, rob + d1);
                if constexpr (LAYER) {
                    bxv[n] = ldb(bxp, colb + d1);
                    byv[n] = ldb(byp, colb + d1);
                    hbv[n] = ldb(hsrc, hob + d1);
                }
                wc[n] = ldb(chat, colb + dw);
                ws[n] = ldb(s2, colb + dw);
                if constexpr (!SWIN) srv[n] = ldb(s2, colb + d1);
                s3v[n] = ldn(s3, colb + d1);
                snv[n] = ldn(snap, colb + d1);
                gv[n] = ldn(grad, colb + d1);
                if constexpr (LAYER) {
                    bzw[(r + 8 + APD) % AZR] = ldb(bzp, colb + dw);
                    ev[n] = ldb(ee, two.plane(g, z + APD) ? colb + d1 : 0u);
                }
            }
            float qw[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) qw[m] = q[(r + m) % AZR];
            const float *cc = P + (ly + 4) * W + lx + 4;
            float sraw;
            if constexpr (SWIN) sraw = sw[(r + 4) % AZR];
            else sraw = srv[c];
            const float s3f = s3v[c];
            float v = lap3(cc, W, qw);
            bool nearz = false;
            float hs = 0.f;
            if (valid_xy) {
                nearz = LAYER || plane_near_z(g, z);
                if constexpr (LAYER) {
                    const float hz = tz[z];
                    hs = hxo + hyo + hz;
                    const float drx = d8(SB + ly * WX + lx + 4, 1), dtx = d8(SB + NPX + ly * WX + lx + 4, 1);
                    const float dry = d8(SB + 2 * NPX + (ly + 4) * WY + lx, (long long)WY);
                    const float dty = d8(SB + 2 * NPX + NPY + (ly + 4) * WY + lx, (long long)WY);
                    float drz = 0.f, dtz = 0.f;
#pragma unroll
                    for (int m = 1; m <= 4; ++m) {
                        const float rp = iz[z + m] * bzw[(r + 4 + m) % AZR], rm = iz[z - m] * bzw[(r + 4 - m) % AZR];
                        drz += dcoef(m) * (rp - rm);
                        dtz += dcoef(m) * (tz[z + m] * rp - tz[z - m] * rm);
                    }
                    v -= 2.f * ((hyo + hz) * drx + (hz + hxo) * dry + (hxo + hyo) * drz - (dtx + dty + dtz));
                    const float de = 4.f * a.inv_dt * (hyo * hz * drx + hz * hxo * dry + hxo * hyo * drz);
                    if (hs > 0.f) {
                        const float en = ev[c] - 8.f * hxo * hyo * hz * a.inv_dt * sraw - de;
                        esw = two_axis_cell(hxo, hyo, hz);
                        esn = en;
                        esf = fb;
                        v += a.dt * en;
                    }
                    v += sraw + ((sraw - s3f) + (hs * s3f - 4.f * (hxo * hyo + hyo * hz + hz * hxo) * sraw));
                } else if (nearz) {
                    // slab plane of an interior tile; the offset comes from
                    // an opaque copy of z (no strength-reduced addresses)
                    const int zz = __builtin_amdgcn_readfirstlane(z);
                    const unsigned fo = colb + pb(zz);
                    hs = tz[zz];
                    float dq = 0.f;
#pragma unroll
                    for (int m = 1; m <= 4; ++m)
                        dq += dcoef(m) * (tz[zz - m] * iz[zz - m] * ldb(bzp, fo - m * SZB)
                                          - tz[zz + m] * iz[zz + m] * ldb(bzp, fo + m * SZB));
                    v -= 2.f * (hs * (d8b(bxp, fo, 4u) + d8b(byp, fo, SYB)) + dq);
                    v += sraw + ((sraw - s3f) + hs * s3f);
                } else {
                    v += sraw + (sraw - s3f);
                }
            }
            // receiver residual injection (deterministic per cell)
            if (z == zr) {                              // uniform over the block
                int pe = rb;
                while (pe < re && (a.rec_ent[pe].x >> CELL3_BITS) == z) ++pe;
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
                zr = rb < re ? a.rec_ent[rb].x >> CELL3_BITS : INT_MAX;
            }
            const float s1 = valid_xy ? (nearz ? v / (1.f + hs) : v) : 0.f;
            stn(s3, fb, s1);                            // 0 outside the grid, as the frame holds
            stn(grad, fb, valid_xy ? gv[c] + s1 * snv[c] : gv[c]);
            if (a.gwav && z == srcp && colb == srcc) a.gwav[(long long)shot * a.nt + a.k] = s1 * a.src_scale;
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    if (esw) stb(ee, esf, esn);
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
    Ac3PhiArgs b = a;
    b.nitems = a.nfree;
    if (b.nitems > 0) ac3_phi_kernel<false><<<b.nitems * nshots, NTH3, 0, s>>>(b);
    b.items = a.items + a.nfree;
    b.nitems = a.nitems - a.nfree;
    if (b.nitems > 0) ac3_phi_kernel<true><<<b.nitems * nshots, NTH3, 0, s>>>(b);
}

void launch_ac3_phi_adj(const Ac3PhiAdjArgs &a, int nshots, hipStream_t s)
{
    if (a.g.P == 0 || nshots == 0 || a.nitems == 0) return;
    ac3_phi_adj_kernel<<<a.nitems * nshots, NTH3, 0, s>>>(a);
}

template <bool LAYER>
void launch_ac3_fwd_part(Ac3FwdArgs a, int t0, int ntl, hipStream_t s)
{
    a.t0 = t0;
    a.ntl = ntl;
    if (ntl == 0 || a.nshots == 0) return;
    const int nb = band_per(ntl) * NXCD * ((a.g.NZ + a.g.zcf - 1) / a.g.zcf) * a.nshots;
    const bool snap = a.snap != nullptr, rec = a.seis != nullptr;
    if (snap) { if (rec) ac3_fwd_kernel<true, true, LAYER><<<nb, NTH3, 0, s>>>(a); else ac3_fwd_kernel<true, false, LAYER><<<nb, NTH3, 0, s>>>(a); }
    else      { if (rec) ac3_fwd_kernel<false, true, LAYER><<<nb, NTH3, 0, s>>>(a); else ac3_fwd_kernel<false, false, LAYER><<<nb, NTH3, 0, s>>>(a); }
}

void launch_ac3_fwd(const Ac3FwdArgs &a, hipStream_t s)
{
    const int nxy = a.g.ntx * a.g.nty;
    launch_ac3_fwd_part<true>(a, 0, a.nnear, s);
    launch_ac3_fwd_part<false>(a, a.nnear, nxy - a.nnear, s);
}

void launch_ac3_adj(const Ac3AdjArgs &a, hipStream_t s)
{
    const int nxy = a.g.ntx * a.g.nty;
    for (int part = 0; part < 2; ++part) {
        Ac3AdjArgs b = a;
        b.t0 = part ? a.nnear : 0;
        b.ntl = part ? nxy - a.nnear : a.nnear;
        if (b.ntl == 0 || a.nshots == 0) continue;
        const int nb = band_per(b.ntl) * NXCD * a.g.nzc * a.nshots;
        if (part) ac3_adj_kernel<false><<<nb, NTH3, 0, s>>>(b);
        else ac3_adj_kernel<true><<<nb, NTH3, 0, s>>>(b);
    }
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
