// ac2.hip -- gfx950 kernels of the 2-D acoustic recursion and its adjoint.
//
// Forward step k (paper: U_{k+1} = A(theta) U_k + F_k, Eq. (1); PDE Eq. (11)
// in the constant-density form u_tt = c^2 lap(u) + f with an auxiliary-field
// absorbing layer).  In scaled variables (chat = dt^2 c^2/dx^2, phi~ = dx*phi,
// h = zeta dt/2, L~ and D~ the 8th-order stencils without the 1/dx factors):
//     phi~_j^k = p_j phi~_j^{k-1} + q_j D~_j u^k,  p = (1-h_j)/(1+h_j),
//                                                  q = 2(h_other - h_j)/(1+h_j)
//     w~^k     = L~ u^k + D~_x phi~_x^k + D~_z phi~_z^k
//     u^{k+1}  = alpha (beta u^k - gamma u^{k-1} + chat w~^k + dt^2 f^k)
// with alpha = 1/(1+h_x+h_z), beta = 2 - 4 h_x h_z, gamma = 1 - h_x - h_z.
// The stored state after step k is (u^{k+1}, u^k, phi~^k): phi is updated at
// the start of the next step from the u it needs, so one launch per step does
// the whole update.  A tile needs phi~^k on its cells +-4, hence u^k on +-8:
// tiles near the layer ("PML tiles") load an 8-cell halo and recompute phi on
// the 4-cell ring; interior tiles load a 4-cell halo and skip phi entirely.
//
// Adjoint step k (Eq. (4): lambda_k = A^T lambda_{k+1} + residual; Eq. (5)
// for the gradient), in the alpha-scaled variable s = alpha * dJ/du:
//     b_j^{k+1} = p_j b_j^{k+2} - D~_j(chat s^{k+2})
//     a^{k+1}   = R^T dJ/dd^{k+1} - sum_j D~_j(q_j b_j^{k+1})
//                 + beta s^{k+2} + L~(chat s^{k+2}) - gamma s^{k+3}
//     s^{k+1}   = alpha a^{k+1};   dJ/dchat += s^{k+1} w~^k
// using L~^T = L~ and D~^T = -D~ (zero cells beyond the grid).
#include "sg_internal.h"

namespace sg {

// 8th-order centred weights: second derivative and first derivative.
constexpr float A0 = (float)(-205.0 / 72.0);
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

__device__ __forceinline__ float lap8(const float *c, int W)
{
    return 2.f * A0 * c[0]
         + A1 * ((c[1] + c[-1]) + (c[W] + c[-W]))
         + A2 * ((c[2] + c[-2]) + (c[2 * W] + c[-2 * W]))
         + A3 * ((c[3] + c[-3]) + (c[3 * W] + c[-3 * W]))
         + A4 * ((c[4] + c[-4]) + (c[4 * W] + c[-4 * W]));
}

__device__ __forceinline__ float d8(const float *c, int s)
{
    return D1 * (c[s] - c[-s]) + D2 * (c[2 * s] - c[-2 * s])
         + D3 * (c[3 * s] - c[-3 * s]) + D4 * (c[4 * s] - c[-4 * s]);
}

// Fill the (TZ+2H) x (TX+2H) LDS tile from `src` (one shot's frame) with
// f(value, frame index) -- own cells are loaded by the caller.
template <int H, class Fn>
__device__ __forceinline__ void load_halo(const Grid2 &g, float *lds, int x0, int z0, Fn f)
{
    constexpr int W = TX + 2 * H;
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

template <bool PML, bool SNAP, bool REC>
__global__ __launch_bounds__(NTH) void ac2_fwd_kernel(Ac2FwdArgs a)
{
    constexpr int H = PML ? 8 : 4;
    constexpr int W = TX + 2 * H;
    constexpr int HH = TZ + 2 * H;
    constexpr int WX = TX + 8;
    __shared__ float su[HH * W];
    __shared__ float spx[PML ? TZ * WX : 1];
    __shared__ float spz[PML ? (TZ + 8) * TX : 1];

    const Grid2 &g = a.g;
    const int2 t = a.tiles[blockIdx.x];
    const int shot = blockIdx.y;
    const int x0 = t.x * TX, z0 = t.y * TZ;
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
    load_halo<H>(g, su, x0, z0, [&](long long f) { return u[f]; });
    __syncthreads();

    if constexpr (PML) {
        // phi~_x^k on rows z0.., columns x0-4 .. x0+TX+3
        for (int i = tid; i < TZ * WX; i += NTH) {
            const int r = i / WX, c = i - r * WX;
            const int iz = z0 + r, jx = x0 - 4 + c;
            float v = 0.f;
            if (iz < g.NZ && jx >= 0 && jx < g.NX) {
                const float hx = a.hx[jx], hz = a.hz[iz];
                const float inv = 1.f / (1.f + hx);
                const float p = (1.f - hx) * inv, q = 2.f * (hz - hx) * inv;
                v = p * a.phx_old[so + fidx(g, iz, jx)] + q * d8(su + (r + H) * W + (c - 4 + H), 1);
            }
            spx[i] = v;
        }
        // phi~_z^k on rows z0-4 .. z0+TZ+3, columns x0..
        for (int i = tid; i < (TZ + 8) * TX; i += NTH) {
            const int r = i / TX, c = i - r * TX;
            const int iz = z0 - 4 + r, jx = x0 + c;
            float v = 0.f;
            if (iz >= 0 && iz < g.NZ && jx < g.NX) {
                const float hx = a.hx[jx], hz = a.hz[iz];
                const float inv = 1.f / (1.f + hz);
                const float p = (1.f - hz) * inv, q = 2.f * (hx - hz) * inv;
                v = p * a.phz_old[so + fidx(g, iz, jx)] + q * d8(su + (r - 4 + H) * W + (c + H), W);
            }
            spz[i] = v;
        }
        __syncthreads();
    }

    const float *chat = a.chat + (long long)(shot / a.shots_per_model) * g.plane;
    float *um = a.um + so;
    const long long src = a.src_cell[shot];
    const float sval = a.src_scale * a.wav[(long long)shot * a.nt + a.k];
    float un[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        float w = lap8(su + (r + H) * W + lx + H, W);
        float pxc = 0.f, pzc = 0.f;
        if constexpr (PML) {
            const float *px = spx + r * WX + lx + 4;
            const float *pz = spz + (r + 4) * TX + lx;
            w += d8(px, 1) + d8(pz, TX);
            pxc = px[0];
            pzc = pz[0];
        }
        un[j] = 0.f;
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fidx(g, iz, ix);
            float v;
            if constexpr (PML) {
                const float hx = a.hx[ix], hz = a.hz[iz];
                const float alpha = 1.f / (1.f + hx + hz);
                const float beta = 2.f - 4.f * hx * hz, gamma = 1.f - hx - hz;
                float acc = beta * uc[j] - gamma * um[f] + chat[f] * w;
                if (f == src) acc += sval;
                v = alpha * acc;
                a.phx_new[so + f] = pxc;
                a.phz_new[so + f] = pzc;
            } else {
                float acc = 2.f * uc[j] - um[f] + chat[f] * w;
                if (f == src) acc += sval;
                v = acc;
            }
            um[f] = v;
            un[j] = v;
            if constexpr (SNAP) a.snap[so + f] = w;
        }
    }

    if constexpr (REC) {
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int tile = t.y * g.ntx + t.x;
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

template <bool PML>
__global__ __launch_bounds__(NTH) void ac2_adj_kernel(Ac2AdjArgs a)
{
    constexpr int H = PML ? 8 : 4;
    constexpr int W = TX + 2 * H;
    constexpr int HH = TZ + 2 * H;
    constexpr int WX = TX + 8;
    __shared__ float sc[HH * W];                 // chat * s^{k+2}
    __shared__ float sqx[PML ? TZ * WX : 1];     // q_x * b_x^{k+1}
    __shared__ float sqz[PML ? (TZ + 8) * TX : 1];

    const Grid2 &g = a.g;
    const int2 t = a.tiles[blockIdx.x];
    const int shot = blockIdx.y;
    const int x0 = t.x * TX, z0 = t.y * TZ;
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
    load_halo<H>(g, sc, x0, z0, [&](long long f) { return chat[f] * s2[f]; });
    __syncthreads();

    if constexpr (PML) {
        for (int i = tid; i < TZ * WX; i += NTH) {
            const int r = i / WX, c = i - r * WX;
            const int iz = z0 + r, jx = x0 - 4 + c;
            float v = 0.f;
            if (iz < g.NZ && jx >= 0 && jx < g.NX) {
                const float hx = a.hx[jx], hz = a.hz[iz];
                const float inv = 1.f / (1.f + hx);
                const float p = (1.f - hx) * inv, q = 2.f * (hz - hx) * inv;
                const long long f = so + fidx(g, iz, jx);
                const float bn = p * a.bx_old[f] - d8(sc + (r + H) * W + (c - 4 + H), 1);
                if (c >= 4 && c < TX + 4) a.bx_new[f] = bn;
                v = q * bn;
            }
            sqx[i] = v;
        }
        for (int i = tid; i < (TZ + 8) * TX; i += NTH) {
            const int r = i / TX, c = i - r * TX;
            const int iz = z0 - 4 + r, jx = x0 + c;
            float v = 0.f;
            if (iz >= 0 && iz < g.NZ && jx < g.NX) {
                const float hx = a.hx[jx], hz = a.hz[iz];
                const float inv = 1.f / (1.f + hz);
                const float p = (1.f - hz) * inv, q = 2.f * (hx - hz) * inv;
                const long long f = so + fidx(g, iz, jx);
                const float bn = p * a.bz_old[f] - d8(sc + (r - 4 + H) * W + (c + H), W);
                if (r >= 4 && r < TZ + 4) a.bz_new[f] = bn;
                v = q * bn;
            }
            sqz[i] = v;
        }
        __syncthreads();
    }

    float *s3 = a.s3 + so;
    float av[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        float v = lap8(sc + (r + H) * W + lx + H, W);
        if constexpr (PML) v -= d8(sqx + r * WX + lx + 4, 1) + d8(sqz + (r + 4) * TX + lx, TX);
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fidx(g, iz, ix);
            if constexpr (PML) {
                const float hx = a.hx[ix], hz = a.hz[iz];
                v += (2.f - 4.f * hx * hz) * sc2[j] - (1.f - hx - hz) * s3[f];
            } else {
                v += 2.f * sc2[j] - s3[f];
            }
        }
        av[j] = v;
    }

    {   // receiver residual injection R^T dJ/dd^{k+1}, deterministic per cell
        const int ntiles = g.ntx * g.ntz;
        const int *off = a.rec_off + (long long)shot * (ntiles + 1);
        const int tile = t.y * g.ntx + t.x;
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

    const long long src = a.src_cell[shot];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = ly * RPT + j, iz = z0 + r;
        if (iz < g.NZ && ix < g.NX) {
            const long long f = fidx(g, iz, ix);
            float s1 = av[j];
            if constexpr (PML) s1 = s1 / (1.f + a.hx[ix] + a.hz[iz]);
            s3[f] = s1;
            a.grad[so + f] += s1 * a.snap[so + f];
            if (a.gwav && f == src) a.gwav[(long long)shot * a.nt + a.k] = s1 * a.src_scale;
        }
    }
}

void launch_ac2_fwd(const Ac2FwdArgs &a, int ntiles, int nshots, bool pml, hipStream_t s)
{
    if (ntiles == 0 || nshots == 0) return;
    dim3 grid(ntiles, nshots), block(NTH);
    const bool snap = a.snap != nullptr, rec = a.seis != nullptr;
    if (pml) {
        if (snap) { if (rec) ac2_fwd_kernel<true, true, true><<<grid, block, 0, s>>>(a); else ac2_fwd_kernel<true, true, false><<<grid, block, 0, s>>>(a); }
        else      { if (rec) ac2_fwd_kernel<true, false, true><<<grid, block, 0, s>>>(a); else ac2_fwd_kernel<true, false, false><<<grid, block, 0, s>>>(a); }
    } else {
        if (snap) { if (rec) ac2_fwd_kernel<false, true, true><<<grid, block, 0, s>>>(a); else ac2_fwd_kernel<false, true, false><<<grid, block, 0, s>>>(a); }
        else      { if (rec) ac2_fwd_kernel<false, false, true><<<grid, block, 0, s>>>(a); else ac2_fwd_kernel<false, false, false><<<grid, block, 0, s>>>(a); }
    }
}

void launch_ac2_adj(const Ac2AdjArgs &a, int ntiles, int nshots, bool pml, hipStream_t s)
{
    if (ntiles == 0 || nshots == 0) return;
    dim3 grid(ntiles, nshots), block(NTH);
    if (pml) ac2_adj_kernel<true><<<grid, block, 0, s>>>(a);
    else     ac2_adj_kernel<false><<<grid, block, 0, s>>>(a);
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
// dJ/dc(phys) = sum over the model's shots (in order) and over the padded
// cells replicating the physical cell of 2 dt^2 c / dx^2 * dJ/dchat.
__global__ void ac2_finalize_kernel(Grid2 g, int nmodels, int spm, const float *grad,
                                    const float *cpad, double dt, double dx, float *g_vp)
{
    const long long n = (long long)nmodels * g.nz * g.nx;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = i / ((long long)g.nz * g.nx);
        const long long rem = i - m * g.nz * g.nx;
        const int iz = (int)(rem / g.nx), ix = (int)(rem - (long long)iz * g.nx);
        const int zlo = iz == 0 ? 0 : iz + g.P, zhi = iz == g.nz - 1 ? g.NZ - 1 : iz + g.P;
        const int xlo = ix == 0 ? 0 : ix + g.P, xhi = ix == g.nx - 1 ? g.NX - 1 : ix + g.P;
        float acc = 0.f;
        for (int s = 0; s < spm; ++s) {
            const float *gs = grad + (m * spm + s) * g.plane;
            for (int pz = zlo; pz <= zhi; ++pz)
                for (int px = xlo; px <= xhi; ++px)
                    acc += gs[(long long)(pz + OZ) * g.SX + px + OX];
        }
        const double c = cpad[m * g.plane + (long long)(iz + g.P + OZ) * g.SX + ix + g.P + OX];
        g_vp[i] = (float)(2.0 * dt * dt * c / (dx * dx)) * acc;
    }
}

void launch_ac2_finalize(const Grid2 &g, int nmodels, int spm, const float *grad,
                         const float *cpad, double dt, double dx, float *g_vp, hipStream_t s)
{
    const long long n = (long long)nmodels * g.nz * g.nx;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 65536);
    ac2_finalize_kernel<<<blocks, 256, 0, s>>>(g, nmodels, spm, grad, cpad, dt, dx, g_vp);
}

} // namespace sg
