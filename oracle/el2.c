/* el2.c -- FP64 oracle for the 2-D elastic velocity-stress equations on a
 * staggered grid with CPML, and their exact adjoint.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper anchors: the elastic equations, Implementation, Eq. (13)
 * (rho v_i,t = sigma_ij,j + rho f_i;  sigma_ij,t = lambda delta_ij v_k,k +
 * mu (v_i,j + v_j,i), the Kronecker delta being implied), the explicit
 * recursion Eq. (1), the misfit after Eq. (1), the adjoint recursion and
 * gradient Eqs. (4)-(5); parameters lambda, mu, rho (Implementation).
 *
 * Grid (Virieux staggering), every field stored as [iz][ix] on the padded
 * grid, the index naming the node below-left of its position:
 *     sxx, szz at (ix, iz);  vx at (ix+1/2, iz);  vz at (ix, iz+1/2);
 *     sxz at (ix+1/2, iz+1/2).
 * 4th-order staggered differences (weights 9/8, -1/24):
 *     Dp f[i] = (9/8 (f[i+1]-f[i]) - 1/24 (f[i+2]-f[i-1])) / dx   (at i+1/2)
 *     Dm f[i] = (9/8 (f[i]-f[i-1]) - 1/24 (f[i+1]-f[i-2])) / dx   (at i, f at half points)
 * with zero values beyond the padded grid (rigid), so Dm^T = -Dp.
 * Step n (v^{n-1/2}, sigma^n -> v^{n+1/2}, sigma^{n+1}):
 *     vx += dt bx (Dxp sxx + Dzm sxz + m_sxx_x + m_sxz_z)
 *     vz += dt bz (Dxm sxz + Dzp szz + m_sxz_x + m_szz_z)
 *     (memory variables updated first from the same differences:
 *      m = b m + a D(.))
 *     Exx = Dxm vx + m_vx_x,  Ezz = Dzm vz + m_vz_z,  Exz = Dzp vx + m_vx_z + Dxp vz + m_vz_x
 *     sxx += dt ((lam + 2 mu) Exx + lam Ezz) + dt Mxx r(t_n)/(dx dz) at the source
 *     szz += dt (lam Exx + (lam + 2 mu) Ezz) + dt Mzz r(t_n)/(dx dz)
 *     sxz += dt muxz Exz                     + dt Mxz r(t_n)/(dx dz) (at the sxz node)
 * CPML (Roden & Gedney; Komatitsch & Martin, cited by the paper), kappa = 1:
 *     b = exp(-(d + al) dt), a = d (b - 1)/(d + al), d(x) = d0 (x/L)^2,
 *     al(x) = pi f0 (1 - x/L), d0 = 3 vmax ln(1/R) / (2 L), L = npml dx,
 *     x = distance into the layer at the node's own (staggered) position.
 * Model: lam = rho (vp^2 - 2 vs^2), mu = rho vs^2 at integer nodes;
 *     muxz = 4 / sum(1/mu) over the four surrounding integer nodes;
 *     bx = 2/(rho_i + rho_{i+1}), bz = 2/(rho_j + rho_{j+1}); neighbours beyond
 *     the padded grid are the edge values (edge replication continued).
 * Receivers record vx and vz of the receiver cell after each velocity update:
 * seismogram sample n = v^{n+1/2}.
 * State X = (vx, vz, sxx, szz, sxz, m_vx_x, m_vx_z, m_vz_x, m_vz_z,
 *            m_sxx_x, m_sxz_z, m_sxz_x, m_szz_z).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_int.h"

#define G 4
#define NS OR_EL2_NSTATE
enum { VX, VZ, SXX, SZZ, SXZ, MVXX, MVXZ, MVZX, MVZZ, MSXXX, MSXZZ, MSXZX, MSZZZ };
enum { LAM, MU, MUXZ, BX, BZ };   /* model fields */

typedef struct {
    int nx, nz, P, NX, NZ, SX, SZ;
    long N;
    double dx, dt;
    /* CPML coefficients per axis at integer (0) and half (1) positions */
    double *ax[2], *bx[2], *az[2], *bz[2];
} el_ctx;

static inline long fi(const el_ctx *c, int iz, int ix) { return (long)(iz + G) * c->SX + ix + G; }

/* staggered differences along stride s (1 = x, SX = z) */
static inline double Dp(const el_ctx *c, const double *f, long i, long s)
{
    return (OR_S4[0] * (f[i + s] - f[i]) + OR_S4[1] * (f[i + 2 * s] - f[i - s])) / c->dx;
}
static inline double Dm(const el_ctx *c, const double *f, long i, long s)
{
    return (OR_S4[0] * (f[i] - f[i - s]) + OR_S4[1] * (f[i + s] - f[i - 2 * s])) / c->dx;
}
/* transposes as literal scatters: out[j] += weight * in[i].  A z scatter
 * from row iz reaches four consecutive rows, so rows four apart write
 * disjoint rows: they run in four phases (iz mod 4), the rows of a phase in
 * parallel; an x scatter stays in its row (one phase).  No cell is written by
 * two threads and its terms arrive in an order fixed by the phases alone. */
static void Dp_T(const el_ctx *c, const double *in, double *out, long s)
{
    const int period = s == 1 ? 1 : 4;
    for (int ph = 0; ph < period; ++ph) {
        #pragma omp parallel for schedule(static)
        for (int iz = ph; iz < c->NZ; iz += period)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, ix);
                double v = in[i] / c->dx;
                out[i + s] += OR_S4[0] * v; out[i] -= OR_S4[0] * v;
                out[i + 2 * s] += OR_S4[1] * v; out[i - s] -= OR_S4[1] * v;
            }
    }
}
static void Dm_T(const el_ctx *c, const double *in, double *out, long s)
{
    const int period = s == 1 ? 1 : 4;
    for (int ph = 0; ph < period; ++ph) {
        #pragma omp parallel for schedule(static)
        for (int iz = ph; iz < c->NZ; iz += period)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, ix);
                double v = in[i] / c->dx;
                out[i] += OR_S4[0] * v; out[i - s] -= OR_S4[0] * v;
                out[i + s] += OR_S4[1] * v; out[i - 2 * s] -= OR_S4[1] * v;
            }
    }
}
static void clear_ghosts(const el_ctx *c, double *a)
{
    for (int iz = 0; iz < c->SZ; ++iz)
        for (int ix = 0; ix < c->SX; ++ix)
            if (iz < G || iz >= c->NZ + G || ix < G || ix >= c->NX + G) a[(long)iz * c->SX + ix] = 0.0;
}

static void ctx_init(el_ctx *c, const or_grid *g)
{
    c->nx = g->nx; c->nz = g->nz; c->P = g->npml;
    c->NX = g->nx + 2 * c->P; c->NZ = g->nz + 2 * c->P;
    c->SX = c->NX + 2 * G; c->SZ = c->NZ + 2 * G;
    c->N = (long)c->SX * c->SZ;
    c->dx = g->dx; c->dt = g->dt;
    for (int h = 0; h < 2; ++h) {
        c->ax[h] = malloc(sizeof(double) * c->NX); c->bx[h] = malloc(sizeof(double) * c->NX);
        c->az[h] = malloc(sizeof(double) * c->NZ); c->bz[h] = malloc(sizeof(double) * c->NZ);
        for (int i = 0; i < c->NX; ++i) or_cpml_at(g, g->nx, i + 0.5 * h, &c->ax[h][i], &c->bx[h][i]);
        for (int i = 0; i < c->NZ; ++i) or_cpml_at(g, g->nz, i + 0.5 * h, &c->az[h][i], &c->bz[h][i]);
    }
}

static void ctx_free(el_ctx *c)
{
    for (int h = 0; h < 2; ++h) { free(c->ax[h]); free(c->bx[h]); free(c->az[h]); free(c->bz[h]); }
}

void or_el2_pad(const or_grid *g, const double *vp, const double *vs, const double *rho,
                double *lam, double *mu, double *muxz, double *bx, double *bz)
{
    const int P = g->npml, NX = g->nx + 2 * P, NZ = g->nz + 2 * P;
#define PH(iz, ix) ((long)or_clampi((iz) - P, 0, g->nz - 1) * g->nx + or_clampi((ix) - P, 0, g->nx - 1))
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix) {
            long i = (long)iz * NX + ix;
            double r = rho[PH(iz, ix)], a = vp[PH(iz, ix)], b = vs[PH(iz, ix)];
            lam[i] = r * (a * a - 2.0 * b * b);
            mu[i] = r * b * b;
        }
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix) {
            long i = (long)iz * NX + ix;
            int ix1 = ix + 1 < NX ? ix + 1 : NX - 1, iz1 = iz + 1 < NZ ? iz + 1 : NZ - 1;
            double m00 = mu[i], m01 = mu[(long)iz * NX + ix1], m10 = mu[(long)iz1 * NX + ix], m11 = mu[(long)iz1 * NX + ix1];
            muxz[i] = 4.0 / (1.0 / m00 + 1.0 / m01 + 1.0 / m10 + 1.0 / m11);
            bx[i] = 2.0 / (rho[PH(iz, ix)] + rho[PH(iz, ix1)]);
            bz[i] = 2.0 / (rho[PH(iz, ix)] + rho[PH(iz1, ix)]);
        }
#undef PH
}

/* One step on framed fields.  M: model fields (framed); X, Y: NS fields. */
static void step(const el_ctx *c, double *const *M, double *const *X, long src, const double *mt,
                 double src_val, double *const *Y, double *const *snap)
{
    const double dt = c->dt;
    const long sx = 1, sz = c->SX;
    for (int f = 0; f < NS; ++f) memcpy(Y[f], X[f], sizeof(double) * c->N);
    /* velocity half step with the stress memory variables */
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double dsxx = Dp(c, X[SXX], i, sx), dsxz_z = Dm(c, X[SXZ], i, sz);
            double dsxz_x = Dm(c, X[SXZ], i, sx), dszz = Dp(c, X[SZZ], i, sz);
            /* positions: vx at (ix+1/2, iz), vz at (ix, iz+1/2) */
            Y[MSXXX][i] = c->bx[1][ix] * X[MSXXX][i] + c->ax[1][ix] * dsxx;
            Y[MSXZZ][i] = c->bz[0][iz] * X[MSXZZ][i] + c->az[0][iz] * dsxz_z;
            Y[MSXZX][i] = c->bx[0][ix] * X[MSXZX][i] + c->ax[0][ix] * dsxz_x;
            Y[MSZZZ][i] = c->bz[1][iz] * X[MSZZZ][i] + c->az[1][iz] * dszz;
            double fx = dsxx + dsxz_z + Y[MSXXX][i] + Y[MSXZZ][i];
            double fz = dsxz_x + dszz + Y[MSXZX][i] + Y[MSZZZ][i];
            Y[VX][i] = X[VX][i] + dt * M[BX][i] * fx;
            Y[VZ][i] = X[VZ][i] + dt * M[BZ][i] * fz;
            if (snap) { snap[3][i] = fx; snap[4][i] = fz; }
        }
    /* stress step with the velocity memory variables */
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double dvxx = Dm(c, Y[VX], i, sx), dvzz = Dm(c, Y[VZ], i, sz);
            double dvxz = Dp(c, Y[VX], i, sz), dvzx = Dp(c, Y[VZ], i, sx);
            /* sxx/szz at (ix, iz); sxz at (ix+1/2, iz+1/2) */
            Y[MVXX][i] = c->bx[0][ix] * X[MVXX][i] + c->ax[0][ix] * dvxx;
            Y[MVZZ][i] = c->bz[0][iz] * X[MVZZ][i] + c->az[0][iz] * dvzz;
            Y[MVXZ][i] = c->bz[1][iz] * X[MVXZ][i] + c->az[1][iz] * dvxz;
            Y[MVZX][i] = c->bx[1][ix] * X[MVZX][i] + c->ax[1][ix] * dvzx;
            double exx = dvxx + Y[MVXX][i], ezz = dvzz + Y[MVZZ][i];
            double exz = dvxz + Y[MVXZ][i] + dvzx + Y[MVZX][i];
            double lam = M[LAM][i], mu = M[MU][i];
            Y[SXX][i] = X[SXX][i] + dt * ((lam + 2.0 * mu) * exx + lam * ezz);
            Y[SZZ][i] = X[SZZ][i] + dt * (lam * exx + (lam + 2.0 * mu) * ezz);
            Y[SXZ][i] = X[SXZ][i] + dt * M[MUXZ][i] * exz;
            if (snap) { snap[0][i] = exx; snap[1][i] = ezz; snap[2][i] = exz; }
        }
    if (src >= 0 && mt) {
        double s = dt * src_val / (c->dx * c->dx);
        Y[SXX][src] += s * mt[0];
        Y[SZZ][src] += s * mt[1];
        Y[SXZ][src] += s * mt[2];
    }
}

/* Transpose of step's linear map (source excluded), in reverse order.
 * snapshot-free: the parameter derivatives are formed from the forward
 * state X.  gM (nullable): dJ/d(lam, mu, muxz, bx, bz) accumulated. */
static void step_T(const el_ctx *c, double *const *M, double *const *X, double *const *aY,
                   double *const *aX, double *const *gM, long src, const double *mt, double *src_bar)
{
    const double dt = c->dt;
    const long sx = 1, sz = c->SX;
    double *Y[NS];
    double *work = malloc(sizeof(double) * NS * c->N);
    for (int f = 0; f < NS; ++f) Y[f] = work + f * c->N;
    double *snap[5];
    double *sw = malloc(sizeof(double) * 5 * c->N);
    for (int k = 0; k < 5; ++k) { snap[k] = sw + k * c->N; memset(snap[k], 0, sizeof(double) * c->N); }
    step(c, M, X, -1, NULL, 0.0, Y, snap);           /* recompute intermediate values */
    /* adjoint accumulators of the step's output state; start from aY */
    double *A[NS];
    double *aw = malloc(sizeof(double) * NS * c->N);
    for (int f = 0; f < NS; ++f) { A[f] = aw + f * c->N; memcpy(A[f], aY[f], sizeof(double) * c->N); }
    for (int f = 0; f < NS; ++f) memset(aX[f], 0, sizeof(double) * c->N);
    if (src_bar && src >= 0 && mt)
        *src_bar = dt / (c->dx * c->dx) * (mt[0] * A[SXX][src] + mt[1] * A[SZZ][src] + mt[2] * A[SXZ][src]);
    /* ---- stress step, reversed ---- */
    double *t_exx = calloc(c->N, sizeof(double)), *t_ezz = calloc(c->N, sizeof(double)),
           *t_exz = calloc(c->N, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double lam = M[LAM][i], mu = M[MU][i];
            double axx = A[SXX][i], azz = A[SZZ][i], axz = A[SXZ][i];
            aX[SXX][i] += axx; aX[SZZ][i] += azz; aX[SXZ][i] += axz;
            t_exx[i] = dt * ((lam + 2.0 * mu) * axx + lam * azz);
            t_ezz[i] = dt * (lam * axx + (lam + 2.0 * mu) * azz);
            t_exz[i] = dt * M[MUXZ][i] * axz;
            if (gM) {
                gM[LAM][i] += dt * (snap[0][i] + snap[1][i]) * (axx + azz);
                gM[MU][i] += 2.0 * dt * (snap[0][i] * axx + snap[1][i] * azz);
                gM[MUXZ][i] += dt * snap[2][i] * axz;
            }
            /* exx = dvxx + m_vx_x^new: m^new = b m^old + a dvxx */
            A[MVXX][i] += t_exx[i];
            A[MVZZ][i] += t_ezz[i];
            A[MVXZ][i] += t_exz[i];
            A[MVZX][i] += t_exz[i];
        }
    /* memory variables m^new = b m^old + a D v: adjoint to m^old and to D v */
    double *dvxx_b = calloc(c->N, sizeof(double)), *dvzz_b = calloc(c->N, sizeof(double)),
           *dvxz_b = calloc(c->N, sizeof(double)), *dvzx_b = calloc(c->N, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            aX[MVXX][i] += c->bx[0][ix] * A[MVXX][i];
            aX[MVZZ][i] += c->bz[0][iz] * A[MVZZ][i];
            aX[MVXZ][i] += c->bz[1][iz] * A[MVXZ][i];
            aX[MVZX][i] += c->bx[1][ix] * A[MVZX][i];
            dvxx_b[i] = t_exx[i] + c->ax[0][ix] * A[MVXX][i];
            dvzz_b[i] = t_ezz[i] + c->az[0][iz] * A[MVZZ][i];
            dvxz_b[i] = t_exz[i] + c->az[1][iz] * A[MVXZ][i];
            dvzx_b[i] = t_exz[i] + c->ax[1][ix] * A[MVZX][i];
        }
    /* the differences of the new velocities */
    Dm_T(c, dvxx_b, A[VX], sx);
    Dp_T(c, dvxz_b, A[VX], sz);
    Dm_T(c, dvzz_b, A[VZ], sz);
    Dp_T(c, dvzx_b, A[VZ], sx);
    clear_ghosts(c, A[VX]);
    clear_ghosts(c, A[VZ]);
    /* ---- velocity step, reversed ---- */
    double *fx_b = t_exx, *fz_b = t_ezz;   /* reuse */
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            aX[VX][i] += A[VX][i];
            aX[VZ][i] += A[VZ][i];
            fx_b[i] = dt * M[BX][i] * A[VX][i];
            fz_b[i] = dt * M[BZ][i] * A[VZ][i];
            if (gM) {
                gM[BX][i] += dt * snap[3][i] * A[VX][i];
                gM[BZ][i] += dt * snap[4][i] * A[VZ][i];
            }
            A[MSXXX][i] += fx_b[i]; A[MSXZZ][i] += fx_b[i];
            A[MSXZX][i] += fz_b[i]; A[MSZZZ][i] += fz_b[i];
            aX[MSXXX][i] += c->bx[1][ix] * A[MSXXX][i];
            aX[MSXZZ][i] += c->bz[0][iz] * A[MSXZZ][i];
            aX[MSXZX][i] += c->bx[0][ix] * A[MSXZX][i];
            aX[MSZZZ][i] += c->bz[1][iz] * A[MSZZZ][i];
            dvxx_b[i] = fx_b[i] + c->ax[1][ix] * A[MSXXX][i];   /* d sxx / dx */
            dvzz_b[i] = fx_b[i] + c->az[0][iz] * A[MSXZZ][i];   /* d sxz / dz */
            dvxz_b[i] = fz_b[i] + c->ax[0][ix] * A[MSXZX][i];   /* d sxz / dx */
            dvzx_b[i] = fz_b[i] + c->az[1][iz] * A[MSZZZ][i];   /* d szz / dz */
        }
    Dp_T(c, dvxx_b, aX[SXX], sx);
    Dm_T(c, dvzz_b, aX[SXZ], sz);
    Dm_T(c, dvxz_b, aX[SXZ], sx);
    Dp_T(c, dvzx_b, aX[SZZ], sz);
    for (int f = 0; f < NS; ++f) clear_ghosts(c, aX[f]);
    free(t_exx); free(t_ezz); free(t_exz);
    free(dvxx_b); free(dvzz_b); free(dvxz_b); free(dvzx_b);
    free(work); free(sw); free(aw);
}

static void alloc_model(const or_grid *g, const el_ctx *c, const double *vp, const double *vs,
                        const double *rho, double **Mf)
{
    const long NP = (long)c->NX * c->NZ;
    double *tmp = malloc(sizeof(double) * 5 * NP);
    or_el2_pad(g, vp, vs, rho, tmp, tmp + NP, tmp + 2 * NP, tmp + 3 * NP, tmp + 4 * NP);
    for (int k = 0; k < 5; ++k) {
        Mf[k] = calloc(c->N, sizeof(double));
        for (int iz = 0; iz < c->NZ; ++iz)
            memcpy(Mf[k] + fi(c, iz, 0), tmp + k * NP + (long)iz * c->NX, sizeof(double) * c->NX);
    }
    free(tmp);
}

/* public single-step helpers on framed-free arrays (NZ*NX each) */
static void to_frame(const el_ctx *c, const double *a, double *f)
{
    memset(f, 0, sizeof(double) * c->N);
    for (int iz = 0; iz < c->NZ; ++iz) memcpy(f + fi(c, iz, 0), a + (long)iz * c->NX, sizeof(double) * c->NX);
}
static void from_frame(const el_ctx *c, const double *f, double *a)
{
    for (int iz = 0; iz < c->NZ; ++iz) memcpy(a + (long)iz * c->NX, f + fi(c, iz, 0), sizeof(double) * c->NX);
}

void or_el2_step(const or_grid *g, const double *const *model, const double *const *X,
                 int64_t src_idx, const double *mt, double src_val, double *const *Xn)
{
    el_ctx c;
    ctx_init(&c, g);
    double *F = calloc((5 + 2 * NS) * c.N, sizeof(double));
    double *M[5], *Xf[NS], *Yf[NS];
    for (int k = 0; k < 5; ++k) { M[k] = F + k * c.N; to_frame(&c, model[k], M[k]); }
    for (int f = 0; f < NS; ++f) {
        Xf[f] = F + (5 + f) * c.N; Yf[f] = F + (5 + NS + f) * c.N;
        to_frame(&c, X[f], Xf[f]);
    }
    long src = src_idx >= 0 ? fi(&c, (int)(src_idx / c.NX), (int)(src_idx % c.NX)) : -1;
    step(&c, M, Xf, src, mt, src_val, Yf, NULL);
    for (int f = 0; f < NS; ++f) from_frame(&c, Yf[f], Xn[f]);
    free(F);
    ctx_free(&c);
}

void or_el2_step_T(const or_grid *g, const double *const *model, const double *const *X,
                   const double *const *aXn, double *const *aX, double *const *gmodel,
                   int64_t src_idx, const double *mt, double *src_bar)
{
    el_ctx c;
    ctx_init(&c, g);
    double *F = calloc((10 + 3 * NS) * c.N, sizeof(double));
    double *M[5], *gM[5], *Xf[NS], *aYf[NS], *aXf[NS];
    for (int k = 0; k < 5; ++k) { M[k] = F + k * c.N; gM[k] = F + (5 + k) * c.N; to_frame(&c, model[k], M[k]); }
    for (int f = 0; f < NS; ++f) {
        Xf[f] = F + (10 + f) * c.N; aYf[f] = F + (10 + NS + f) * c.N; aXf[f] = F + (10 + 2 * NS + f) * c.N;
        to_frame(&c, X[f], Xf[f]);
        to_frame(&c, aXn[f], aYf[f]);
    }
    long src = src_idx >= 0 ? fi(&c, (int)(src_idx / c.NX), (int)(src_idx % c.NX)) : -1;
    step_T(&c, M, Xf, aYf, aXf, gM, src, mt, src_bar);
    for (int f = 0; f < NS; ++f) from_frame(&c, aXf[f], aX[f]);
    if (gmodel) for (int k = 0; k < 5; ++k) from_frame(&c, gM[k], gmodel[k]);
    free(F);
    ctx_free(&c);
}

static int check_geom(const or_grid *g, int32_t nshots, const int32_t *src, int32_t nrec, const int32_t *rec)
{
    if (g->ndim != 2 || g->nx < 1 || g->nz < 1 || g->npml < 0 || g->nt < 1) return -1;
    for (int s = 0; s < nshots; ++s) {
        if (src[2 * s] < 0 || src[2 * s] >= g->nx || src[2 * s + 1] < 0 || src[2 * s + 1] >= g->nz) return -1;
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = rec + ((long)s * nrec + r) * 2;
            if (q[0] < 0 || q[0] >= g->nx || q[1] < 0 || q[1] >= g->nz) return -1;
        }
    }
    return 0;
}

static void run_shot(const or_grid *g, double *const *M, const int32_t *src, const double *mt,
                     const double *wav, int32_t nrec, const int32_t *rec, double *seis,
                     const double *dJdd, int32_t ckpt, double *const *gM)
{
    el_ctx c;
    ctx_init(&c, g);
    const long N = c.N;
    const int nt = g->nt, P = g->npml;
    const long sidx = fi(&c, src[1] + P, src[0] + P);
    long *ridx = malloc(sizeof(long) * (nrec > 0 ? nrec : 1));
    for (int r = 0; r < nrec; ++r) ridx[r] = fi(&c, rec[2 * r + 1] + P, rec[2 * r] + P);
    const int K = (dJdd && ckpt > 0 && ckpt < nt) ? ckpt : nt;
    const int nseg = (nt + K - 1) / K;
    double *ck = dJdd ? calloc((size_t)nseg * NS * N, sizeof(double)) : NULL;
    double *A = calloc(NS * N, sizeof(double)), *B = calloc(NS * N, sizeof(double));
    double *X[NS], *Y[NS];
    for (int k = 0; k < nt; ++k) {
        for (int f = 0; f < NS; ++f) { X[f] = A + f * N; Y[f] = B + f * N; }
        if (ck && k % K == 0) memcpy(ck + (size_t)(k / K) * NS * N, A, sizeof(double) * NS * N);
        step(&c, M, X, sidx, mt, wav[k], Y, NULL);
        double *t = A; A = B; B = t;
        if (seis)
            for (int r = 0; r < nrec; ++r) {
                seis[(long)k * nrec + r] = A[VX * N + ridx[r]];
                seis[((long)nt + k) * nrec + r] = A[VZ * N + ridx[r]];
            }
    }
    if (dJdd) {
        double *seg = calloc((size_t)K * NS * N, sizeof(double));
        double *L = calloc(NS * N, sizeof(double)), *Ln = calloc(NS * N, sizeof(double));
        for (int s = nseg - 1; s >= 0; --s) {
            int k0 = s * K, k1 = (k0 + K < nt) ? k0 + K : nt;
            memcpy(seg, ck + (size_t)s * NS * N, sizeof(double) * NS * N);
            for (int k = k0; k < k1 - 1; ++k) {
                double *a = seg + (size_t)(k - k0) * NS * N, *b = a + NS * N;
                for (int f = 0; f < NS; ++f) { X[f] = a + f * N; Y[f] = b + f * N; }
                step(&c, M, X, sidx, mt, wav[k], Y, NULL);
            }
            for (int k = k1 - 1; k >= k0; --k) {
                double *a = seg + (size_t)(k - k0) * NS * N;
                double *aY[NS], *aX[NS];
                for (int f = 0; f < NS; ++f) { X[f] = a + f * N; aY[f] = L + f * N; aX[f] = Ln + f * N; }
                /* sample k is v^{k+1/2}, part of the step's output */
                for (int r = 0; r < nrec; ++r) {
                    L[VX * N + ridx[r]] += dJdd[(long)k * nrec + r];
                    L[VZ * N + ridx[r]] += dJdd[((long)nt + k) * nrec + r];
                }
                step_T(&c, M, X, aY, aX, gM, sidx, mt, NULL);
                double *t = L; L = Ln; Ln = t;
            }
        }
        free(seg); free(L); free(Ln);
    }
    free(ck); free(A); free(B); free(ridx);
    ctx_free(&c);
}

int or_el2_forward(const or_grid *g, const double *vp, const double *vs, const double *rho,
                   int32_t nshots, const int32_t *src, const double *mt, const double *wav,
                   int32_t nrec, const int32_t *rec, double *seis)
{
    if (check_geom(g, nshots, src, nrec, rec)) return -1;
    el_ctx c;
    ctx_init(&c, g);
    double *M[5];
    alloc_model(g, &c, vp, vs, rho, M);
    for (int s = 0; s < nshots; ++s)
        run_shot(g, M, src + 2 * s, mt + 3 * s, wav + (long)s * g->nt, nrec, rec + (long)s * nrec * 2,
                 seis + (long)s * 2 * g->nt * nrec, NULL, 0, NULL);
    for (int k = 0; k < 5; ++k) free(M[k]);
    ctx_free(&c);
    return 0;
}

/* Chain rules: padded (lam, mu, muxz, bx, bz) -> padded (vp, vs, rho) -> fold. */
int or_el2_gradient(const or_grid *g, const double *vp, const double *vs, const double *rho,
                    int32_t nshots, const int32_t *src, const double *mt, const double *wav,
                    int32_t nrec, const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *g_vp, double *g_vs, double *g_rho, double *seis)
{
    if (check_geom(g, nshots, src, nrec, rec)) return -1;
    el_ctx c;
    ctx_init(&c, g);
    double *M[5], *gM[5];
    alloc_model(g, &c, vp, vs, rho, M);
    for (int k = 0; k < 5; ++k) gM[k] = calloc(c.N, sizeof(double));
    for (int s = 0; s < nshots; ++s)
        run_shot(g, M, src + 2 * s, mt + 3 * s, wav + (long)s * g->nt, nrec, rec + (long)s * nrec * 2,
                 seis ? seis + (long)s * 2 * g->nt * nrec : NULL, dJdd + (long)s * 2 * g->nt * nrec, ckpt, gM);
    const int P = g->npml, NX = c.NX, NZ = c.NZ;
    /* padded-grid derivatives with respect to lam, mu and rho */
    double *glam = calloc((long)NX * NZ, sizeof(double)), *gmu = calloc((long)NX * NZ, sizeof(double)),
           *grho = calloc((long)NX * NZ, sizeof(double));
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix) {
            long i = (long)iz * NX + ix, f = fi(&c, iz, ix);
            int ix1 = ix + 1 < NX ? ix + 1 : NX - 1, iz1 = iz + 1 < NZ ? iz + 1 : NZ - 1;
            long n01 = (long)iz * NX + ix1, n10 = (long)iz1 * NX + ix, n11 = (long)iz1 * NX + ix1;
            glam[i] += gM[LAM][f];
            gmu[i] += gM[MU][f];
            /* muxz = 4 / sum 1/mu_k: d muxz / d mu_k = muxz^2 / (4 mu_k^2) */
            double mxz = M[MUXZ][f];
            const long nb[4] = {i, n01, n10, n11};
            const long fb[4] = {f, fi(&c, iz, ix1), fi(&c, iz1, ix), fi(&c, iz1, ix1)};
            for (int q = 0; q < 4; ++q) {
                double mk = M[MU][fb[q]];
                gmu[nb[q]] += gM[MUXZ][f] * mxz * mxz / (4.0 * mk * mk);
            }
            /* bx = 2/(rho_i + rho_{i+1}): d bx / d rho = -bx^2 / 2 for both */
            double bxv = M[BX][f], bzv = M[BZ][f];
            grho[i] += -0.5 * bxv * bxv * gM[BX][f];
            grho[n01] += -0.5 * bxv * bxv * gM[BX][f];
            grho[i] += -0.5 * bzv * bzv * gM[BZ][f];
            grho[n10] += -0.5 * bzv * bzv * gM[BZ][f];
        }
    memset(g_vp, 0, sizeof(double) * g->nx * g->nz);
    memset(g_vs, 0, sizeof(double) * g->nx * g->nz);
    memset(g_rho, 0, sizeof(double) * g->nx * g->nz);
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix) {
            long i = (long)iz * NX + ix;
            long p = (long)or_clampi(iz - P, 0, g->nz - 1) * g->nx + or_clampi(ix - P, 0, g->nx - 1);
            double r = rho[p], a = vp[p], b = vs[p];
            /* lam = rho (vp^2 - 2 vs^2), mu = rho vs^2 */
            g_vp[p] += glam[i] * 2.0 * r * a;
            g_vs[p] += 2.0 * r * b * (gmu[i] - 2.0 * glam[i]);
            g_rho[p] += grho[i] + (a * a - 2.0 * b * b) * glam[i] + b * b * gmu[i];
        }
    free(glam); free(gmu); free(grho);
    for (int k = 0; k < 5; ++k) { free(M[k]); free(gM[k]); }
    ctx_free(&c);
    return 0;
}
