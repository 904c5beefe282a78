/* ad2.c -- FP64 oracle for the 2-D acoustic wave equation in divergence form,
 * u_tt = div(c^2 grad u) + f, on a staggered grid with CPML, and its exact
 * adjoint.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper anchors: the acoustic equation of the Implementation section,
 * Eq. (12), as printed (divergence form); the staggered-grid finite
 * differences with a convolutional PML named in the same paragraph (Roden &
 * Gedney; Komatitsch & Martin); the explicit recursion Eq. (1), the misfit
 * after it, the adjoint recursion Eq. (4) and the gradient Eq. (5).
 *
 * Grid: u at the integer nodes (ix, iz) of the padded grid; the flux
 * components at half nodes, qx at (ix + 1/2, iz) and qz at (ix, iz + 1/2),
 * each stored at the index of its node (ix, iz).  Half-node fields exist for
 * ix in [0, NX) and iz in [0, NZ) only; every value beyond is zero.
 * 4th-order staggered differences (weights 9/8, -1/24):
 *     Dp u[i] = (9/8 (u[i+1] - u[i]) - 1/24 (u[i+2] - u[i-1])) / dx   (at i + 1/2)
 *     Dm q[i] = (9/8 (q[i] - q[i-1]) - 1/24 (q[i+1] - q[i-2])) / dx   (at i)
 * With both truncated to the same index range, Dm = -Dp^T exactly.
 * Coefficient at half nodes: kx[i] = (c_i^2 + c_{i+1}^2)/2 along x and kz
 * likewise along z; a neighbour beyond the padded grid takes the edge value
 * (edge replication continued, as for the padding itself).
 * CPML (kappa = 1) on both the inner and the outer derivative of each axis,
 * the memory variables updated from the same step's differences:
 *     Gx = Dpx u^n;   psix <- bh_x psix + ah_x Gx;   qx = kx (Gx + psix)
 *     Hx = Dmx qx;    xix  <- b_x xix  + a_x Hx
 *     (z alike)
 *     u^{n+1} = 2 u^n - u^{n-1} + dt^2 (Hx + xix + Hz + xiz) + dt^2 f^n,
 *     f^n = r_j(t_n) / (dx dz) at source node j (several nodes add up).
 * b = exp(-(d + al) dt), a = d (b - 1)/(d + al), d = d0 (x/L)^2,
 * al = pi f0 (1 - x/L), d0 = 3 vmax ln(1/R)/(2L), at integer (b, a) and half
 * (bh, ah) positions, x the distance into the layer.
 * Receivers: seismogram sample n = u^{n+1} at the receiver node.
 * State X_n = (u^n, u^{n-1}, psix, psiz, xix, xiz).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_int.h"

#define G 4
#define NS 6
enum { U, UM, PX, PZ, XX, XZ };

typedef struct {
    int nx, nz, P, NX, NZ, SX, SZ;
    long N;
    double dx, dt;
    double *ax[2], *bx[2], *az[2], *bz[2];   /* [0] integer, [1] half positions */
    double *qx, *qz, *t;                     /* scratch */
    double *aH[2], *aq[2], *aG[2];           /* scratch of the transposed step */
} ad_ctx;

static inline long fi(const ad_ctx *c, int iz, int ix) { return (long)(iz + G) * c->SX + ix + G; }

static void ctx_init(ad_ctx *c, const or_grid *g)
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
    double **s[] = {&c->qx, &c->qz, &c->t, &c->aH[0], &c->aH[1], &c->aq[0], &c->aq[1],
                    &c->aG[0], &c->aG[1]};
    for (size_t i = 0; i < sizeof(s) / sizeof(s[0]); ++i) *s[i] = calloc(c->N, sizeof(double));
}

static void ctx_free(ad_ctx *c)
{
    for (int h = 0; h < 2; ++h) { free(c->ax[h]); free(c->bx[h]); free(c->az[h]); free(c->bz[h]); }
    free(c->qx); free(c->qz); free(c->t);
    for (int a = 0; a < 2; ++a) { free(c->aH[a]); free(c->aq[a]); free(c->aG[a]); }
}

static int inside(const ad_ctx *c, int iz, int ix) { return iz >= 0 && iz < c->NZ && ix >= 0 && ix < c->NX; }

/* Dp along axis a (0: x, 1: z) of a node field at (iz, ix); zero beyond the grid. */
static double dp(const ad_ctx *c, const double *u, int iz, int ix, int a)
{
    const long s = a == 0 ? 1 : c->SX;
    const long i = fi(c, iz, ix);
    return (OR_S4[0] * (u[i + s] - u[i]) + OR_S4[1] * (u[i + 2 * s] - u[i - s])) / c->dx;
}

/* Dm along axis a of a half-node field at node (iz, ix). */
static double dm(const ad_ctx *c, const double *q, int iz, int ix, int a)
{
    const long s = a == 0 ? 1 : c->SX;
    const long i = fi(c, iz, ix);
    return (OR_S4[0] * (q[i] - q[i - s]) + OR_S4[1] * (q[i + s] - q[i - 2 * s])) / c->dx;
}

/* Transposes as literal scatters of the gathered stencils above. */
static void dp_T(const ad_ctx *c, const double *in, double *out, int a)
{
    const long s = a == 0 ? 1 : c->SX;
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const long i = fi(c, iz, ix);
            const double v = in[i] / c->dx;
            out[i + s] += OR_S4[0] * v; out[i] -= OR_S4[0] * v;
            out[i + 2 * s] += OR_S4[1] * v; out[i - s] -= OR_S4[1] * v;
        }
}

static void dm_T(const ad_ctx *c, const double *in, double *out, int a)
{
    const long s = a == 0 ? 1 : c->SX;
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const long i = fi(c, iz, ix);
            const double v = in[i] / c->dx;
            out[i] += OR_S4[0] * v; out[i - s] -= OR_S4[0] * v;
            out[i + s] += OR_S4[1] * v; out[i - 2 * s] -= OR_S4[1] * v;
        }
}

/* zero every entry outside the padded grid (scatters may reach the frame) */
static void clear_outside(const ad_ctx *c, double *a)
{
    for (int iz = -G; iz < c->NZ + G; ++iz)
        for (int ix = -G; ix < c->NX + G; ++ix)
            if (!inside(c, iz, ix)) a[fi(c, iz, ix)] = 0.0;
}

/* Half-node coefficients kx, kz (framed) from the padded velocity (NZ*NX). */
static void coefficients(const ad_ctx *c, const double *cpad, double *kx, double *kz)
{
    memset(kx, 0, sizeof(double) * c->N);
    memset(kz, 0, sizeof(double) * c->N);
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const double c0 = cpad[(long)iz * c->NX + ix];
            const double cx = cpad[(long)iz * c->NX + (ix + 1 < c->NX ? ix + 1 : ix)];
            const double cz = cpad[(long)(iz + 1 < c->NZ ? iz + 1 : iz) * c->NX + ix];
            kx[fi(c, iz, ix)] = 0.5 * (c0 * c0 + cx * cx);
            kz[fi(c, iz, ix)] = 0.5 * (c0 * c0 + cz * cz);
        }
}

typedef struct {
    int n;
    const long *cell;
    const double *val;   /* this step's wavelet value per node */
} srcs_t;

/* The step.  X, Y: NS framed fields; S (optional): the fluxes divided by
 * the coefficient, Sx = Gx + psix^{n+1} and Sz, at the half nodes. */
static void step(const ad_ctx *c, const double *kx, const double *kz, const double *X, const srcs_t *sr,
                 double *Y, double *Sx, double *Sz)
{
    const long N = c->N;
    const double dt = c->dt;
    double *qx = c->qx, *qz = c->qz;
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const long i = fi(c, iz, ix);
            const double gx = dp(c, X + U * N, iz, ix, 0), gz = dp(c, X + U * N, iz, ix, 1);
            const double px = c->bx[1][ix] * X[PX * N + i] + c->ax[1][ix] * gx;
            const double pz = c->bz[1][iz] * X[PZ * N + i] + c->az[1][iz] * gz;
            Y[PX * N + i] = px;
            Y[PZ * N + i] = pz;
            qx[i] = kx[i] * (gx + px);
            qz[i] = kz[i] * (gz + pz);
            if (Sx) { Sx[i] = gx + px; Sz[i] = gz + pz; }
        }
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const long i = fi(c, iz, ix);
            const double hx = dm(c, qx, iz, ix, 0), hz = dm(c, qz, iz, ix, 1);
            const double xx = c->bx[0][ix] * X[XX * N + i] + c->ax[0][ix] * hx;
            const double xz = c->bz[0][iz] * X[XZ * N + i] + c->az[0][iz] * hz;
            Y[XX * N + i] = xx;
            Y[XZ * N + i] = xz;
            Y[U * N + i] = 2.0 * X[U * N + i] - X[UM * N + i] + dt * dt * (hx + xx + hz + xz);
            Y[UM * N + i] = X[U * N + i];
        }
    for (int j = 0; sr && j < sr->n; ++j)
        Y[U * N + sr->cell[j]] += dt * dt * sr->val[j] / (c->dx * c->dx);
}

/* Transpose of the step's linear map, operation by operation in reverse
 * order.  X: forward state at step n; aY: adjoint of the step's output;
 * out: aX, the adjoint of its input.  gkx, gkz += dJ/dkx, dJ/dkz of this
 * step (need Sx, Sz of the same forward step); src_bar[j] = dJ/dr_j(t_n). */
static void step_T(const ad_ctx *c, const double *kx, const double *kz, const double *Sx, const double *Sz,
                   const double *aY, double *aX, double *gkx, double *gkz, const srcs_t *sr, double *src_bar)
{
    const long N = c->N;
    const double dt = c->dt;
    const double *k[2] = {kx, kz}, *S[2] = {Sx, Sz};
    const double *const *a0[2] = {(const double *const *)c->ax, (const double *const *)c->az};
    const double *const *b0[2] = {(const double *const *)c->bx, (const double *const *)c->bz};
    memset(aX, 0, sizeof(double) * NS * N);
    double *t = c->t;
    memcpy(t, aY + U * N, sizeof(double) * N);               /* adjoint of u^{n+1} */
    /* u^{n+1} = 2 u^n - u^{n-1} + dt^2 (Hx + xix + Hz + xiz) + source */
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            const long i = fi(c, iz, ix);
            aX[U * N + i] += 2.0 * t[i] + aY[UM * N + i];   /* u^{n-1} of the output is u^n */
            aX[UM * N + i] -= t[i];
        }
    for (int j = 0; sr && j < sr->n; ++j) src_bar[j] = t[sr->cell[j]] * dt * dt / (c->dx * c->dx);
    for (int a = 0; a < 2; ++a) {
        const int XI = a == 0 ? XX : XZ, PSI = a == 0 ? PX : PZ;
        double *aH = c->aH[a], *aq = c->aq[a], *aG = c->aG[a];
        memset(aH, 0, sizeof(double) * N);
        memset(aq, 0, sizeof(double) * N);
        memset(aG, 0, sizeof(double) * N);
        for (int iz = 0; iz < c->NZ; ++iz)
            for (int ix = 0; ix < c->NX; ++ix) {
                const long i = fi(c, iz, ix);
                const int p = a == 0 ? ix : iz;
                /* xi^{n+1} = b xi^n + a H, and xi^{n+1} enters u^{n+1} with dt^2 */
                const double axi = aY[XI * N + i] + dt * dt * t[i];
                aX[XI * N + i] += b0[a][0][p] * axi;
                aH[i] = dt * dt * t[i] + a0[a][0][p] * axi;
            }
        /* H = Dm q */
        dm_T(c, aH, aq, a);
        clear_outside(c, aq);
        for (int iz = 0; iz < c->NZ; ++iz)
            for (int ix = 0; ix < c->NX; ++ix) {
                const long i = fi(c, iz, ix);
                const int p = a == 0 ? ix : iz;
                /* q = k (G + psi^{n+1}) */
                const double aS = k[a][i] * aq[i];
                if (a == 0) gkx[i] += aq[i] * S[a][i]; else gkz[i] += aq[i] * S[a][i];
                /* psi^{n+1} = bh psi^n + ah G */
                const double apsi = aY[PSI * N + i] + aS;
                aX[PSI * N + i] += b0[a][1][p] * apsi;
                aG[i] = aS + a0[a][1][p] * apsi;
            }
        /* G = Dp u^n */
        dp_T(c, aG, aX + U * N, a);
    }
    clear_outside(c, aX + U * N);
}

/* padded grid (NZ*NX) <-> framed storage */
static void to_frame(const ad_ctx *c, const double *a, double *f)
{
    memset(f, 0, sizeof(double) * c->N);
    for (int iz = 0; iz < c->NZ; ++iz)
        memcpy(f + fi(c, iz, 0), a + (long)iz * c->NX, sizeof(double) * c->NX);
}

static void from_frame(const ad_ctx *c, const double *f, double *a)
{
    for (int iz = 0; iz < c->NZ; ++iz)
        memcpy(a + (long)iz * c->NX, f + fi(c, iz, 0), sizeof(double) * c->NX);
}

static double *padded_velocity(const or_grid *g, const double *cphys)
{
    const int P = g->npml, NX = g->nx + 2 * P, NZ = g->nz + 2 * P;
    double *cp = malloc(sizeof(double) * NX * NZ);
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix)
            cp[(long)iz * NX + ix] = cphys[(long)or_clampi(iz - P, 0, g->nz - 1) * g->nx + or_clampi(ix - P, 0, g->nx - 1)];
    return cp;
}

void or_ad2_coefficients(const or_grid *g, const double *cphys, double *kx, double *kz)
{
    ad_ctx c;
    ctx_init(&c, g);
    double *cp = padded_velocity(g, cphys), *F = malloc(sizeof(double) * 2 * c.N);
    coefficients(&c, cp, F, F + c.N);
    from_frame(&c, F, kx);
    from_frame(&c, F + c.N, kz);
    free(F); free(cp);
    ctx_free(&c);
}

void or_ad2_step(const or_grid *g, const double *cphys, const double *X, int64_t src_idx, double src_val,
                 double *Y)
{
    ad_ctx c;
    ctx_init(&c, g);
    const long NP = (long)c.NX * c.NZ;
    double *cp = padded_velocity(g, cphys);
    double *F = calloc((2 + 2 * NS) * c.N, sizeof(double));
    double *kx = F, *kz = F + c.N, *Xf = F + 2 * c.N, *Yf = Xf + NS * c.N;
    coefficients(&c, cp, kx, kz);
    for (int f = 0; f < NS; ++f) to_frame(&c, X + f * NP, Xf + f * c.N);
    long cell = -1;
    if (src_idx >= 0) cell = fi(&c, (int)(src_idx / c.NX), (int)(src_idx % c.NX));
    srcs_t sr = {1, &cell, &src_val};
    step(&c, kx, kz, Xf, src_idx >= 0 ? &sr : NULL, Yf, NULL, NULL);
    for (int f = 0; f < NS; ++f) from_frame(&c, Yf + f * c.N, Y + f * NP);
    free(F); free(cp);
    ctx_free(&c);
}

void or_ad2_step_T(const or_grid *g, const double *cphys, const double *X, const double *aY, double *aX,
                   double *gkx, double *gkz)
{
    ad_ctx c;
    ctx_init(&c, g);
    const long NP = (long)c.NX * c.NZ;
    double *cp = padded_velocity(g, cphys);
    double *F = calloc((6 + 4 * NS) * c.N, sizeof(double));
    double *kx = F, *kz = F + c.N, *Sx = F + 2 * c.N, *Sz = F + 3 * c.N, *gx = F + 4 * c.N, *gz = F + 5 * c.N;
    double *Xf = F + 6 * c.N, *Yf = Xf + NS * c.N, *aYf = Yf + NS * c.N, *aXs = aYf + NS * c.N;
    coefficients(&c, cp, kx, kz);
    for (int f = 0; f < NS; ++f) {
        to_frame(&c, X + f * NP, Xf + f * c.N);
        to_frame(&c, aY + f * NP, aYf + f * c.N);
    }
    step(&c, kx, kz, Xf, NULL, Yf, Sx, Sz);
    step_T(&c, kx, kz, Sx, Sz, aYf, aXs, gx, gz, NULL, NULL);
    for (int f = 0; f < NS; ++f) from_frame(&c, aXs + f * c.N, aX + f * NP);
    from_frame(&c, gx, gkx);
    from_frame(&c, gz, gkz);
    free(F); free(cp);
    ctx_free(&c);
}

static int check_geom(const or_grid *g, int32_t nshots, int32_t nsrc, const int32_t *src, int32_t nrec,
                      const int32_t *rec)
{
    if (g->ndim != 2 || g->nx < 1 || g->nz < 1 || g->npml < 0 || g->nt < 1 || nsrc < 1 || nrec < 0) return -1;
    for (long j = 0; j < (long)nshots * nsrc; ++j)
        if (src[2 * j] < 0 || src[2 * j] >= g->nx || src[2 * j + 1] < 0 || src[2 * j + 1] >= g->nz) return -1;
    for (long j = 0; j < (long)nshots * nrec; ++j)
        if (rec[2 * j] < 0 || rec[2 * j] >= g->nx || rec[2 * j + 1] < 0 || rec[2 * j + 1] >= g->nz) return -1;
    return 0;
}

/* One shot: forward and optionally the checkpointed reverse sweep
 * (checkpoints every K steps; each segment is recomputed with its states and
 * fluxes kept, then swept backwards).  gkx, gkz accumulate dJ/dk. */
static void run_shot(const or_grid *g, const double *kx, const double *kz, int32_t nsrc, const int32_t *src,
                     const double *wav, int32_t nrec, const int32_t *rec, double *seis, const double *dJdd,
                     int32_t ckpt, double *gkx, double *gkz, double *gwav)
{
    ad_ctx c;
    ctx_init(&c, g);
    const long N = c.N;
    const int nt = g->nt, P = g->npml;
    long *cell = malloc(sizeof(long) * nsrc);
    double *val = malloc(sizeof(double) * nsrc), *bar = malloc(sizeof(double) * nsrc);
    for (int j = 0; j < nsrc; ++j) cell[j] = fi(&c, src[2 * j + 1] + P, src[2 * j] + P);
    srcs_t sr = {nsrc, cell, val};
    long *ridx = malloc(sizeof(long) * (nrec > 0 ? nrec : 1));
    for (int r = 0; r < nrec; ++r) ridx[r] = fi(&c, rec[2 * r + 1] + P, rec[2 * r] + P);
    const int K = (dJdd && ckpt > 0 && ckpt < nt) ? ckpt : nt;
    const int nseg = (nt + K - 1) / K;
    double *ck = dJdd ? calloc((size_t)nseg * NS * N, sizeof(double)) : NULL;
    double *X = calloc(NS * N, sizeof(double)), *Y = calloc(NS * N, sizeof(double));
    for (int k = 0; k < nt; ++k) {
        if (ck && k % K == 0) memcpy(ck + (size_t)(k / K) * NS * N, X, sizeof(double) * NS * N);
        for (int j = 0; j < nsrc; ++j) val[j] = wav[(long)j * nt + k];
        step(&c, kx, kz, X, &sr, Y, NULL, NULL);
        double *tmp = X; X = Y; Y = tmp;
        if (seis) for (int r = 0; r < nrec; ++r) seis[(long)k * nrec + r] = X[U * N + ridx[r]];
    }
    if (dJdd) {
        /* per segment: states X_k (k0..k1) and fluxes S_k (k0..k1-1) */
        double *st = calloc((size_t)(K + 1) * NS * N, sizeof(double));
        double *fl = calloc((size_t)K * 2 * N, sizeof(double));
        double *L = calloc(NS * N, sizeof(double)), *Ln = calloc(NS * N, sizeof(double));
        for (int s = nseg - 1; s >= 0; --s) {
            const int k0 = s * K, k1 = (k0 + K < nt) ? k0 + K : nt;
            memcpy(st, ck + (size_t)s * NS * N, sizeof(double) * NS * N);
            for (int k = k0; k < k1; ++k) {
                for (int j = 0; j < nsrc; ++j) val[j] = wav[(long)j * nt + k];
                double *f = fl + (size_t)(k - k0) * 2 * N;
                step(&c, kx, kz, st + (size_t)(k - k0) * NS * N, &sr, st + (size_t)(k - k0 + 1) * NS * N, f, f + N);
            }
            for (int k = k1 - 1; k >= k0; --k) {
                /* sample k is u^{k+1}: its residual joins the adjoint of X_{k+1} */
                for (int r = 0; r < nrec; ++r) L[U * N + ridx[r]] += dJdd[(long)k * nrec + r];
                const double *f = fl + (size_t)(k - k0) * 2 * N;
                step_T(&c, kx, kz, f, f + N, L, Ln, gkx, gkz, &sr, bar);
                if (gwav) for (int j = 0; j < nsrc; ++j) gwav[(long)j * nt + k] = bar[j];
                double *tmp = L; L = Ln; Ln = tmp;
            }
        }
        free(st); free(fl); free(L); free(Ln);
    }
    free(ck); free(X); free(Y); free(ridx); free(cell); free(val); free(bar);
    ctx_free(&c);
}

int or_ad2_forward(const or_grid *g, const double *cphys, int32_t nshots, int32_t nsrc, const int32_t *src,
                   const double *wav, int32_t nrec, const int32_t *rec, double *seis)
{
    if (check_geom(g, nshots, nsrc, src, nrec, rec)) return -1;
    ad_ctx c;
    ctx_init(&c, g);
    double *cp = padded_velocity(g, cphys), *k = malloc(sizeof(double) * 2 * c.N);
    coefficients(&c, cp, k, k + c.N);
    for (int s = 0; s < nshots; ++s)
        run_shot(g, k, k + c.N, nsrc, src + 2L * nsrc * s, wav + (long)s * nsrc * g->nt, nrec,
                 rec + 2L * nrec * s, seis + (long)s * g->nt * nrec, NULL, 0, NULL, NULL, NULL);
    free(k); free(cp);
    ctx_free(&c);
    return 0;
}

/* dJ/dc on the physical grid: dJ/dkx at half node i feeds c_i and its +x
 * neighbour through kx = (c_i^2 + c_{i+1}^2)/2 (the neighbour beyond the
 * padded grid being c_i itself), then padded cells fold onto the physical
 * cells they replicate; shots in order. */
int or_ad2_gradient(const or_grid *g, const double *cphys, int32_t nshots, int32_t nsrc, const int32_t *src,
                    const double *wav, int32_t nrec, const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *grad_c, double *seis, double *grad_wav)
{
    if (check_geom(g, nshots, nsrc, src, nrec, rec)) return -1;
    ad_ctx c;
    ctx_init(&c, g);
    const int P = g->npml;
    double *cp = padded_velocity(g, cphys), *k = malloc(sizeof(double) * 2 * c.N);
    coefficients(&c, cp, k, k + c.N);
    double *gk = calloc(2 * c.N, sizeof(double));
    for (int s = 0; s < nshots; ++s)
        run_shot(g, k, k + c.N, nsrc, src + 2L * nsrc * s, wav + (long)s * nsrc * g->nt, nrec, rec + 2L * nrec * s,
                 seis ? seis + (long)s * g->nt * nrec : NULL, dJdd + (long)s * g->nt * nrec, ckpt, gk, gk + c.N,
                 grad_wav ? grad_wav + (long)s * nsrc * g->nt : NULL);
    double *gpad = calloc((size_t)c.NX * c.NZ, sizeof(double));
    for (int iz = 0; iz < c.NZ; ++iz)
        for (int ix = 0; ix < c.NX; ++ix) {
            const long i = fi(&c, iz, ix);
            const int jx = ix + 1 < c.NX ? ix + 1 : ix, jz = iz + 1 < c.NZ ? iz + 1 : iz;
            gpad[(long)iz * c.NX + ix] += gk[i] * cp[(long)iz * c.NX + ix];
            gpad[(long)iz * c.NX + jx] += gk[i] * cp[(long)iz * c.NX + jx];
            gpad[(long)iz * c.NX + ix] += gk[c.N + i] * cp[(long)iz * c.NX + ix];
            gpad[(long)jz * c.NX + ix] += gk[c.N + i] * cp[(long)jz * c.NX + ix];
        }
    memset(grad_c, 0, sizeof(double) * g->nx * g->nz);
    for (int iz = 0; iz < c.NZ; ++iz)
        for (int ix = 0; ix < c.NX; ++ix)
            grad_c[(long)or_clampi(iz - P, 0, g->nz - 1) * g->nx + or_clampi(ix - P, 0, g->nx - 1)] +=
                gpad[(long)iz * c.NX + ix];
    free(gpad); free(gk); free(k); free(cp);
    ctx_free(&c);
    return 0;
}
