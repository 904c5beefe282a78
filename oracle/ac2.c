/* ac2.c -- FP64 oracle for the 2-D constant-density acoustic wave equation
 * u_tt = c^2 lap(u) + f with an auxiliary-field PML, and its exact adjoint.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper anchors:
 *   - explicit recursion U_k = A(theta) U_{k-1} + F_{k-1}: Method,
 *     "Relationship to the Adjoint Method", Eq. (1);
 *   - misfit J = 1/2 sum_k ||U_k - U_k^obs||^2 (display after Eq. (1)), taken
 *     on the receiver samples;
 *   - adjoint recursion lambda_k = A^T lambda_{k+1} + residual, Eq. (4);
 *   - gradient sum_k lambda_k^T (dA/dtheta) U_{k-1}, Eq. (5) (equal to the
 *     reverse-mode result of Eq. (9) by the Theorem);
 *   - the PDE, Implementation, Eq. (12), read in its constant-density form
 *     c^2 lap(u); the PML is the complex-coordinate-stretched auxiliary-field
 *     family the paper cites (Grote & Sim 2010):
 *         u_tt + (zx+zz) u_t + zx zz u = c^2 (lap u + d_x phix + d_z phiz) + f
 *         phix_t = -zx phix + (zz - zx) d_x u
 *         phiz_t = -zz phiz + (zx - zz) d_z u
 *     discretised by central differences, u first and then phi from the new u.
 *
 * State of the recursion: X_k = (u^k, u^{k-1}, phix^k, phiz^k).
 * The step (alpha = 1/(1+s1 dt/2), beta = 2 - dt^2 s2, gamma = 1 - s1 dt/2,
 * s1 = zx+zz, s2 = zx zz, C = dt^2 c^2, D = 8th-order d/dx, L = 8th-order
 * Laplacian, f^k = r(t_k)/(dx dz) at the source node):
 *     w^k     = L u^k + D_x phix^k + D_z phiz^k
 *     u^{k+1} = alpha (beta u^k - gamma u^{k-1} + C w^k + dt^2 f^k)
 *     phij^{k+1} = [(1 - zj dt/2) phij^k + dt (zother - zj) D_j u^{k+1}] / (1 + zj dt/2)
 *
 * Storage: every field lives in a frame with G = 4 zero ghost cells on each
 * side of the padded grid, so stencils index plainly; the ghost cells stand
 * for the zero values beyond the rigid outer boundary and are never written
 * by a forward operation.  Transposed operators scatter into the frame and
 * then clear the ghost cells (those entries do not exist in the matrix).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_int.h"

#define G 4

typedef struct {
    int nx, nz, P, NX, NZ, SX, SZ; /* SX, SZ: framed extents */
    long N;                        /* framed size */
    double dx, dt;
    double *zx, *zz;               /* damping profiles on the padded grid */
    double *aun, *qx, *qz, *t, *Ct;/* scratch of the transposed step */
} ac2_ctx;

static inline long fi(const ac2_ctx *c, int iz, int ix) { return (long)(iz + G) * c->SX + ix + G; }

/* 8th-order Laplacian at framed index i. */
static inline double lap(const ac2_ctx *c, const double *u, long i)
{
    double sx = OR_L8[0] * u[i], sz = OR_L8[0] * u[i];
    for (int m = 1; m <= 4; ++m) {
        sx += OR_L8[m] * (u[i + m] + u[i - m]);
        sz += OR_L8[m] * (u[i + (long)m * c->SX] + u[i - (long)m * c->SX]);
    }
    return sx / (c->dx * c->dx) + sz / (c->dx * c->dx);
}

/* 8th-order first derivative along x (dir 0) or z (dir 1). */
static inline double d1(const ac2_ctx *c, const double *a, long i, int dir)
{
    const long s = dir == 0 ? 1 : c->SX;
    double r = 0.0;
    for (int m = 1; m <= 4; ++m) r += OR_D8[m] * (a[i + m * s] - a[i - m * s]);
    return r / c->dx;
}

static void clear_ghosts(const ac2_ctx *c, double *a)
{
    for (int iz = 0; iz < c->SZ; ++iz)
        for (int ix = 0; ix < c->SX; ++ix)
            if (iz < G || iz >= c->NZ + G || ix < G || ix >= c->NX + G)
                a[(long)iz * c->SX + ix] = 0.0;
}

/* Transposes, written as literal scatters of the gathered stencils above:
 * every weight a applied at (row i, column j) in the forward becomes
 * out[j] += a * in[i]. */
static void lap_T(const ac2_ctx *c, const double *in, double *out)
{
    const double h2 = c->dx * c->dx;
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double v = in[i] / h2;
            out[i] += 2.0 * OR_L8[0] * v;
            for (int m = 1; m <= 4; ++m) {
                out[i + m] += OR_L8[m] * v;
                out[i - m] += OR_L8[m] * v;
                out[i + (long)m * c->SX] += OR_L8[m] * v;
                out[i - (long)m * c->SX] += OR_L8[m] * v;
            }
        }
    clear_ghosts(c, out);
}

static void d1_T(const ac2_ctx *c, const double *in, double *out, int dir)
{
    const long s = dir == 0 ? 1 : c->SX;
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            for (int m = 1; m <= 4; ++m) {
                double a = OR_D8[m] * in[i] / c->dx;
                out[i + m * s] += a;
                out[i - m * s] -= a;
            }
        }
    clear_ghosts(c, out);
}

static void ctx_init(ac2_ctx *c, const or_grid *g)
{
    c->nx = g->nx; c->nz = g->nz; c->P = g->npml;
    c->NX = g->nx + 2 * g->npml; c->NZ = g->nz + 2 * g->npml;
    c->SX = c->NX + 2 * G; c->SZ = c->NZ + 2 * G;
    c->N = (long)c->SX * c->SZ;
    c->dx = g->dx; c->dt = g->dt;
    c->zx = malloc(sizeof(double) * c->NX);
    c->zz = malloc(sizeof(double) * c->NZ);
    or_zeta_profile(g, g->nx, c->zx);
    or_zeta_profile(g, g->nz, c->zz);
    c->aun = calloc(c->N, sizeof(double)); c->qx = calloc(c->N, sizeof(double));
    c->qz = calloc(c->N, sizeof(double)); c->t = calloc(c->N, sizeof(double));
    c->Ct = calloc(c->N, sizeof(double));
}

static void ctx_free(ac2_ctx *c)
{
    free(c->zx); free(c->zz); free(c->aun); free(c->qx); free(c->qz); free(c->t); free(c->Ct);
}

/* padded grid (NZ*NX) <-> framed storage */
static void to_frame(const ac2_ctx *c, const double *a, double *f)
{
    memset(f, 0, sizeof(double) * c->N);
    for (int iz = 0; iz < c->NZ; ++iz)
        memcpy(f + fi(c, iz, 0), a + (long)iz * c->NX, sizeof(double) * c->NX);
}

static void from_frame(const ac2_ctx *c, const double *f, double *a)
{
    for (int iz = 0; iz < c->NZ; ++iz)
        memcpy(a + (long)iz * c->NX, f + fi(c, iz, 0), sizeof(double) * c->NX);
}

void or_ac2_pad(const or_grid *g, const double *cphys, double *c_pad,
                double *zeta_x, double *zeta_z)
{
    const int P = g->npml, NX = g->nx + 2 * P, NZ = g->nz + 2 * P;
    for (int iz = 0; iz < NZ; ++iz)
        for (int ix = 0; ix < NX; ++ix) {
            int pz = or_clampi(iz - P, 0, g->nz - 1), px = or_clampi(ix - P, 0, g->nx - 1);
            c_pad[(long)iz * NX + ix] = cphys[(long)pz * g->nx + px];
        }
    if (zeta_x) or_zeta_profile(g, g->nx, zeta_x);
    if (zeta_z) or_zeta_profile(g, g->nz, zeta_z);
}

/* Several source cells of one shot (the Gaussian-footprint location source
 * and the multi-point rupture of the Applications section): cell indices
 * and their values at the current step; f = value / dx^2 at each cell. */
typedef struct {
    int n;
    const long *cell;
    const double *val;   /* this step's wavelet value per cell */
} msrc_t;

/* The step; cf is the velocity in framed storage, fields framed.  A point
 * source (src >= 0) enters inside the update; the cells of ms (if any) are
 * added to u^{k+1} (times alpha) before phi is formed from u^{k+1}. */
static void step(const ac2_ctx *c, const double *cf,
                 const double *u, const double *um, const double *px, const double *pz,
                 long src, double src_val, const msrc_t *ms,
                 double *un, double *unm, double *pxn, double *pzn, double *w_out)
{
    const double dt = c->dt;
    /* every cell is independent: rows may run on separate threads */
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double w = lap(c, u, i) + d1(c, px, i, 0) + d1(c, pz, i, 1);
            double s1 = c->zx[ix] + c->zz[iz], s2 = c->zx[ix] * c->zz[iz];
            double alpha = 1.0 / (1.0 + 0.5 * s1 * dt);
            double beta = 2.0 - dt * dt * s2, gamma = 1.0 - 0.5 * s1 * dt;
            double C = dt * dt * cf[i] * cf[i];
            double f = (i == src) ? src_val / (c->dx * c->dx) : 0.0;
            un[i] = alpha * (beta * u[i] - gamma * um[i] + C * w + dt * dt * f);
            if (w_out) w_out[i] = w;
        }
    for (int j = 0; ms && j < ms->n; ++j) {
        const long i = ms->cell[j];
        const int iz = (int)(i / c->SX) - G, ix = (int)(i % c->SX) - G;
        const double alpha = 1.0 / (1.0 + 0.5 * (c->zx[ix] + c->zz[iz]) * dt);
        un[i] += alpha * dt * dt * ms->val[j] / (c->dx * c->dx);
    }
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double zx = c->zx[ix], zz = c->zz[iz];
            pxn[i] = ((1.0 - 0.5 * zx * dt) * px[i] + dt * (zz - zx) * d1(c, un, i, 0)) / (1.0 + 0.5 * zx * dt);
            pzn[i] = ((1.0 - 0.5 * zz * dt) * pz[i] + dt * (zx - zz) * d1(c, un, i, 1)) / (1.0 + 0.5 * zz * dt);
        }
    memcpy(unm, u, sizeof(double) * c->N);
}

/* Transpose of step's linear map (source excluded), operation by operation
 * in reverse order.  Inputs: forward state (u, px, pz) at step k and the
 * adjoint of the step's output (au_n, aum_n, apx_n, apz_n).  Outputs: the
 * adjoint of the step's input (au, aum, apx, apz); gC += t .* w^k;
 * src_bar = dJ/dr(t_k). */
static void step_T(const ac2_ctx *c, const double *cf,
                   const double *u, const double *px, const double *pz,
                   const double *au_n, const double *aum_n, const double *apx_n, const double *apz_n,
                   double *au, double *aum, double *apx, double *apz,
                   double *gC, long src, double *src_bar, const msrc_t *ms, double *ms_bar)
{
    const double dt = c->dt;
    double *aun = c->aun, *qx = c->qx, *qz = c->qz, *t = c->t, *Ct = c->Ct;
    memcpy(aun, au_n, sizeof(double) * c->N);
    /* u^k passes through unchanged into the second state slot */
    memcpy(au, aum_n, sizeof(double) * c->N);
    memset(aum, 0, sizeof(double) * c->N);
    memset(apx, 0, sizeof(double) * c->N);
    memset(apz, 0, sizeof(double) * c->N);
    /* phi update: phij^{k+1} = p_j phij^k + q_j D_j u^{k+1} */
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double zx = c->zx[ix], zz = c->zz[iz];
            apx[i] += (1.0 - 0.5 * zx * dt) / (1.0 + 0.5 * zx * dt) * apx_n[i];
            apz[i] += (1.0 - 0.5 * zz * dt) / (1.0 + 0.5 * zz * dt) * apz_n[i];
            qx[i] = dt * (zz - zx) / (1.0 + 0.5 * zx * dt) * apx_n[i];
            qz[i] = dt * (zx - zz) / (1.0 + 0.5 * zz * dt) * apz_n[i];
        }
    d1_T(c, qx, aun, 0);
    d1_T(c, qz, aun, 1);
    /* u update: u^{k+1} = alpha (beta u^k - gamma u^{k-1} + C w^k + ...) */
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int ix = 0; ix < c->NX; ++ix) {
            long i = fi(c, iz, ix);
            double s1 = c->zx[ix] + c->zz[iz], s2 = c->zx[ix] * c->zz[iz];
            double alpha = 1.0 / (1.0 + 0.5 * s1 * dt);
            double beta = 2.0 - dt * dt * s2, gamma = 1.0 - 0.5 * s1 * dt;
            double C = dt * dt * cf[i] * cf[i];
            t[i] = alpha * aun[i];
            au[i] += beta * t[i];
            aum[i] += -gamma * t[i];
            Ct[i] = C * t[i];
            if (gC) gC[i] += t[i] * (lap(c, u, i) + d1(c, px, i, 0) + d1(c, pz, i, 1));
        }
    if (src_bar && src >= 0) *src_bar = t[src] * dt * dt / (c->dx * c->dx);
    for (int j = 0; ms && ms_bar && j < ms->n; ++j) ms_bar[j] = t[ms->cell[j]] * dt * dt / (c->dx * c->dx);
    /* w^k = L u^k + D_x phix^k + D_z phiz^k */
    lap_T(c, Ct, au);
    d1_T(c, Ct, apx, 0);
    d1_T(c, Ct, apz, 1);
}

/* ---- public single-step entry points (unframed NZ*NX arrays) ---- */
void or_ac2_step(const or_grid *g, const double *c_pad,
                 const double *u, const double *um, const double *px,
                 const double *pz, int64_t src_idx, double src_val,
                 double *un, double *unm, double *pxn, double *pzn,
                 double *w_out)
{
    ac2_ctx c;
    ctx_init(&c, g);
    double *F = calloc(11 * c.N, sizeof(double));
    double *cf = F, *X = F + c.N, *Y = F + 5 * c.N, *W = F + 9 * c.N;
    to_frame(&c, c_pad, cf);
    to_frame(&c, u, X); to_frame(&c, um, X + c.N);
    to_frame(&c, px, X + 2 * c.N); to_frame(&c, pz, X + 3 * c.N);
    long src = -1;
    if (src_idx >= 0) src = fi(&c, (int)(src_idx / c.NX), (int)(src_idx % c.NX));
    step(&c, cf, X, X + c.N, X + 2 * c.N, X + 3 * c.N, src, src_val, NULL,
         Y, Y + c.N, Y + 2 * c.N, Y + 3 * c.N, W);
    from_frame(&c, Y, un); from_frame(&c, Y + c.N, unm);
    from_frame(&c, Y + 2 * c.N, pxn); from_frame(&c, Y + 3 * c.N, pzn);
    if (w_out) from_frame(&c, W, w_out);
    free(F);
    ctx_free(&c);
}

void or_ac2_step_T(const or_grid *g, const double *c_pad,
                   const double *u, const double *px, const double *pz,
                   const double *au_n, const double *aum_n,
                   const double *apx_n, const double *apz_n,
                   double *au, double *aum, double *apx, double *apz,
                   double *gC, int64_t src_idx, double *src_bar)
{
    ac2_ctx c;
    ctx_init(&c, g);
    double *F = calloc(13 * c.N, sizeof(double));
    double *cf = F, *X = F + c.N, *aY = F + 4 * c.N, *aX = F + 8 * c.N, *gf = F + 12 * c.N;
    to_frame(&c, c_pad, cf);
    to_frame(&c, u, X); to_frame(&c, px, X + c.N); to_frame(&c, pz, X + 2 * c.N);
    to_frame(&c, au_n, aY); to_frame(&c, aum_n, aY + c.N);
    to_frame(&c, apx_n, aY + 2 * c.N); to_frame(&c, apz_n, aY + 3 * c.N);
    long src = -1;
    if (src_idx >= 0) src = fi(&c, (int)(src_idx / c.NX), (int)(src_idx % c.NX));
    step_T(&c, cf, X, X + c.N, X + 2 * c.N, aY, aY + c.N, aY + 2 * c.N, aY + 3 * c.N,
           aX, aX + c.N, aX + 2 * c.N, aX + 3 * c.N, gf, src, src_bar, NULL, NULL);
    from_frame(&c, aX, au); from_frame(&c, aX + c.N, aum);
    from_frame(&c, aX + 2 * c.N, apx); from_frame(&c, aX + 3 * c.N, apz);
    if (gC) from_frame(&c, gf, gC);
    free(F);
    ctx_free(&c);
}

static int check_geom(const or_grid *g, int32_t nshots, int32_t nsrc, const int32_t *src,
                      int32_t nrec, const int32_t *rec)
{
    if (g->ndim != 2 || g->nx < 1 || g->nz < 1 || g->npml < 0 || g->nt < 1 || nsrc < 1) return -1;
    for (long j = 0; j < (long)nshots * nsrc; ++j)
        if (src[2 * j] < 0 || src[2 * j] >= g->nx || src[2 * j + 1] < 0 || src[2 * j + 1] >= g->nz) return -1;
    for (int s = 0; s < nshots; ++s) {
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = rec + ((long)s * nrec + r) * 2;
            if (q[0] < 0 || q[0] >= g->nx || q[1] < 0 || q[1] >= g->nz) return -1;
        }
    }
    return 0;
}

/* One shot: forward, then optionally the two-level checkpointed reverse
 * sweep (checkpoints every K steps, each segment recomputed and stored
 * whole; K >= nt stores every state).  cf: framed velocity.  nsrc = 1: a
 * point source (src[2], wav[nt], gwav[nt]); nsrc > 1: source cells src[nsrc][2]
 * with wavelets wav[nsrc][nt] and gradients gwav[nsrc][nt]. */
static void run_shot(const or_grid *g, const double *cf, int32_t nsrc, const int32_t *src,
                     const double *wav, int32_t nrec, const int32_t *rec,
                     double *seis, const double *dJdd, int32_t ckpt,
                     double *gC, double *gwav)
{
    ac2_ctx c;
    ctx_init(&c, g);
    const long N = c.N;
    const int nt = g->nt, P = g->npml;
    const long sidx = nsrc == 1 ? fi(&c, src[1] + P, src[0] + P) : -1;
    long *mcell = malloc(sizeof(long) * nsrc);
    double *mval = malloc(sizeof(double) * nsrc), *mbar = malloc(sizeof(double) * nsrc);
    for (int j = 0; j < nsrc; ++j) mcell[j] = fi(&c, src[2 * j + 1] + P, src[2 * j] + P);
    msrc_t msv = {nsrc, mcell, mval};
    const msrc_t *ms = nsrc > 1 ? &msv : NULL;
    #define SET_MS(k) do { for (int j_ = 0; ms && j_ < nsrc; ++j_) mval[j_] = wav[(long)j_ * nt + (k)]; } while (0)
    long *ridx = malloc(sizeof(long) * (nrec > 0 ? nrec : 1));
    for (int r = 0; r < nrec; ++r) ridx[r] = fi(&c, rec[2 * r + 1] + P, rec[2 * r] + P);

    const int K = (dJdd && ckpt > 0 && ckpt < nt) ? ckpt : nt;
    const int nseg = (nt + K - 1) / K;
    double *ck = dJdd ? calloc((size_t)nseg * 4 * N, sizeof(double)) : NULL;
    double *X = calloc(4 * N, sizeof(double)), *Y = calloc(4 * N, sizeof(double));

    for (int k = 0; k < nt; ++k) {
        if (ck && k % K == 0) memcpy(ck + (size_t)(k / K) * 4 * N, X, sizeof(double) * 4 * N);
        SET_MS(k);
        step(&c, cf, X, X + N, X + 2 * N, X + 3 * N, sidx, nsrc == 1 ? wav[k] : 0.0, ms,
             Y, Y + N, Y + 2 * N, Y + 3 * N, NULL);
        double *tmp = X; X = Y; Y = tmp;
        if (seis) for (int r = 0; r < nrec; ++r) seis[(long)k * nrec + r] = X[ridx[r]];
    }

    if (dJdd) {
        double *seg = calloc((size_t)K * 4 * N, sizeof(double));
        double *L = calloc(4 * N, sizeof(double)), *Ln = calloc(4 * N, sizeof(double));
        for (int s = nseg - 1; s >= 0; --s) {
            int k0 = s * K, k1 = (k0 + K < nt) ? k0 + K : nt;
            memcpy(seg, ck + (size_t)s * 4 * N, sizeof(double) * 4 * N);
            for (int k = k0; k < k1 - 1; ++k) {
                double *a = seg + (size_t)(k - k0) * 4 * N, *b = a + 4 * N;
                SET_MS(k);
                step(&c, cf, a, a + N, a + 2 * N, a + 3 * N, sidx, nsrc == 1 ? wav[k] : 0.0, ms,
                     b, b + N, b + 2 * N, b + 3 * N, NULL);
            }
            for (int k = k1 - 1; k >= k0; --k) {
                const double *a = seg + (size_t)(k - k0) * 4 * N;
                /* the adjoint of X_{k+1} takes the residual of sample k+1,
                 * which is u^{k+1} at the receivers */
                for (int r = 0; r < nrec; ++r) L[ridx[r]] += dJdd[(long)k * nrec + r];
                double sb = 0.0;
                step_T(&c, cf, a, a + 2 * N, a + 3 * N, L, L + N, L + 2 * N, L + 3 * N,
                       Ln, Ln + N, Ln + 2 * N, Ln + 3 * N, gC, sidx, &sb, ms, mbar);
                if (gwav) {
                    if (nsrc == 1) gwav[k] = sb;
                    else for (int j = 0; j < nsrc; ++j) gwav[(long)j * nt + k] = mbar[j];
                }
                double *tmp = L; L = Ln; Ln = tmp;
            }
        }
        free(seg); free(L); free(Ln);
    }
    #undef SET_MS
    free(ck); free(X); free(Y); free(ridx); free(mcell); free(mval); free(mbar); ctx_free(&c);
}

static double *framed_velocity(const or_grid *g, const double *cphys, ac2_ctx *c)
{
    const long NP = (long)c->NX * c->NZ;
    double *cp = malloc(sizeof(double) * NP), *cf = malloc(sizeof(double) * c->N);
    or_ac2_pad(g, cphys, cp, NULL, NULL);
    to_frame(c, cp, cf);
    free(cp);
    return cf;
}

int or_ac2_forward_ms(const or_grid *g, const double *cphys, int32_t nshots, int32_t nsrc,
                      const int32_t *src, const double *wav, int32_t nrec,
                      const int32_t *rec, double *seis)
{
    if (check_geom(g, nshots, nsrc, src, nrec, rec)) return -1;
    ac2_ctx c;
    ctx_init(&c, g);
    double *cf = framed_velocity(g, cphys, &c);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nshots; ++s)
        run_shot(g, cf, nsrc, src + 2L * nsrc * s, wav + (long)s * nsrc * g->nt, nrec, rec + (long)s * nrec * 2,
                 seis + (long)s * g->nt * nrec, NULL, 0, NULL, NULL);
    free(cf);
    ctx_free(&c);
    return 0;
}

int or_ac2_forward(const or_grid *g, const double *cphys, int32_t nshots,
                   const int32_t *src, const double *wav, int32_t nrec,
                   const int32_t *rec, double *seis)
{
    return or_ac2_forward_ms(g, cphys, nshots, 1, src, wav, nrec, rec, seis);
}

int or_ac2_gradient(const or_grid *g, const double *cphys, int32_t nshots,
                    const int32_t *src, const double *wav, int32_t nrec,
                    const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *grad_c, double *seis, double *grad_wav)
{
    return or_ac2_gradient_ms(g, cphys, nshots, 1, src, wav, nrec, rec, dJdd, ckpt, grad_c, seis, grad_wav);
}

int or_ac2_gradient_ms(const or_grid *g, const double *cphys, int32_t nshots, int32_t nsrc,
                       const int32_t *src, const double *wav, int32_t nrec,
                       const int32_t *rec, const double *dJdd, int32_t ckpt,
                       double *grad_c, double *seis, double *grad_wav)
{
    if (check_geom(g, nshots, nsrc, src, nrec, rec)) return -1;
    ac2_ctx c;
    ctx_init(&c, g);
    const int P = g->npml;
    double *cf = framed_velocity(g, cphys, &c);
    double *gC = calloc((size_t)nshots * c.N, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nshots; ++s)
        run_shot(g, cf, nsrc, src + 2L * nsrc * s, wav + (long)s * nsrc * g->nt, nrec, rec + (long)s * nrec * 2,
                 seis ? seis + (long)s * g->nt * nrec : NULL,
                 dJdd + (long)s * g->nt * nrec, ckpt, gC + (size_t)s * c.N,
                 grad_wav ? grad_wav + (long)s * nsrc * g->nt : NULL);
    /* chain rule C = dt^2 c^2 -> dJ/dc = 2 dt^2 c dJ/dC, then fold the padded
     * cells back onto the physical cells they replicate; shots in order */
    memset(grad_c, 0, sizeof(double) * g->nx * g->nz);
    for (int s = 0; s < nshots; ++s)
        for (int iz = 0; iz < c.NZ; ++iz)
            for (int ix = 0; ix < c.NX; ++ix) {
                long i = fi(&c, iz, ix);
                int pz = or_clampi(iz - P, 0, g->nz - 1), px = or_clampi(ix - P, 0, g->nx - 1);
                grad_c[(long)pz * g->nx + px] += 2.0 * g->dt * g->dt * cf[i] * gC[(size_t)s * c.N + i];
            }
    free(gC); free(cf);
    ctx_free(&c);
    return 0;
}
