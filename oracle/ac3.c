/* ac3.c -- FP64 oracle for the 3-D constant-density acoustic wave equation
 * u_tt = c^2 lap(u) + f with an auxiliary-field PML, and its exact adjoint.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Same paper anchors as the 2-D oracle (Eqs. (1), (4), (5), (12)).  The
 * absorbing layer follows from complex coordinate stretching
 * d_j -> s/(s+zeta_j) d_j of s^2 u = c^2 lap u, multiplied through by
 * (s+zx)(s+zy)(s+zz)/s^3:
 *     u_tt + s1 u_t + s2 u + s3 psi = c^2 (lap u + div phi) + f,  psi_t = u
 *     phij_t = -zj phij + (zsum - 2 zj) d_j u + (prod_{i != j} zi) d_j psi
 * with s1 = zx+zy+zz, s2 = zx zy + zy zz + zz zx, s3 = zx zy zz,
 * zsum - 2 zj = sum of the other two minus zj.  Central differences in time,
 * u first, then psi and phi from the new u:
 *     w^k     = L u^k + sum_j D_j phij^k
 *     u^{k+1} = alpha (beta u^k - gamma u^{k-1} - dt^2 s3 psi^k + C w^k + dt^2 f^k)
 *     psi^{k+1} = psi^k + dt u^{k+1}
 *     phij^{k+1} = [(1 - zj dt/2) phij^k + dt ((zsum - 2 zj) D_j u^{k+1}
 *                   + (prod_{i != j} zi) D_j psi^{k+1})] / (1 + zj dt/2)
 * alpha = 1/(1 + s1 dt/2), beta = 2 - dt^2 s2, gamma = 1 - s1 dt/2,
 * C = dt^2 c^2, f^k = r(t_k)/dx^3 at the source node.
 * State X_k = (u^k, u^{k-1}, phix^k, phiy^k, phiz^k, psi^k).
 *
 * Storage: fields framed by G = 4 zero ghost cells on every side
 * ([iz][iy][ix], x fastest); transposed operators scatter into the frame and
 * then clear the ghosts.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_int.h"

#define G 4
#define NF 6

typedef struct {
    int nx, ny, nz, P, NX, NY, NZ, SX, SY, SZ;
    long N, sy, sz;  /* framed size, strides */
    double dx, dt;
    double *zx, *zy, *zz;
    double *t1, *t2; /* scratch */
} ac3_ctx;

static inline long fi(const ac3_ctx *c, int iz, int iy, int ix)
{
    return (long)(iz + G) * c->sz + (long)(iy + G) * c->sy + ix + G;
}

static inline double lap(const ac3_ctx *c, const double *u, long i)
{
    double s = 3.0 * OR_L8[0] * u[i];
    for (int m = 1; m <= 4; ++m)
        s += OR_L8[m] * (u[i + m] + u[i - m] + u[i + m * c->sy] + u[i - m * c->sy]
                         + u[i + m * c->sz] + u[i - m * c->sz]);
    return s / (c->dx * c->dx);
}

static inline double d1(const ac3_ctx *c, const double *a, long i, int dir)
{
    const long s = dir == 0 ? 1 : (dir == 1 ? c->sy : c->sz);
    double r = 0.0;
    for (int m = 1; m <= 4; ++m) r += OR_D8[m] * (a[i + m * s] - a[i - m * s]);
    return r / c->dx;
}

static void clear_ghosts(const ac3_ctx *c, double *a)
{
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < c->SZ; ++z)
        for (int y = 0; y < c->SY; ++y)
            for (int x = 0; x < c->SX; ++x)
                if (z < G || z >= c->NZ + G || y < G || y >= c->NY + G || x < G || x >= c->NX + G)
                    a[(long)z * c->sz + (long)y * c->sy + x] = 0.0;
}

/* The transposes scatter from plane iz into planes iz-4 .. iz+4.  Planes nine
 * apart reach disjoint planes, so they are taken in nine phases (iz mod 9),
 * the planes of one phase in parallel: no cell is written by two threads, and
 * the order in which a cell receives its terms does not depend on the thread
 * count. */
static void lap_T(const ac3_ctx *c, const double *in, double *out)
{
    const double h2 = c->dx * c->dx;
    for (int ph = 0; ph < 9; ++ph) {
        #pragma omp parallel for schedule(static)
        for (int iz = ph; iz < c->NZ; iz += 9)
            for (int iy = 0; iy < c->NY; ++iy)
                for (int ix = 0; ix < c->NX; ++ix) {
                    long i = fi(c, iz, iy, ix);
                    double v = in[i] / h2;
                    out[i] += 3.0 * OR_L8[0] * v;
                    for (int m = 1; m <= 4; ++m) {
                        out[i + m] += OR_L8[m] * v;
                        out[i - m] += OR_L8[m] * v;
                        out[i + m * c->sy] += OR_L8[m] * v;
                        out[i - m * c->sy] += OR_L8[m] * v;
                        out[i + m * c->sz] += OR_L8[m] * v;
                        out[i - m * c->sz] += OR_L8[m] * v;
                    }
                }
    }
    clear_ghosts(c, out);
}

/* x and y scatters stay in their plane (one phase); z needs nine. */
static void d1_T(const ac3_ctx *c, const double *in, double *out, int dir)
{
    const long s = dir == 0 ? 1 : (dir == 1 ? c->sy : c->sz);
    const int period = dir == 2 ? 9 : 1;
    for (int ph = 0; ph < period; ++ph) {
    #pragma omp parallel for schedule(static)
    for (int iz = ph; iz < c->NZ; iz += period)
        for (int iy = 0; iy < c->NY; ++iy)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, iy, ix);
                for (int m = 1; m <= 4; ++m) {
                    double a = OR_D8[m] * in[i] / c->dx;
                    out[i + m * s] += a;
                    out[i - m * s] -= a;
                }
            }
    }
    clear_ghosts(c, out);
}

static void ctx_init(ac3_ctx *c, const or_grid *g)
{
    c->nx = g->nx; c->ny = g->ny; c->nz = g->nz; c->P = g->npml;
    c->NX = g->nx + 2 * c->P; c->NY = g->ny + 2 * c->P; c->NZ = g->nz + 2 * c->P;
    c->SX = c->NX + 2 * G; c->SY = c->NY + 2 * G; c->SZ = c->NZ + 2 * G;
    c->sy = c->SX; c->sz = (long)c->SX * c->SY;
    c->N = c->sz * c->SZ;
    c->dx = g->dx; c->dt = g->dt;
    c->zx = malloc(sizeof(double) * c->NX);
    c->zy = malloc(sizeof(double) * c->NY);
    c->zz = malloc(sizeof(double) * c->NZ);
    or_zeta_profile(g, g->nx, c->zx);
    or_zeta_profile(g, g->ny, c->zy);
    or_zeta_profile(g, g->nz, c->zz);
    c->t1 = calloc(c->N, sizeof(double));
    c->t2 = calloc(c->N, sizeof(double));
}

static void ctx_free(ac3_ctx *c)
{
    free(c->zx); free(c->zy); free(c->zz); free(c->t1); free(c->t2);
}

static void to_frame(const ac3_ctx *c, const double *a, double *f)
{
    memset(f, 0, sizeof(double) * c->N);
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int iy = 0; iy < c->NY; ++iy)
            memcpy(f + fi(c, iz, iy, 0), a + ((long)iz * c->NY + iy) * c->NX, sizeof(double) * c->NX);
}

static void from_frame(const ac3_ctx *c, const double *f, double *a)
{
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int iy = 0; iy < c->NY; ++iy)
            memcpy(a + ((long)iz * c->NY + iy) * c->NX, f + fi(c, iz, iy, 0), sizeof(double) * c->NX);
}

void or_ac3_pad(const or_grid *g, const double *cphys, double *c_pad,
                double *zeta_x, double *zeta_y, double *zeta_z)
{
    const int P = g->npml, NX = g->nx + 2 * P, NY = g->ny + 2 * P, NZ = g->nz + 2 * P;
    for (int iz = 0; iz < NZ; ++iz)
        for (int iy = 0; iy < NY; ++iy)
            for (int ix = 0; ix < NX; ++ix) {
                int pz = or_clampi(iz - P, 0, g->nz - 1), py = or_clampi(iy - P, 0, g->ny - 1),
                    px = or_clampi(ix - P, 0, g->nx - 1);
                c_pad[((long)iz * NY + iy) * NX + ix] = cphys[((long)pz * g->ny + py) * g->nx + px];
            }
    if (zeta_x) or_zeta_profile(g, g->nx, zeta_x);
    if (zeta_y) or_zeta_profile(g, g->ny, zeta_y);
    if (zeta_z) or_zeta_profile(g, g->nz, zeta_z);
}

/* X, Y: arrays of NF framed fields. */
static void step(const ac3_ctx *c, const double *cf, double *const *X, long src, double src_val,
                 double *const *Y, double *w_out)
{
    const double dt = c->dt;
    const double *u = X[0], *um = X[1], *psi = X[5];
    const double *ph[3] = {X[2], X[3], X[4]};
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int iy = 0; iy < c->NY; ++iy)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, iy, ix);
                double zx = c->zx[ix], zy = c->zy[iy], zz = c->zz[iz];
                double s1 = zx + zy + zz, s2 = zx * zy + zy * zz + zz * zx, s3 = zx * zy * zz;
                double w = lap(c, u, i) + d1(c, ph[0], i, 0) + d1(c, ph[1], i, 1) + d1(c, ph[2], i, 2);
                double alpha = 1.0 / (1.0 + 0.5 * s1 * dt);
                double beta = 2.0 - dt * dt * s2, gamma = 1.0 - 0.5 * s1 * dt;
                double C = dt * dt * cf[i] * cf[i];
                double f = (i == src) ? src_val / (c->dx * c->dx * c->dx) : 0.0;
                Y[0][i] = alpha * (beta * u[i] - gamma * um[i] - dt * dt * s3 * psi[i] + C * w + dt * dt * f);
                Y[5][i] = psi[i] + dt * Y[0][i];
                if (w_out) w_out[i] = w;
            }
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int iy = 0; iy < c->NY; ++iy)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, iy, ix);
                double zeta[3] = {c->zx[ix], c->zy[iy], c->zz[iz]};
                double sum = zeta[0] + zeta[1] + zeta[2];
                for (int j = 0; j < 3; ++j) {
                    double others = sum - zeta[j];
                    double prod = zeta[(j + 1) % 3] * zeta[(j + 2) % 3];
                    Y[2 + j][i] = ((1.0 - 0.5 * zeta[j] * dt) * ph[j][i]
                                   + dt * ((others - zeta[j]) * d1(c, Y[0], i, j) + prod * d1(c, Y[5], i, j)))
                                  / (1.0 + 0.5 * zeta[j] * dt);
                }
            }
    memcpy(Y[1], u, sizeof(double) * c->N);
}

/* Transpose of step's linear map, operation by operation in reverse order.
 * aY: adjoint of the output state; aX: adjoint of the input state. */
static void step_T(const ac3_ctx *c, const double *cf, double *const *X, double *const *aY,
                   double *const *aX, double *gC, long src, double *src_bar)
{
    const double dt = c->dt;
    double *aun = c->t1, *apsin = c->t2;   /* adjoints of u^{k+1}, psi^{k+1} */
    memcpy(aun, aY[0], sizeof(double) * c->N);
    memcpy(apsin, aY[5], sizeof(double) * c->N);
    memcpy(aX[0], aY[1], sizeof(double) * c->N);   /* u^k passes into slot 1 */
    for (int f = 1; f < NF; ++f) memset(aX[f], 0, sizeof(double) * c->N);
    double *q = malloc(sizeof(double) * c->N), *r = malloc(sizeof(double) * c->N);
    /* phij^{k+1} = p phij^k + qj D_j u^{k+1} + rj D_j psi^{k+1} */
    for (int j = 0; j < 3; ++j) {
        memset(q, 0, sizeof(double) * c->N);
        memset(r, 0, sizeof(double) * c->N);
        #pragma omp parallel for schedule(static)
        for (int iz = 0; iz < c->NZ; ++iz)
            for (int iy = 0; iy < c->NY; ++iy)
                for (int ix = 0; ix < c->NX; ++ix) {
                    long i = fi(c, iz, iy, ix);
                    double zeta[3] = {c->zx[ix], c->zy[iy], c->zz[iz]};
                    double sum = zeta[0] + zeta[1] + zeta[2];
                    double den = 1.0 + 0.5 * zeta[j] * dt;
                    aX[2 + j][i] += (1.0 - 0.5 * zeta[j] * dt) / den * aY[2 + j][i];
                    q[i] = dt * (sum - 2.0 * zeta[j]) / den * aY[2 + j][i];
                    r[i] = dt * zeta[(j + 1) % 3] * zeta[(j + 2) % 3] / den * aY[2 + j][i];
                }
        d1_T(c, q, aun, j);
        d1_T(c, r, apsin, j);
    }
    free(q); free(r);
    /* psi^{k+1} = psi^k + dt u^{k+1} */
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < c->N; ++i) { aX[5][i] += apsin[i]; aun[i] += dt * apsin[i]; }
    /* u^{k+1} = alpha (beta u^k - gamma u^{k-1} - dt^2 s3 psi^k + C w^k + ...) */
    double *Ct = c->t2;   /* apsin no longer needed */
    memset(Ct, 0, sizeof(double) * c->N);
    #pragma omp parallel for schedule(static)
    for (int iz = 0; iz < c->NZ; ++iz)
        for (int iy = 0; iy < c->NY; ++iy)
            for (int ix = 0; ix < c->NX; ++ix) {
                long i = fi(c, iz, iy, ix);
                double zx = c->zx[ix], zy = c->zy[iy], zz = c->zz[iz];
                double s1 = zx + zy + zz, s2 = zx * zy + zy * zz + zz * zx, s3 = zx * zy * zz;
                double alpha = 1.0 / (1.0 + 0.5 * s1 * dt);
                double beta = 2.0 - dt * dt * s2, gamma = 1.0 - 0.5 * s1 * dt;
                double C = dt * dt * cf[i] * cf[i];
                double t = alpha * aun[i];
                aX[0][i] += beta * t;
                aX[1][i] += -gamma * t;
                aX[5][i] += -dt * dt * s3 * t;
                Ct[i] = C * t;
                if (gC) gC[i] += t * (lap(c, X[0], i) + d1(c, X[2], i, 0) + d1(c, X[3], i, 1) + d1(c, X[4], i, 2));
                if (src_bar && i == src) *src_bar = t * dt * dt / (c->dx * c->dx * c->dx);
            }
    /* w^k = L u^k + sum_j D_j phij^k */
    lap_T(c, Ct, aX[0]);
    for (int j = 0; j < 3; ++j) d1_T(c, Ct, aX[2 + j], j);
}

void or_ac3_step(const or_grid *g, const double *c_pad, const double *const *X,
                 int64_t src_idx, double src_val, double *const *Xn, double *w_out)
{
    ac3_ctx c;
    ctx_init(&c, g);
    double *F = calloc((2 * NF + 2) * c.N, sizeof(double));
    double *cf = F, *W = F + c.N, *Xf[NF], *Yf[NF];
    for (int f = 0; f < NF; ++f) { Xf[f] = F + (2 + f) * c.N; Yf[f] = F + (2 + NF + f) * c.N; }
    to_frame(&c, c_pad, cf);
    for (int f = 0; f < NF; ++f) to_frame(&c, X[f], Xf[f]);
    long src = -1;
    if (src_idx >= 0) {
        long iz = src_idx / ((long)c.NX * c.NY), rem = src_idx % ((long)c.NX * c.NY);
        src = fi(&c, (int)iz, (int)(rem / c.NX), (int)(rem % c.NX));
    }
    step(&c, cf, Xf, src, src_val, Yf, W);
    for (int f = 0; f < NF; ++f) from_frame(&c, Yf[f], Xn[f]);
    if (w_out) from_frame(&c, W, w_out);
    free(F);
    ctx_free(&c);
}

void or_ac3_step_T(const or_grid *g, const double *c_pad, const double *const *X,
                   const double *const *aXn, double *const *aX, double *gC,
                   int64_t src_idx, double *src_bar)
{
    ac3_ctx c;
    ctx_init(&c, g);
    double *F = calloc((3 * NF + 2) * c.N, sizeof(double));
    double *cf = F, *gf = F + c.N, *Xf[NF], *aYf[NF], *aXf[NF];
    for (int f = 0; f < NF; ++f) {
        Xf[f] = F + (2 + f) * c.N; aYf[f] = F + (2 + NF + f) * c.N; aXf[f] = F + (2 + 2 * NF + f) * c.N;
    }
    to_frame(&c, c_pad, cf);
    for (int f = 0; f < NF; ++f) { to_frame(&c, X[f], Xf[f]); to_frame(&c, aXn[f], aYf[f]); }
    long src = -1;
    if (src_idx >= 0) {
        long iz = src_idx / ((long)c.NX * c.NY), rem = src_idx % ((long)c.NX * c.NY);
        src = fi(&c, (int)iz, (int)(rem / c.NX), (int)(rem % c.NX));
    }
    step_T(&c, cf, Xf, aYf, aXf, gf, src, src_bar);
    for (int f = 0; f < NF; ++f) from_frame(&c, aXf[f], aX[f]);
    if (gC) from_frame(&c, gf, gC);
    free(F);
    ctx_free(&c);
}

static int check_geom3(const or_grid *g, int32_t nshots, const int32_t *src, int32_t nrec, const int32_t *rec)
{
    if (g->ndim != 3 || g->nx < 1 || g->ny < 1 || g->nz < 1 || g->npml < 0 || g->nt < 1) return -1;
    const int n[3] = {g->nx, g->ny, g->nz};
    for (int s = 0; s < nshots; ++s) {
        for (int d = 0; d < 3; ++d)
            if (src[3 * s + d] < 0 || src[3 * s + d] >= n[d]) return -1;
        for (int r = 0; r < nrec; ++r)
            for (int d = 0; d < 3; ++d) {
                int v = rec[((long)s * nrec + r) * 3 + d];
                if (v < 0 || v >= n[d]) return -1;
            }
    }
    return 0;
}

static void run_shot3(const or_grid *g, const double *cf, const int32_t *src, const double *wav,
                      int32_t nrec, const int32_t *rec, double *seis, const double *dJdd,
                      int32_t ckpt, double *gC, double *gwav)
{
    ac3_ctx c;
    ctx_init(&c, g);
    const long N = c.N;
    const int nt = g->nt, P = g->npml;
    const long sidx = fi(&c, src[2] + P, src[1] + P, src[0] + P);
    long *ridx = malloc(sizeof(long) * (nrec > 0 ? nrec : 1));
    for (int r = 0; r < nrec; ++r) ridx[r] = fi(&c, rec[3 * r + 2] + P, rec[3 * r + 1] + P, rec[3 * r] + P);
    const int K = (dJdd && ckpt > 0 && ckpt < nt) ? ckpt : nt;
    const int nseg = (nt + K - 1) / K;
    double *ck = dJdd ? calloc((size_t)nseg * NF * N, sizeof(double)) : NULL;
    double *A = calloc(NF * N, sizeof(double)), *B = calloc(NF * N, sizeof(double));
    double *X[NF], *Y[NF];
    for (int k = 0; k < nt; ++k) {
        for (int f = 0; f < NF; ++f) { X[f] = A + f * N; Y[f] = B + f * N; }
        if (ck && k % K == 0) memcpy(ck + (size_t)(k / K) * NF * N, A, sizeof(double) * NF * N);
        step(&c, cf, X, sidx, wav[k], Y, NULL);
        double *t = A; A = B; B = t;
        if (seis) for (int r = 0; r < nrec; ++r) seis[(long)k * nrec + r] = A[ridx[r]];
    }
    if (dJdd) {
        double *seg = calloc((size_t)K * NF * N, sizeof(double));
        double *L = calloc(NF * N, sizeof(double)), *Ln = calloc(NF * N, sizeof(double));
        for (int s = nseg - 1; s >= 0; --s) {
            int k0 = s * K, k1 = (k0 + K < nt) ? k0 + K : nt;
            memcpy(seg, ck + (size_t)s * NF * N, sizeof(double) * NF * N);
            for (int k = k0; k < k1 - 1; ++k) {
                double *a = seg + (size_t)(k - k0) * NF * N, *b = a + NF * N;
                for (int f = 0; f < NF; ++f) { X[f] = a + f * N; Y[f] = b + f * N; }
                step(&c, cf, X, sidx, wav[k], Y, NULL);
            }
            for (int k = k1 - 1; k >= k0; --k) {
                double *a = seg + (size_t)(k - k0) * NF * N;
                double *aY[NF], *aX[NF];
                for (int f = 0; f < NF; ++f) { X[f] = a + f * N; aY[f] = L + f * N; aX[f] = Ln + f * N; }
                for (int r = 0; r < nrec; ++r) L[ridx[r]] += dJdd[(long)k * nrec + r];
                double sb = 0.0;
                step_T(&c, cf, X, aY, aX, gC, sidx, &sb);
                if (gwav) gwav[k] = sb;
                double *t = L; L = Ln; Ln = t;
            }
        }
        free(seg); free(L); free(Ln);
    }
    free(ck); free(A); free(B); free(ridx);
    ctx_free(&c);
}

static double *framed_velocity3(const or_grid *g, const double *cphys, const ac3_ctx *c)
{
    const long NP = (long)c->NX * c->NY * c->NZ;
    double *cp = malloc(sizeof(double) * NP), *cf = malloc(sizeof(double) * c->N);
    or_ac3_pad(g, cphys, cp, NULL, NULL, NULL);
    to_frame(c, cp, cf);
    free(cp);
    return cf;
}

int or_ac3_forward(const or_grid *g, const double *cphys, int32_t nshots, const int32_t *src,
                   const double *wav, int32_t nrec, const int32_t *rec, double *seis)
{
    if (check_geom3(g, nshots, src, nrec, rec)) return -1;
    ac3_ctx c;
    ctx_init(&c, g);
    double *cf = framed_velocity3(g, cphys, &c);
    for (int s = 0; s < nshots; ++s)
        run_shot3(g, cf, src + 3 * s, wav + (long)s * g->nt, nrec, rec + (long)s * nrec * 3,
                  seis + (long)s * g->nt * nrec, NULL, 0, NULL, NULL);
    free(cf);
    ctx_free(&c);
    return 0;
}

int or_ac3_gradient(const or_grid *g, const double *cphys, int32_t nshots, const int32_t *src,
                    const double *wav, int32_t nrec, const int32_t *rec, const double *dJdd,
                    int32_t ckpt, double *grad_c, double *seis, double *grad_wav)
{
    if (check_geom3(g, nshots, src, nrec, rec)) return -1;
    ac3_ctx c;
    ctx_init(&c, g);
    const int P = g->npml;
    double *cf = framed_velocity3(g, cphys, &c);
    double *gC = calloc(c.N, sizeof(double));
    memset(grad_c, 0, sizeof(double) * g->nx * g->ny * g->nz);
    for (int s = 0; s < nshots; ++s) {
        memset(gC, 0, sizeof(double) * c.N);
        run_shot3(g, cf, src + 3 * s, wav + (long)s * g->nt, nrec, rec + (long)s * nrec * 3,
                  seis ? seis + (long)s * g->nt * nrec : NULL, dJdd + (long)s * g->nt * nrec, ckpt,
                  gC, grad_wav ? grad_wav + (long)s * g->nt : NULL);
        for (int iz = 0; iz < c.NZ; ++iz)
            for (int iy = 0; iy < c.NY; ++iy)
                for (int ix = 0; ix < c.NX; ++ix) {
                    long i = fi(&c, iz, iy, ix);
                    int pz = or_clampi(iz - P, 0, g->nz - 1), py = or_clampi(iy - P, 0, g->ny - 1),
                        px = or_clampi(ix - P, 0, g->nx - 1);
                    grad_c[((long)pz * g->ny + py) * g->nx + px] += 2.0 * g->dt * g->dt * cf[i] * gC[i];
                }
    }
    free(gC); free(cf);
    ctx_free(&c);
    return 0;
}
