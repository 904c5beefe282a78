/* oracle.h -- FP64 CPU oracle for explicit finite-difference wave propagation
 * and its exact adjoint (Zhu, Xu, Darve & Beroza, "A General Approach to
 * Seismic Inversion with Automatic Differentiation").
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never includes, links or
 * calls anything in this directory; only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no source with the
 * GPU path.
 *
 * Conventions (the paper leaves them open; every choice is a stated reading):
 *   - physical model arrays are row-major [iz][ix] (2-D) or [iz][iy][ix]
 *     (3-D), x fastest, 0-based indices, z pointing down;
 *   - the absorbing layer of npml cells is padded OUTSIDE the physical grid on
 *     every side, the model being continued there by edge replication;
 *   - cells beyond the padded grid are zero (rigid outer boundary);
 *   - time level k holds u at t_k = k*dt; u^0 = u^{-1} = 0; step k injects the
 *     wavelet sample r(t_k); seismogram sample k (0-based) is u^{k+1} at the
 *     receivers;
 *   - the misfit is J = 1/2 sum over shots, samples, receivers (and
 *     components) of (d - d_obs)^2, with no dt weight.
 */
#ifndef SEIS_ORACLE_H
#define SEIS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Grid and time-stepping parameters shared by all oracle entry points. */
typedef struct or_grid {
    int32_t ndim;      /* 2 or 3 */
    int32_t nx, ny, nz;/* physical cells (ny = 1 in 2-D) */
    int32_t npml;      /* absorbing-layer width in cells, padded outside */
    int32_t nt;        /* number of time steps */
    double dx;         /* grid spacing, equal along every axis (m) */
    double dt;         /* time step (s) */
    double pml_R;      /* target reflection coefficient of the layer */
    double pml_vmax;   /* reference velocity of the damping profile (m/s) */
    double f0_pml;     /* elastic CPML: frequency of the alpha profile (Hz) */
} or_grid;

/* Ricker wavelet r(t_k) = (1 - 2 pi^2 f0^2 (t_k - t0)^2) exp(-pi^2 f0^2 (t_k - t0)^2),
 * t_k = k*dt, k = 0..nt-1. */
void or_ricker(double f0, double t0, double dt, int32_t nt, double *out);

/* Stencil weights: L8 second derivative (w0..w4), D8 first derivative
 * (d1..d4, slot 0 unused), staggered 4th order (s1, s2). */
void or_stencil_weights(double *l8, double *d8, double *s4);

/* ---------------- acoustic, 2-D ---------------- */

/* Padded velocity (edge replication) and the damping profiles.  c_pad has
 * (nz+2P)*(nx+2P) entries, zeta_x nx+2P, zeta_z nz+2P. */
void or_ac2_pad(const or_grid *g, const double *c, double *c_pad,
                double *zeta_x, double *zeta_z);

/* One linear step X_{k+1} = A X_k (+ source) of the 2-D recursion on the
 * padded grid.  State X = (u^k, u^{k-1}, phix^k, phiz^k), each (NZ*NX).
 * src_idx < 0 disables the source; src_val is r(t_k) (the step multiplies by
 * dt^2/(dx*dz)).  w_out (nullable) receives w^k. */
void or_ac2_step(const or_grid *g, const double *c_pad,
                 const double *u, const double *um, const double *px,
                 const double *pz, int64_t src_idx, double src_val,
                 double *un, double *unm, double *pxn, double *pzn,
                 double *w_out);

/* Exact transpose of or_ac2_step's linear part: given the adjoint of the
 * output state (au_n, aum_n, apx_n, apz_n) return the adjoint of the input
 * state (au, aum, apx, apz).  gC (nullable) accumulates t .* w^k, the
 * derivative with respect to C = dt^2 c^2 on the padded grid, which needs the
 * input state (u, px, pz).  src_bar (nullable) receives dJ/dr(t_k) for the
 * source at src_idx. */
void or_ac2_step_T(const or_grid *g, const double *c_pad,
                   const double *u, const double *px, const double *pz,
                   const double *au_n, const double *aum_n,
                   const double *apx_n, const double *apz_n,
                   double *au, double *aum, double *apx, double *apz,
                   double *gC, int64_t src_idx, double *src_bar);

/* Forward modelling of nshots shots.  src [nshots][2] = (ix, iz) physical,
 * wav [nshots][nt], rec [nshots][nrec][2] = (ix, iz), seis [nshots][nt][nrec].
 * Returns 0 or a negative error. */
int or_ac2_forward(const or_grid *g, const double *c, int32_t nshots,
                   const int32_t *src, const double *wav, int32_t nrec,
                   const int32_t *rec, double *seis);

/* Gradient of J with respect to the physical velocity for the seismogram
 * adjoint dJdd [nshots][nt][nrec] (for the L2 misfit dJdd = d - d_obs).
 * ckpt = segment length of the two-level checkpointing (ckpt >= nt stores
 * every state).  grad_c has nz*nx entries (sum over shots, fixed order).
 * seis (nullable) receives the forward seismograms, grad_wav (nullable)
 * receives dJ/dwavelet [nshots][nt]. */
/* Several source cells per shot (Applications: the Gaussian-footprint
 * earthquake location source and the multi-point rupture): src
 * [nshots][nsrc][2], wav [nshots][nsrc][nt]; each cell j injects
 * dt^2 wav_j(t_k)/dx^2 into u^{k+1} (times the layer's alpha);
 * grad_wav [nshots][nsrc][nt] = dJ/dwav.  nsrc = 1 is the point source of
 * or_ac2_forward / or_ac2_gradient. */
int or_ac2_forward_ms(const or_grid *g, const double *c, int32_t nshots, int32_t nsrc,
                      const int32_t *src, const double *wav, int32_t nrec,
                      const int32_t *rec, double *seis);
int or_ac2_gradient_ms(const or_grid *g, const double *c, int32_t nshots, int32_t nsrc,
                       const int32_t *src, const double *wav, int32_t nrec,
                       const int32_t *rec, const double *dJdd, int32_t ckpt,
                       double *grad_c, double *seis, double *grad_wav);
int or_ac2_gradient(const or_grid *g, const double *c, int32_t nshots,
                    const int32_t *src, const double *wav, int32_t nrec,
                    const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *grad_c, double *seis, double *grad_wav);

/* L2 misfit J = 1/2 sum (pred - obs)^2 and residual r = pred - obs. */
double or_misfit(const double *pred, const double *obs, int64_t n, double *resid);

/* ---------------- acoustic, 2-D, divergence form ---------------- */
/* u_tt = div(c^2 grad u) + f on the staggered grid with CPML (see ad2.c for
 * the scheme).  Padded NZ*NX arrays; state X = (u^k, u^{k-1}, psix, psiz,
 * xix, xiz), 6 fields back to back.  kx, kz: the half-node coefficients
 * (c_i^2 + c_{i+1}^2)/2 of the padded model. */
void or_ad2_coefficients(const or_grid *g, const double *c, double *kx, double *kz);
void or_ad2_step(const or_grid *g, const double *c, const double *X, int64_t src_idx, double src_val,
                 double *Y);
/* Exact transpose of the step's linear part (source excluded) at the state
 * X: aX from aY; gkx, gkz receive this step's dJ/dkx, dJ/dkz. */
void or_ad2_step_T(const or_grid *g, const double *c, const double *X, const double *aY, double *aX,
                   double *gkx, double *gkz);
/* nshots shots of nsrc source nodes each: src [nshots][nsrc][2], wav
 * [nshots][nsrc][nt] (node j injects dt^2 wav_j(t_k)/(dx dz) into u^{k+1}),
 * rec [nshots][nrec][2], seis [nshots][nt][nrec]. */
int or_ad2_forward(const or_grid *g, const double *c, int32_t nshots, int32_t nsrc, const int32_t *src,
                   const double *wav, int32_t nrec, const int32_t *rec, double *seis);
/* dJ/dc (nz*nx), optional seismograms and dJ/dwav [nshots][nsrc][nt] for
 * the seismogram adjoint dJdd [nshots][nt][nrec]; ckpt as for or_ac2_gradient. */
int or_ad2_gradient(const or_grid *g, const double *c, int32_t nshots, int32_t nsrc, const int32_t *src,
                    const double *wav, int32_t nrec, const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *grad_c, double *seis, double *grad_wav);

/* ---------------- acoustic, 3-D ---------------- */
void or_ac3_pad(const or_grid *g, const double *c, double *c_pad,
                double *zeta_x, double *zeta_y, double *zeta_z);
/* State X = (u^k, u^{k-1}, phix^k, phiy^k, phiz^k, psi^k). */
void or_ac3_step(const or_grid *g, const double *c_pad, const double *const *X,
                 int64_t src_idx, double src_val, double *const *Xn,
                 double *w_out);
void or_ac3_step_T(const or_grid *g, const double *c_pad, const double *const *X,
                   const double *const *aXn, double *const *aX, double *gC,
                   int64_t src_idx, double *src_bar);
int or_ac3_forward(const or_grid *g, const double *c, int32_t nshots,
                   const int32_t *src, const double *wav, int32_t nrec,
                   const int32_t *rec, double *seis);
int or_ac3_gradient(const or_grid *g, const double *c, int32_t nshots,
                    const int32_t *src, const double *wav, int32_t nrec,
                    const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *grad_c, double *seis, double *grad_wav);

/* ---------------- elastic, 2-D ---------------- */
/* Model fields on the padded grid: lambda, mu (integer nodes), mu_xz
 * (half-half nodes), bx (half-integer in x), bz (half-integer in z). */
void or_el2_pad(const or_grid *g, const double *vp, const double *vs,
                const double *rho, double *lam, double *mu, double *muxz,
                double *bx, double *bz);
/* State X = (vx, vz, sxx, szz, sxz, m_vx_x, m_vx_z, m_vz_x, m_vz_z,
 *            m_sxx_x, m_sxz_z, m_sxz_x, m_szz_z): 13 fields of NZ*NX. */
#define OR_EL2_NSTATE 13
void or_el2_step(const or_grid *g, const double *const *model,
                 const double *const *X, int64_t src_idx, const double *mt,
                 double src_val, double *const *Xn);
void or_el2_step_T(const or_grid *g, const double *const *model,
                   const double *const *X, const double *const *aXn,
                   double *const *aX, double *const *gmodel, int64_t src_idx,
                   const double *mt, double *src_bar);
/* src [nshots][2] (ix, iz); mt [nshots][3] = (Mxx, Mzz, Mxz);
 * rec [nshots][nrec][2]; seis [nshots][2][nt][nrec] (vx then vz). */
int or_el2_forward(const or_grid *g, const double *vp, const double *vs,
                   const double *rho, int32_t nshots, const int32_t *src,
                   const double *mt, const double *wav, int32_t nrec,
                   const int32_t *rec, double *seis);
/* Gradients with respect to vp, vs and rho (physical grids, nz*nx each). */
int or_el2_gradient(const or_grid *g, const double *vp, const double *vs,
                    const double *rho, int32_t nshots, const int32_t *src,
                    const double *mt, const double *wav, int32_t nrec,
                    const int32_t *rec, const double *dJdd, int32_t ckpt,
                    double *g_vp, double *g_vs, double *g_rho, double *seis);

#ifdef __cplusplus
}
#endif
#endif
