/* common.c -- oracle pieces shared by all physics: wavelet, stencil weights,
 * damping profile, misfit.  TEST INFRASTRUCTURE ONLY (see oracle.h). */
#include <math.h>
#include "oracle.h"
#include "oracle_int.h"

/* Ricker wavelet, the source time function of the paper's FWI tests
 * (Applications, "Full-waveform Inversion").  t0 is a free parameter. */
void or_ricker(double f0, double t0, double dt, int32_t nt, double *out)
{
    for (int32_t k = 0; k < nt; ++k) {
        double a = M_PI * f0 * (k * dt - t0);
        a = a * a;
        out[k] = (1.0 - 2.0 * a) * exp(-a);
    }
}

/* Centred finite-difference weights (Fornberg's tables):
 *   second derivative, 8th order: -205/72, 8/5, -1/5, 8/315, -1/560;
 *   first derivative, 8th order:  4/5, -1/5, 4/105, -1/280;
 *   staggered first derivative, 4th order: 9/8, -1/24. */
const double OR_L8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
const double OR_D8[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
const double OR_S4[2] = {9.0 / 8.0, -1.0 / 24.0};

void or_stencil_weights(double *l8, double *d8, double *s4)
{
    for (int i = 0; i < 5; ++i) { l8[i] = OR_L8[i]; d8[i] = OR_D8[i]; }
    s4[0] = OR_S4[0]; s4[1] = OR_S4[1];
}

/* Depth of padded index i into the absorbing layer: 0 inside the physical
 * range [P, P+n), 1 on the first layer cell, P on the outermost cell. */
int or_layer_depth(int i, int n, int P)
{
    if (i < P) return P - i;
    if (i >= P + n) return i - (P + n - 1);
    return 0;
}

/* Quadratic damping profile zeta(i) = zeta_max (d_i/P)^2 with
 * zeta_max = 3 vmax ln(1/R) / (2 P dx).  The profile is fixed by the
 * reference velocity pml_vmax and does not depend on the model. */
void or_zeta_profile(const or_grid *g, int n, double *zeta)
{
    const int P = g->npml;
    const double zmax = P > 0 ? 3.0 * g->pml_vmax * log(1.0 / g->pml_R) / (2.0 * P * g->dx) : 0.0;
    for (int i = 0; i < n + 2 * P; ++i) {
        double r = P > 0 ? (double)or_layer_depth(i, n, P) / P : 0.0;
        zeta[i] = zmax * r * r;
    }
}

/* CPML profile at position x (in cells, padded coordinates) on an axis with
 * n physical cells: distance into the layer measured from the physical edge
 * nodes (index P and P+n-1). */
void or_cpml_at(const or_grid *g, int n, double x, double *a, double *b)
{
    const int P = g->npml;
    double dist = 0.0;
    if (x < P) dist = P - x;
    else if (x > P + n - 1) dist = x - (P + n - 1);
    if (P == 0 || dist <= 0.0) { *a = 0.0; *b = 1.0; return; }
    const double L = P * g->dx;
    const double d0 = 3.0 * g->pml_vmax * log(1.0 / g->pml_R) / (2.0 * L);
    double r = dist / P;
    if (r > 1.0) r = 1.0;
    const double d = d0 * r * r, al = M_PI * g->f0_pml * (1.0 - r);
    *b = exp(-(d + al) * g->dt);
    *a = d * (*b - 1.0) / (d + al);
}

int or_clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* L2 misfit of the paper's Method section: J = 1/2 sum (pred - obs)^2. */
double or_misfit(const double *pred, const double *obs, int64_t n, double *resid)
{
    double J = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = pred[i] - obs[i];
        if (resid) resid[i] = r;
        J += 0.5 * r * r;
    }
    return J;
}
