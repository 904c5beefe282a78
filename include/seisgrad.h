/* seisgrad.h -- C ABI of the MI355X (gfx950) finite-difference wave-propagation
 * and adjoint-gradient library (libseisgrad.so).
 *
 * What the library computes (Zhu, Xu, Darve & Beroza, "A General Approach to
 * Seismic Inversion with Automatic Differentiation"):
 *   - the explicit recursion U_k = A(theta) U_{k-1} + F_{k-1}
 *     (Method, "Relationship to the Adjoint Method", Eq. (1)) for the
 *     acoustic wave equation (Implementation, Eq. (12), constant-density form
 *     u_tt = c^2 lap(u) + f, 2nd order in time, 8th order in space) with an
 *     auxiliary-field absorbing layer (PML) padded outside the model; and the
 *     same equation in the divergence form printed in Eq. (12),
 *     u_tt = div(c^2 grad u) + f (physics SG_ACOUSTIC_DIV, 2-D): the
 *     staggered grid with a convolutional PML of the Implementation section,
 *     4th order in space, flux coefficients c^2 averaged onto the half nodes
 *     ((c_i^2 + c_{i+1}^2)/2), a CPML memory variable on both the inner and
 *     the outer derivative of each axis;
 *   - point-source injection of a wavelet and receiver gathering (the F_k
 *     and the observation operator of the misfit);
 *   - the L2 misfit J = 1/2 sum ||d - d_obs||^2 (display after Eq. (1)) on
 *     the receiver samples, accumulated in FP64;
 *   - the gradient dJ/dtheta = sum_k lambda_k^T (dA/dtheta) U_{k-1}
 *     (Eq. (5)) with lambda_k from the adjoint recursion (Eq. (4)), which the
 *     paper's Theorem shows equal to reverse-mode AD (Eqs. (8)-(9)).
 *
 * Conventions
 *   - Physical model arrays: FP32, row-major [model][iz][ix] (2-D) or
 *     [model][iz][iy][ix] (3-D), x fastest, z down, 0-based.  The absorbing layer of npml cells is padded
 *     OUTSIDE the physical grid on every side, the model being continued by
 *     edge replication; cells beyond the padded grid are zero (rigid).
 *   - Time: u^0 = u^{-1} = 0; step k (0..nt-1) injects wavelet sample k;
 *     seismogram sample k holds u^{k+1} at the receivers.
 *   - Source: a point source at a grid node, f = r(t_k) / (dx*dz) in 2-D,
 *     r(t_k) / dx^3 in 3-D.
 *   - 3-D absorbing layer: the auxiliary-field form of complex coordinate
 *     stretching with psi = time integral of u (phi_x, phi_y, phi_z, psi).
 *   - Seismograms: FP32 [nshots][ncomp][nt][nrec] (ncomp = 1 acoustic).
 *   - Shots are ordered model-major: with nmodels models, shot s uses model
 *     s / (nshots / nmodels); nshots must be a multiple of nmodels.
 *   - The damping profile zeta(d) = zeta_max (d/npml)^2 with
 *     zeta_max = 3 pml_vmax ln(1/pml_R) / (2 npml dx) is fixed by pml_vmax and
 *     does not depend on the model (so the gradient has no profile term).
 *
 * Ownership and memory
 *   - Every array argument marked DEVICE is a caller-owned, contiguous device
 *     pointer on the current HIP device; HOST arrays are read during the call
 *     only.  The library never allocates device memory: all its state
 *     (coefficients, wavefields, checkpoints, snapshots, per-shot gradients,
 *     reduction partials) is carved from the caller's workspace, whose size is
 *     given by workspace_bytes().  The workspace must outlive the model.
 *   - sg_model is an opaque host object owned by the library until
 *     free_model().  One model per stream; calls on one model are not
 *     thread-safe.
 *   - Every call enqueues its GPU work on `stream` (0 = null stream) and
 *     returns after host-side validation; results are valid once the stream
 *     has reached that point.  Outputs are overwritten, never accumulated.
 *
 * Errors: every int-returning entry point returns SG_OK (0) or a negative
 * code; last_error() gives a thread-local message for the last failure.  No
 * C++ exception crosses the ABI.
 */
#ifndef SEISGRAD_H
#define SEISGRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SG_API __attribute__((visibility("default")))
#else
#define SG_API
#endif

typedef struct ihipStream_t *sg_stream_t; /* hipStream_t */

enum {
    SG_OK = 0,
    SG_EINVAL = -1,      /* bad shape, NULL pointer, out-of-grid source/receiver */
    SG_EUNSTABLE = -2,   /* CFL number above 0.95 x the scheme's limit, or zeta_max*dt > 0.3 */
    SG_ENOMEM = -3,      /* workspace smaller than workspace_bytes() */
    SG_ESTATE = -4,      /* adjoint without a matching checkpointed forward */
    SG_EDEVICE = -5,     /* a HIP runtime call failed */
    SG_EUNSUPPORTED = -6,/* a physics / dimension combination this build does not provide */
    SG_ENUMERIC = -7     /* a misfit on this model came out non-finite (NaN or Inf in the
                            seismograms); reported by numeric_status(), the next call that
                            synchronises with the stream */
};

/* SG_ACOUSTIC: u_tt = c^2 lap(u) + f (2-D, 3-D); SG_ELASTIC: velocity-stress
 * equations (2-D); SG_ACOUSTIC_DIV: u_tt = div(c^2 grad u) + f (2-D). */
enum { SG_ACOUSTIC = 0, SG_ELASTIC = 1, SG_ACOUSTIC_DIV = 2 };

/* Grid, time stepping and absorbing layer. */
typedef struct sg_desc {
    int32_t ndim;       /* 2 or 3 */
    int32_t physics;    /* SG_ACOUSTIC, SG_ELASTIC or SG_ACOUSTIC_DIV */
    int32_t nx, ny, nz; /* physical cells; ny = 1 in 2-D */
    int32_t npml;       /* absorbing-layer width in cells (>= 0) */
    int32_t nt;         /* time steps (>= 1) */
    int32_t nmodels;    /* models batched in one launch (>= 1) */
    double dx;          /* grid spacing, all axes (m) */
    double dt;          /* time step (s) */
    double pml_R;       /* target reflection coefficient, e.g. 1e-3 */
    double pml_vmax;    /* reference velocity of the damping profile (m/s) */
    double f0_pml;      /* CPML frequency of the staggered-grid forms (alpha = pi f0_pml (1 - x/L));
                           unused by SG_ACOUSTIC */
} sg_desc;

/* One batch of shots. */
#define SG_MAX_SRC 4096  /* source nodes per shot */

typedef struct sg_shots {
    int32_t nshots;          /* >= 1, multiple of nmodels, <= max_shots of the model */
    int32_t nrec;            /* receivers per shot (>= 0) */
    const int32_t *src;      /* HOST [nshots][nsrc][ndim]: (ix, iz) or (ix, iy, iz) source nodes */
    const int32_t *rec;      /* HOST [nshots][nrec][ndim]: receiver nodes, same order */
    const float *wavelet;    /* DEVICE [nshots][nsrc][nt]: source time function r_j(t_k) of
                                each source node (value r at a node: density r/(dx dz)) */
    const float *mt;         /* HOST [nshots][3]: moment tensor (Mxx, Mzz, Mxz) of elastic
                                sources (stress-rate injection dt M r(t_n)/(dx dz)); NULL for
                                acoustic shots */
    int32_t nsrc;            /* source nodes per shot: 0 or 1 = one point source; up to
                                SG_MAX_SRC nodes, each with its own wavelet, for the 2-D
                                acoustic equations only (the Gaussian-footprint location
                                source and the multi-point rupture of the paper's source
                                applications, a row of delayed wavelets for the
                                bottom-incident plane waves of its layered-model
                                inversion); other physics return SG_EUNSUPPORTED */
} sg_shots;

typedef struct sg_model sg_model;

/* Bytes of device workspace needed for up to max_shots shots of up to
 * max_rec receivers each, with wavefield checkpoints every ckpt_every steps
 * (0 -> ceil(sqrt(nt))).  Returns 0 (reason in last_error()) on an invalid
 * descriptor or a size beyond the build's limits: 2^20 - 1 receivers per
 * shot; 3-D grids below 4096 padded planes in z, and 76 padded planes of
 * the xy frame below 4 GiB; elastic runs of at most 65535 shots, with
 * ceil(NX / 32) * ceil(NZ / 8) * max_shots below 2^31 (NX, NZ: padded). */
SG_API size_t workspace_bytes(const sg_desc *d, int32_t max_shots, int32_t max_rec, int32_t ckpt_every);

/* Bytes that one stored checkpoint segment of adjoint snapshots takes in the
 * workspace beyond workspace_bytes() (see init_model's ws).  0 on an invalid
 * descriptor. */
SG_API size_t snapshot_segment_bytes(const sg_desc *d, int32_t max_shots, int32_t ckpt_every);

/* Prepare a model (paper: the parameter theta of A(theta), Eq. (1); here the
 * velocity c of Eq. (12)): validate the descriptor, check stability
 * (8th-order leapfrog limit c dt/dx <= 2/sqrt(6.5016 ndim); staggered 4th
 * order, elastic and SG_ACOUSTIC_DIV: c dt/dx <= 1/(sqrt(ndim) (9/8 + 1/24));
 * rejected above 0.95 of the limit), pad the velocity by edge replication,
 * form C = dt^2 c^2 on the padded grid and the damping tables.
 *   vp:  DEVICE FP32 [nmodels][nz]([ny])[nx] velocity (m/s), > 0;
 *   vs, rho: elastic only, DEVICE FP32 like vp (0 < vs < vp, rho > 0);
 *        NULL for acoustic models;
 *   ws:  DEVICE workspace, 256-byte aligned, of
 *        ws_bytes >= workspace_bytes(d, max_shots, max_rec, ckpt_every).
 *        Bytes beyond that minimum hold the adjoint's snapshots of as many
 *        of the LAST checkpoint segments as fit: a checkpointed forward
 *        writes them directly, and adjoint_gradient then skips the restore
 *        and recomputation of those segments (same results, bit for bit;
 *        fewer recomputed steps).  Each stored segment takes
 *        ckpt_every x (snapshot fields) x max_shots planes of FP32;
 *   out: receives the model handle.
 * The call synchronises `stream` once (it reads the velocity range back for
 * the stability check).  The velocity is copied into the workspace; vp may be
 * freed afterwards. */
SG_API int init_model(const sg_desc *d, const float *vp, const float *vs, const float *rho,
               int32_t max_shots, int32_t max_rec, int32_t ckpt_every, void *ws,
               size_t ws_bytes, sg_stream_t stream, sg_model **out);

/* New parameters for a prepared model (paper: a new theta in A(theta),
 * Eq. (1), as each iteration of an inversion makes it): the same checks and
 * preparation as init_model, on the model's grid, shots and workspace; the
 * geometry, work lists, tables and captured segment graphs are kept.
 *   vp, vs, rho: DEVICE FP32 as in init_model (vs, rho NULL for acoustic
 *                models); copied, may be freed afterwards.
 * Synchronises `stream` once (the stability check).  The checkpoints and
 * stored snapshots of an earlier forward belong to the old parameters:
 * adjoint_gradient returns SG_ESTATE until a checkpointed forward runs.
 * Errors: SG_EINVAL (NULL model or vp, vs/rho given for acoustic or missing
 * for elastic models, non-positive or non-finite values), SG_EUNSTABLE; the
 * model keeps its old parameters on an error before preparation. */
SG_API int update_model(sg_model *m, const float *vp, const float *vs, const float *rho, sg_stream_t stream);

/* Forward modelling of a batch of shots (Eq. (1) with the source term F_k):
 * runs all nt steps and writes the seismograms.
 *   seis: DEVICE FP32 [nshots][1][nt][nrec], overwritten;
 *   save_ckpt: nonzero stores a wavefield checkpoint every ckpt_every steps
 *   (required before adjoint_gradient).
 * Errors: SG_EINVAL on out-of-grid sources/receivers or nshots too large. */
SG_API int forward_shots(sg_model *m, const sg_shots *sh, float *seis, int32_t save_ckpt,
                  sg_stream_t stream);

/* L2 misfit (display after Eq. (1)): resid = pred - obs (FP32) and
 * J = 1/2 sum resid^2 accumulated in FP64 in a fixed order (bitwise
 * reproducible).
 *   pred, obs: DEVICE FP32 [n] (may be NULL when n == 0, which gives J = 0);
 *   J_dev: DEVICE double[1]; resid: DEVICE FP32 [n] or NULL (may alias
 *   pred).  Errors: SG_EINVAL for n < 0, J_dev NULL, or pred/obs NULL with
 *   n > 0.  With a model the reduction runs over many
 *   workgroups and keeps its partial sums in the model's workspace; with
 *   m == NULL it runs in one workgroup (slower, no workspace).
 * Non-finite inputs give a non-finite J; the call itself does not sync.  With
 * a model, a non-finite J also sets the model's numeric flag, which
 * numeric_status() reports as SG_ENUMERIC. */
SG_API int misfit(sg_model *m, const float *pred, const float *obs, int64_t n,
           double *J_dev, float *resid, sg_stream_t stream);

/* Gradient of J with respect to the velocity by the adjoint sweep
 * (Eqs. (4)-(5)), for ANY seismogram-space adjoint dJ_dd (for the L2 misfit,
 * the resid of misfit()).  Needs the checkpointed forward of the same shots
 * (same geometry) on this model; recomputes each segment of ckpt_every steps
 * from its checkpoint and runs the exact transpose of the forward step
 * backwards in time.
 *   dJ_dd: DEVICE FP32 [nshots][1][nt][nrec];
 *   g_vp:  DEVICE FP32 [nmodels][nz]([ny])[nx], sum over the model's shots in shot
 *          order, absorbing-layer cells folded onto the edge cells they
 *          replicate;
 *   g_vs, g_rho: reserved, NULL;
 *   g_wavelet: DEVICE FP32 [nshots][nsrc][nt] or NULL: dJ/dr_j(t_k) per shot and
 *            source node.
 * Errors: SG_ESTATE when no matching checkpointed forward precedes it. */
SG_API int adjoint_gradient(sg_model *m, const sg_shots *sh, const float *dJ_dd,
                     float *g_vp, float *g_vs, float *g_rho, float *g_wavelet,
                     sg_stream_t stream);

/* misfit() for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the reduction a model's misfit runs -- 4096 workgroup partial sums in
 * FP64, added in a fixed order -- with the partial sums in a static device
 * array of the library instead of a model's workspace, so J_dev and resid
 * are bitwise those of misfit(m, ...).  The array holds 4096 doubles
 * (32 KiB) per device and stays allocated until the process ends; its
 * address is taken once per device on the first call there.  The call
 * allocates nothing and does not synchronise.  Every call on one device
 * shares that device's array: calls that overlap on one device (streams not
 * ordered with each other) race on it and must be serialised by the caller.
 * No model is involved, so no numeric flag is set: a non-finite J is visible
 * in J_dev itself.
 *   pred, obs: DEVICE FP32 [n] (may be NULL when n == 0, which gives J = 0);
 *   J_dev: DEVICE double[1]; resid: DEVICE FP32 [n] or NULL (may alias pred).
 * Errors: SG_EINVAL for n < 0, n above 2^40, J_dev NULL, or pred/obs NULL with
 * n > 0; SG_EDEVICE if the runtime gives no address for the array. */
SG_API int misfit_noalloc(const float *pred, const float *obs, int64_t n, double *J_dev, float *resid,
                          sg_stream_t stream);

/* Numeric state of the model's misfits: waits for `stream`, then returns
 * SG_ENUMERIC if any misfit() on this model since the previous
 * numeric_status() (or since init_model) produced a non-finite J -- a NaN or
 * Inf in the predicted or observed seismograms, or an overflow of the sum --
 * and SG_OK otherwise.  Reading the flag clears it.  The flag is one int in
 * the model's workspace, set by the misfit's final reduction on the device,
 * so a failing misfit itself returns SG_OK (it does not synchronise) and the
 * failure surfaces here.  Not for use inside a captured graph (it
 * synchronises).  Errors: SG_EINVAL for a NULL model, SG_EDEVICE. */
SG_API int numeric_status(sg_model *m, sg_stream_t stream);

/* Optional device timing of the step loops.  With profiling on, the
 * library records one pair of HIP events on the call's stream around every
 * checkpoint segment of the forward sweep (phase 0), of the recompute
 * (phase 1) and of the adjoint steps (phase 2); phase_times() waits for them
 * and returns, per phase, the summed milliseconds and the number of steps
 * they cover, then forgets them.  ms and steps: HOST arrays of 3. */
SG_API int set_profiling(sg_model *m, int32_t enable);
SG_API int phase_times(sg_model *m, double *ms, int64_t *steps);

/* Time blocking of the 2-D acoustic sweeps (the recursion of Eq. (1), run
 * unchanged): with steps = 2 (the default) tiles whose cells and 8-cell halo
 * are all physical and hold no receiver within 4 cells advance two time steps
 * per launch, the other tiles one; steps = 1 advances every tile one step
 * per launch.  Every value is computed with the same operations either way,
 * so seismograms and gradients are bitwise identical; only the memory
 * traffic and the launch count change.  Other physics ignore the setting.
 * Returns SG_EINVAL unless steps is 1 or 2. */
SG_API int set_time_blocking(sg_model *m, int32_t steps);

/* Launch settings of a model, for the autotuner (none changes what is
 * computed): keys and values
 *   SG_TUNE_TIME_BLOCKING  1 or 2: as set_time_blocking();
 *   SG_TUNE_CHUNK_FWD3     planes per z chunk of the 3-D forward tile passes;
 *   SG_TUNE_CHUNK_ADJ3     planes per z chunk of the 3-D adjoint tile passes;
 *   SG_TUNE_CHUNK_LAYER3   planes per work item of the 3-D layer passes
 *                          (3-D chunks: 16 to 64, multiples of 8; defaults
 *                          32, 64, 32);
 *   SG_TUNE_PAIR           2-D acoustic with time blocking: 1 (the default)
 *                          launches the step of the tiles by the layer with
 *                          the two-step launch of the blocked tiles as one
 *                          grid in sweeps that record no seismograms (the
 *                          recompute), 0 apart;
 *   SG_TUNE_SHOT_GROUP     elastic: shots of one model per thread, 1, 2 or 4
 *                          (0: 4 if the shots per model divide by 4, else 2
 *                          if even, else 1; a value that does not divide the
 *                          shots per model falls back to that rule);
 *   SG_TUNE_BLOCK_X        elastic: cell blocks of 32 x 8 (32, the default)
 *                          or 64 x 4 (64) cells;
 *   SG_TUNE_GRAPHS         every physics: 1 runs each checkpoint segment of
 *                          forward_shots (the checkpoint copies and K steps)
 *                          and of adjoint_gradient (restore, recompute, K
 *                          adjoint steps) as one HIP graph, captured on a
 *                          stream of the model at the first call and
 *                          replayed on `stream` by later calls with the same
 *                          arguments (seismogram, wavelet, residual and
 *                          wavelet-gradient pointers, shot counts, settings,
 *                          geometry); other arguments re-capture the
 *                          segments.  0 (the default): launches per step.
 *                          Per-phase timing (set_profiling) is not recorded
 *                          in graph mode.
 * Chunks, block widths and graphs compute every value with the same
 * operations, so results do not change; the shot
 * group changes the order in which the elastic gradient sums over shots
 * (fixed for a given setting, so results stay reproducible).  Changing the
 * layer chunk rebuilds and uploads the work list: the call waits for
 * `stream` (which must be the stream of the model's launches) before and
 * after the upload.  Call between sweeps.  Errors: SG_EINVAL for an unknown
 * key, a value out of range, or a key that does not apply to the model. */
enum { SG_TUNE_TIME_BLOCKING = 0, SG_TUNE_CHUNK_FWD3 = 1, SG_TUNE_CHUNK_ADJ3 = 2, SG_TUNE_CHUNK_LAYER3 = 3,
       SG_TUNE_SHOT_GROUP = 4, SG_TUNE_BLOCK_X = 5, SG_TUNE_GRAPHS = 6, SG_TUNE_PAIR = 7 };
SG_API int set_tuning(sg_model *m, int32_t key, int32_t value, sg_stream_t stream);

/* Limited-memory BFGS helpers of the outer inversion loop (the paper's
 * optimizer is L-BFGS-B, Applications, FWI; bounds are kept by clipping the
 * model after each step).  Models of a batch keep separate histories in ring
 * buffers S, Y: DEVICE FP32 [mem][nmodels][n]; ysyy: DEVICE FP64
 * [mem][nmodels][2] holding (y.s, y.y) of each stored pair; 1 <= mem <= 64.
 *
 * lbfgs_push: for each model b with 0 <= slot[b] < mem, writes
 *   s = m_new - m_old and y = g_new - g_old (all DEVICE FP32 [nmodels][n])
 *   into ring slot slot[b] and their (y.s, y.y) in FP64 (fixed order); a
 *   model with slot[b] outside [0, mem) is left unchanged.  slot: DEVICE
 *   int32 [nmodels].  The caller keeps a pair only if y.s > 0.
 * lbfgs_direction: p = -H g per model by the two-loop recursion (Nocedal &
 *   Wright, Algorithm 7.4) over hist[2b] pairs ending at ring slot
 *   hist[2b+1] (newest), with H0 = (y.s / y.y of the newest pair) I; no
 *   pairs (or hist[2b+1] outside [0, mem)) gives p = -g.  hist: DEVICE int32
 *   [nmodels][2]; g, p: DEVICE FP32 [nmodels][n], p must not alias g.
 *   Inner products in FP64, fixed order: bitwise reproducible. */
SG_API int lbfgs_push(int32_t nmodels, int64_t n, int32_t mem, const int32_t *slot, const float *m_new,
                      const float *m_old, const float *g_new, const float *g_old, float *S, float *Y,
                      double *ysyy, sg_stream_t stream);
SG_API int lbfgs_direction(int32_t nmodels, int64_t n, int32_t mem, const int32_t *hist, const float *S,
                           const float *Y, const double *ysyy, const float *g, float *p, sg_stream_t stream);

/* Source parameterisations of the paper's source applications (2-D; nodes
 * are physical (ix, iz) indices, node (ix, iz) sits at (ix dx, iz dx)).
 *
 * Earthquake location (Applications, "Earthquake Location and Source Time
 * Function Retrieval"): f(x, t) = g(t) exp(-|x - x0|^2/(2 sigma^2))/(2 pi
 * sigma^2) sampled at nsrc footprint nodes (the caller picks the nodes, e.g.
 * the 7 x 7 around the node nearest x0 for sigma = dx/2):
 *   source_gaussian: wav[j][k] = g(t_k) w_j, w_j = dx^2 exp(-r_j^2/(2
 *     sigma^2))/(2 pi sigma^2) -- the wavelets of one shot's nodes;
 *   source_gaussian_grad: from gw = dJ/dwav [nsrc][nt] (adjoint_gradient's
 *     g_wavelet), dg[k] = dJ/dg(t_k) and dxz = (dJ/dx0, dJ/dz0).
 * Rupture (Applications, "Earthquake Rupture Imaging"): points j with
 * f_j(t) = A0_j exp(-(t - t0_j)^2/(2 sigma_t^2)):
 *   source_rupture: wav[j][k] = f_j(k dt);
 *   source_rupture_grad: dA0[j] = dJ/dA0_j and dt0[j] = dJ/dt0_j from gw.
 * cells: DEVICE int32 [nsrc][2]; g, A0, t0, wav, gw, dg: DEVICE FP32; dxz
 * (2), dA0, dt0 (npt): DEVICE FP64.  Sums over steps and nodes in FP64, in a
 * fixed order. */
SG_API int source_gaussian(int32_t nsrc, int32_t nt, const int32_t *cells, double x0, double z0, double sigma,
                           double dx, const float *g, float *wav, sg_stream_t stream);
SG_API int source_gaussian_grad(int32_t nsrc, int32_t nt, const int32_t *cells, double x0, double z0,
                                double sigma, double dx, const float *g, const float *gw, float *dg, double *dxz,
                                sg_stream_t stream);
SG_API int source_rupture(int32_t npt, int32_t nt, const float *A0, const float *t0, double sigma_t, double dt,
                          float *wav, sg_stream_t stream);
SG_API int source_rupture_grad(int32_t npt, int32_t nt, const float *A0, const float *t0, double sigma_t, double dt,
                               const float *gw, double *dA0, double *dt0, sg_stream_t stream);

/* Bottom-incident plane wave (Applications, FWI: the layered model is probed
 * by plane waves arriving from below at -30, -10, 10 and 30 degrees, with a
 * Ricker source time function): a row of n source nodes at
 * x_j = x_first + j spacing (metres) firing the Ricker wavelet
 * r(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0 - tau_j))^2, with delays
 * tau_j = (x_j - x_ref) sin(theta)/c, x_ref the first node to fire, so that
 * the row emits a front travelling at theta from the vertical through a
 * medium of velocity c (positive theta: towards +x).
 *   wav: DEVICE FP32 [n][nt] (a shot's wavelets for its n row nodes),
 *   computed in FP64.  Errors: SG_EINVAL unless n, nt >= 1, c, f0, dt > 0
 *   and |theta_deg| < 90. */
SG_API int source_plane_wave(int32_t n, int32_t nt, double x_first, double spacing, double theta_deg, double c,
                             double f0, double t0, double dt, float *wav, sg_stream_t stream);

/* Release the host object (the workspace stays the caller's). */
SG_API int free_model(sg_model *m);

/* Message of the last failed call on this thread ("" if none). */
SG_API const char *last_error(void);

/* Ricker wavelet r(t_k) = (1 - 2 pi^2 f0^2 (t_k - t0)^2) exp(-pi^2 f0^2 (t_k - t0)^2),
 * t_k = k dt, the source time function of the paper's FWI tests
 * (Applications, "Full-waveform Inversion"); evaluated in FP64, stored FP32.
 *   out: DEVICE FP32 [nt]. */
SG_API int ricker(double f0, double t0, double dt, int32_t nt, float *out, sg_stream_t stream);

/* FP64 inner product sum x[i]*y[i] of two FP32 device vectors in a fixed
 * reduction order, one workgroup (dot-product tests, gradient norms).
 *   x, y: DEVICE FP32 [n]; out: DEVICE double[1]. */
SG_API int dot_f64(const float *x, const float *y, int64_t n, double *out, sg_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif
