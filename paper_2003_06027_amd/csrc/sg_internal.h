// sg_internal.h -- types shared by the HIP kernels and the host runtime of
// libseisgrad (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sg {

// 2-D acoustic tile: TX columns (one wavefront) x TZ rows, 256 threads; each
// thread owns one column and RPT consecutive rows of the tile.
constexpr int TX = 64;
constexpr int TZ = 32;
constexpr int NTH = 256;
constexpr int RPT = TZ / (NTH / TX);

// Frame of every 2-D field: cell (iz, ix) of the padded grid lives at
// (iz + OZ) * SX + ix + OX; everything outside the padded grid is zero.
// OX keeps tile rows 128-byte aligned; 8 ghost cells cover the widest halo.
constexpr int OX = 32;
constexpr int OZ = 8;

// Accelerator complex dies of an MI355X (workgroups are dealt round-robin).
constexpr int NXCD = 8;

struct Grid2 {
    int NX, NZ;      // padded grid
    int P, nx, nz;   // layer width, physical extents
    int SX, SZ;      // frame extents (floats)
    long long plane; // SX * SZ
    int ntx, ntz;    // tiles
};

// Forward pass A: phi~^k = p phi~^{k-1} + q D~ u^k on the layer cells.
struct Ac2PhiArgs {
    Grid2 g;
    const float *u;                   // u^k [shot][plane]
    float *phx, *phz;                 // phi~ in place
    const float *hx, *hz;             // h = zeta dt / 2 on the padded grid
    const float *px, *pz, *ihx, *ihz; // (1-h)/(1+h) and 1/(1+h)
};

// Forward pass B over (tile, shot) pairs.
struct Ac2FwdArgs {
    Grid2 g;
    int nshots;
    const float *u;         // u^k       [shot][plane]
    float *um;              // u^{k-1} in, u^{k+1} out (same cells)
    const float *chat;      // dt^2 c^2 / dx^2  [model][plane]
    int shots_per_model;
    const float *phx, *phz; // phi~^k
    const float *hx, *hz;
    const int *src_cell;    // [shot] frame index of the source node
    const float *wav;       // [shot][nt]
    int nt, k;
    float src_scale;        // dt^2 / (dx dz)
    const int *rec_off;     // [shot][ntiles + 1] CSR over tiles
    const int *rec_ent;     // rec_pack(local cell, receiver id), sorted by cell per tile
    float *seis;            // [shot][nt][nrec] or null
    int nrec;
    float *snap;            // w~^k [shot][plane] of this step, or null
};

// Adjoint pass A: c^{k+1} = p c^{k+2} - q D~(chat s^{k+2}) on the layer cells.
struct Ac2PhiAdjArgs {
    Grid2 g;
    const float *s2;        // s^{k+2}
    const float *chat;
    int shots_per_model;
    float *cx, *cz;         // q-scaled adjoint of phi~, in place
    const float *hx, *hz, *px, *pz, *ihx, *ihz;
};

struct Ac2AdjArgs {
    Grid2 g;
    int nshots;
    const float *s2;        // s^{k+2}  (alpha-scaled adjoint), read with halo
    float *s3;              // s^{k+3} in, s^{k+1} out
    const float *chat;
    int shots_per_model;
    const float *cx, *cz;   // c^{k+1}
    const float *hx, *hz;
    const int *src_cell;
    float *gwav;            // [shot][nt] or null
    int nt, k;
    float src_scale;
    const int *rec_off;
    const int *rec_ent;
    const float *dJdd;      // [shot][nt][nrec]
    int nrec;
    const float *snap;      // w~^k [shot][plane]
    float *grad;            // dJ/dchat per shot [shot][plane], accumulated
};

void launch_ac2_phi(const Ac2PhiArgs &a, int nshots, hipStream_t s);
void launch_ac2_phi_adj(const Ac2PhiAdjArgs &a, int nshots, hipStream_t s);
void launch_ac2_fwd(const Ac2FwdArgs &a, hipStream_t s);
void launch_ac2_adj(const Ac2AdjArgs &a, hipStream_t s);
void launch_ac2_prep(const Grid2 &g, int nmodels, const float *vp, double dt, double dx,
                     float *chat, float *cpad, hipStream_t s);
void launch_ac2_finalize(const Grid2 &g, int nmodels, int shots_per_model, const float *grad,
                         float *acc, const float *cpad, double dt, double dx, float *g_vp,
                         hipStream_t s);
void launch_fill(float *p, long long n, float v, hipStream_t s);
void launch_misfit(const float *pred, const float *obs, long long n, float *resid,
                   double *partials, int nparts, double *J, hipStream_t s);
void launch_dot(const float *x, const float *y, long long n, double *out, hipStream_t s);
void launch_ricker(double f0, double t0, double dt, int nt, float *out, hipStream_t s);

// receiver entry packing: local tile cell (< 2^11) and receiver id (< 2^20)
constexpr int REC_ID_BITS = 20;
__host__ __device__ inline int rec_pack(int cell, int id) { return (cell << REC_ID_BITS) | id; }
__host__ __device__ inline int rec_cell(int e) { return e >> REC_ID_BITS; }
__host__ __device__ inline int rec_id(int e) { return e & ((1 << REC_ID_BITS) - 1); }

} // namespace sg
