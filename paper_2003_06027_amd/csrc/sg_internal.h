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

// One forward step over (tile, shot) pairs: tiles away from the layer, or
// the one-step list, whose near tiles also run pass A
// (phi~^k = p phi~^{k-1} + q D~ u^k on the layer cells of the tile + 4).
struct Ac2FwdArgs {
    Grid2 g;
    int nshots;
    const int *tiles;       // tile indices to update
    int ntl;                // number of entries in tiles
    const float *u;         // u^k       [shot][plane]
    const float *um;        // u^{k-1}
    float *un;              // u^{k+1} out (may alias um: each cell reads um before writing)
    const float *chat;      // dt^2 c^2 / dx^2  [model][plane]
    int shots_per_model;
    const float *phx0, *phz0; // phi~^{k-1} (near tiles: read on the layer cells of the tile + 4)
    float *phx, *phz;       // phi~^k out (near tiles: their own layer cells; a different buffer)
    const float *hx, *hz;   // h = zeta dt / 2 on the padded grid
    const float *px, *pz, *ihx, *ihz; // (1-h)/(1+h) and 1/(1+h)
    const long long *src_f; // [shot] frame index of the source node
    const float *wav;       // [shot][nt]
    int nt, k;
    float src_scale;        // dt^2 / (dx dz)
    const int *rec_off;     // [shot][ntiles + 1] CSR over tiles
    const int *rec_ent;     // rec_pack(local cell, receiver id), sorted by cell per tile
    float *seis;            // [shot][nt][nrec] or null
    int nrec;
    float *snap;            // w~^k [shot][plane] of this step, or null
    // several source nodes per shot (nsrc > 1; src_f is then -1): CSR over
    // tiles per shot of src_pack(local tile cell, node), wavelets [shot][nsrc][nt]
    int nsrc;
    const int *src_off;     // [shot][ntiles + 1]
    const int *src_ent;
};

// One adjoint step over (tile, shot) pairs; near tiles also run pass A
// (c^{k+1} = p c^{k+2} - q D~(chat s^{k+2}) on the layer cells of the tile + 4).
struct Ac2AdjArgs {
    Grid2 g;
    int nshots;
    const int *tiles;       // tile indices to update
    int ntl;
    const float *s2;        // s^{k+2}  (alpha-scaled adjoint), read with halo
    const float *s3;        // s^{k+3}
    float *s1;              // s^{k+1} out (may alias s3)
    const float *chat;
    int shots_per_model;
    const float *cx0, *cz0; // c^{k+2} (near tiles, q-scaled layer adjoint)
    float *cx, *cz;         // c^{k+1} out (near tiles: their own layer cells; a different buffer)
    const float *hx, *hz, *px, *pz, *ihx, *ihz;
    const long long *src_f;
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

// Two steps k, k+1 in one launch on "blocked" tiles: tiles whose cells and
// 8-cell halo are all physical (no layer terms) and which hold no receiver
// within 4 cells.  u^{k+1} is recomputed on the 4-cell halo in LDS; every
// cell gets exactly the arithmetic of two single steps.
struct Ac2Fwd2Args {
    Grid2 g;
    int nshots;
    const int *tiles;
    int ntl;
    const float *u0;        // u^k, read on the tile + 8
    const float *um;        // u^{k-1}, read on the tile + 4
    float *u1, *u2;         // u^{k+1}, u^{k+2} out (slots distinct from u0, um)
    const float *chat;
    int shots_per_model;
    const long long *src_f;
    const float *wav;
    int nt, k;
    float src_scale;
    float *snap0, *snap1;   // w~^k, w~^{k+1} [shot][plane], or null
};

// Two adjoint steps k, k-1 in one launch on blocked tiles.
struct Ac2Adj2Args {
    Grid2 g;
    int nshots;
    const int *tiles;
    int ntl;
    const float *s2;        // s^{k+2}, read on the tile + 8
    const float *s3;        // s^{k+3}, read on the tile + 4
    float *o1, *o0;         // s^{k+1}, s^k out (slots distinct from s2, s3)
    const float *chat;
    int shots_per_model;
    const long long *src_f;
    float *gwav;
    int nt, k;
    float src_scale;
    const float *snap1, *snap0;  // w~^k, w~^{k-1}
    float *grad;
};

// Halo of a blocked tile: its cells within BLK_HALO of the tile must be physical.
constexpr int BLK_HALO = 8;

// Adjoint of several source nodes: gw[shot][j][k] = scale * s^{k+1}[node j].
void launch_ac2_src_gather(int nshots, int nsrc, long long plane, const long long *node_f, const float *s1,
                           float *gw, int nt, int k, float scale, hipStream_t s);
void launch_ac2_fwd2(const Ac2Fwd2Args &a, hipStream_t s);
void launch_ac2_adj2(const Ac2Adj2Args &a, hipStream_t s);
// near: the one-step list (pass A folded into its near tiles); else tiles away from the layer
void launch_ac2_fwd(const Ac2FwdArgs &a, bool near, hipStream_t s);
// the near tiles' step k (a) and the blocked tiles' steps k, k+1 (b) in one launch
void launch_ac2_fwd_pair(const Ac2FwdArgs &a, const Ac2Fwd2Args &b, hipStream_t s);
void launch_ac2_adj(const Ac2AdjArgs &a, bool near, hipStream_t s);
void launch_ac2_prep(const Grid2 &g, int nmodels, const float *vp, double dt, double dx,
                     float *chat, float *cpad, hipStream_t s);
void launch_ac2_finalize(const Grid2 &g, int nmodels, int shots_per_model, const float *grad,
                         float *acc, const float *cpad, double dt, double dx, float *g_vp,
                         hipStream_t s);
void launch_fill(float *p, long long n, float v, hipStream_t s);
// Partial sums of the misfit reduction (a model's workspace slot, or the
// static array of the allocation-free entry point).
constexpr int NOALLOC_PARTS = 4096;
// The device address of this device's static partial-sum array (taken once
// per device); 0 on success, -1 if the runtime cannot give it.
int noalloc_scratch(double **out);
// flag (nullable): set to 1 when J comes out non-finite, left alone otherwise.
void launch_misfit(const float *pred, const float *obs, long long n, float *resid,
                   double *partials, int nparts, double *J, int *flag, hipStream_t s);
void launch_dot(const float *x, const float *y, long long n, double *out, hipStream_t s);
void launch_ricker(double f0, double t0, double dt, int nt, float *out, hipStream_t s);

// receiver entry packing: local tile cell (< 2^11) and receiver id (< 2^20)
constexpr int REC_ID_BITS = 20;
__host__ __device__ inline int rec_pack(int cell, int id) { return (cell << REC_ID_BITS) | id; }
__host__ __device__ inline int rec_cell(int e) { return e >> REC_ID_BITS; }
__host__ __device__ inline int rec_id(int e) { return e & ((1 << REC_ID_BITS) - 1); }

// source-node entry packing: local tile cell (< 2^11) and node index (< 2^12)
constexpr int SRC_NODE_BITS = 12;
__host__ __device__ inline int src_pack(int cell, int node) { return (cell << SRC_NODE_BITS) | node; }
__host__ __device__ inline int src_cell(int e) { return e >> SRC_NODE_BITS; }
__host__ __device__ inline int src_node(int e) { return e & ((1 << SRC_NODE_BITS) - 1); }

} // namespace sg
