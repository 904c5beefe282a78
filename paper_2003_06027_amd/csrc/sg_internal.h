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
    const int *tiles;       // tile indices to update, or null for all tiles
    int ntl;                // number of entries in tiles
    const float *u;         // u^k       [shot][plane]
    const float *um;        // u^{k-1}
    float *un;              // u^{k+1} out (may alias um: each cell reads um before writing)
    const float *chat;      // dt^2 c^2 / dx^2  [model][plane]
    int shots_per_model;
    const float *phx, *phz; // phi~^k
    const float *hx, *hz;
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

// Adjoint pass A: c^{k+1} = p c^{k+2} - q D~(chat s^{k+2}) on the layer cells.
struct Ac2PhiAdjArgs {
    Grid2 g;
    const int *tiles;       // tiles holding layer cells
    int ntl;
    const float *s2;        // s^{k+2}
    const float *chat;
    int shots_per_model;
    float *cx, *cz;         // q-scaled adjoint of phi~, in place
    const float *hx, *hz, *px, *pz, *ihx, *ihz;
};

struct Ac2AdjArgs {
    Grid2 g;
    int nshots;
    const int *tiles;       // tile indices to update, or null for all tiles
    int ntl;
    const float *s2;        // s^{k+2}  (alpha-scaled adjoint), read with halo
    const float *s3;        // s^{k+3}
    float *s1;              // s^{k+1} out (may alias s3)
    const float *chat;
    int shots_per_model;
    const float *cx, *cz;   // c^{k+1}
    const float *hx, *hz;
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
void launch_ac2_phi(const Ac2PhiArgs &a, int nshots, hipStream_t s);
void launch_ac2_fwd2(const Ac2Fwd2Args &a, hipStream_t s);
void launch_ac2_adj2(const Ac2Adj2Args &a, hipStream_t s);
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

// source-node entry packing: local tile cell (< 2^11) and node index (< 2^12)
constexpr int SRC_NODE_BITS = 12;
__host__ __device__ inline int src_pack(int cell, int node) { return (cell << SRC_NODE_BITS) | node; }
__host__ __device__ inline int src_cell(int e) { return e >> SRC_NODE_BITS; }
__host__ __device__ inline int src_node(int e) { return e & ((1 << SRC_NODE_BITS) - 1); }


// ---------------------------------------------------------------- 3-D
// Tile of the 3-D kernels: TX3 x TY3 columns (one thread each), marching in
// z over chunks of TZC planes with a register window of 9 planes.
constexpr int TX3 = 32;
constexpr int TY3 = 16;
constexpr int NTH3 = TX3 * TY3;
constexpr int TZC = 64;
constexpr int OX3 = 32;  // x offset (128-byte aligned rows)
constexpr int OY3 = 4;
constexpr int OZ3 = 4;
constexpr int CELL3_BITS = 9;   // local cell of a TX3 x TY3 plane tile

struct Grid3 {
    int NX, NY, NZ;
    int P, nx, ny, nz;
    int SX, SY, SZ;
    long long sy, sz, plane;   // strides: sy = SX, sz = SX*SY, plane = sz*SZ
    int ntx, nty, nzc;         // tiles in x, y; z chunks
};

struct Ac3Tabs {               // per-axis damping tables, h = zeta dt / 2
    const float *h[3], *p[3], *ih[3];  // x, y, z: h, (1-h)/(1+h), 1/(1+h)
};

struct Ac3FwdArgs {
    Grid3 g;
    int nshots;
    const float *u;            // u^k
    float *um;                 // u^{k-1} in, u^{k+1} out
    const float *chat;
    int shots_per_model;
    const float *ph[3];        // phi~_j^k
    float *psi;                // psi^k in, psi^{k+1} out (layer cells)
    Ac3Tabs t;
    float dt, inv_dt;
    const long long *src_f;    // [shot] frame index of the source node
    const float *wav;
    int nt, k;
    float src_scale;           // dt^2 / dx^3
    const int *rec_off;        // [shot][ntx*nty + 1]
    const int2 *rec_ent;       // x: (iz << CELL3_BITS) | cell, y: receiver id
    float *seis;
    int nrec;
    float *snap;
    const int *tiles;          // xy tiles, the nnear within 4 cells of the layer in x or y first
    int nnear;
    int t0, ntl;               // this launch's slice of tiles (set by the launcher)
};

struct Ac3PhiArgs {
    Grid3 g;
    const int4 *items;         // (xy tile, first plane, end plane) of the layer work
    int nitems;
    const float *u, *psi;      // u^k, psi^k
    float *ph[3];              // in place
    Ac3Tabs t;
    float inv_dt;
};

struct Ac3PhiAdjArgs {
    Grid3 g;
    const int4 *items;         // as in Ac3PhiArgs
    int nitems;
    const float *s2;
    const float *chat;
    int shots_per_model;
    float *b[3];               // adjoint of phi~_j, in place
    Ac3Tabs t;
};

struct Ac3AdjArgs {
    Grid3 g;
    int nshots;
    const float *s2;
    float *s3;
    const float *chat;
    int shots_per_model;
    const float *b[3];
    float *e;                  // adjoint of psi, in place (layer cells)
    Ac3Tabs t;
    float dt, inv_dt;
    const long long *src_f;
    float *gwav;
    int nt, k;
    float src_scale;
    const int *rec_off;
    const int2 *rec_ent;
    const float *dJdd;
    int nrec;
    const float *snap;
    float *grad;
    const int *tiles;          // as in Ac3FwdArgs
    int nnear;
    int t0, ntl;
};

void launch_ac3_phi(const Ac3PhiArgs &a, int nshots, hipStream_t s);
void launch_ac3_fwd(const Ac3FwdArgs &a, hipStream_t s);
void launch_ac3_phi_adj(const Ac3PhiAdjArgs &a, int nshots, hipStream_t s);
void launch_ac3_adj(const Ac3AdjArgs &a, hipStream_t s);
void launch_ac3_prep(const Grid3 &g, int nmodels, const float *vp, double dt, double dx,
                     float *chat, float *cpad, hipStream_t s);
void launch_ac3_finalize(const Grid3 &g, int nmodels, int spm, const float *grad, float *acc,
                         const float *cpad, double dt, double dx, float *g_vp, hipStream_t s);

// ---------------------------------------------------------------- elastic 2-D
// Staggered velocity-stress fields on a 2-D frame (same frame as the 2-D
// acoustic fields); one thread per cell, 64 x 4 cell blocks.
constexpr int EL_NS = 13;      // vx vz sxx szz sxz + 8 CPML memory variables
enum { E_VX, E_VZ, E_SXX, E_SZZ, E_SXZ, E_MVXX, E_MVXZ, E_MVZX, E_MVZZ,
       E_MSXXX, E_MSXZZ, E_MSXZX, E_MSZZZ };
enum { M_LAM, M_MU, M_MUXZ, M_BX, M_BZ };

struct El2Tabs {               // CPML a, b at integer (0) and half (1) positions
    const float *ax[2], *bx[2], *az[2], *bz[2];
};

struct El2Args {
    Grid2 g;                   // NX, NZ, P, nx, nz, SX, SZ, plane (tiles unused)
    int nshots, shots_per_model;
    float *f[EL_NS];           // state fields [shot][plane]
    const float *m[5];         // model fields [model][plane]
    El2Tabs t;
    float kap;                 // dt / dx
    float *snap;               // 5 fields [5][shot][plane] or null
    long long snap_stride;     // floats between snapshot fields
    // source (stress step)
    const long long *src_f;
    const float *mt;           // [shot][3]
    const float *wav;
    int nt, k;
    float src_scale;           // dt / (dx dz)
};

struct El2AdjArgs {
    Grid2 g;
    int nshots, shots_per_model;
    float *a[EL_NS];           // adjoint state
    float *tmp[8];             // e1..e4 then d1..d4
    const float *m[5];
    El2Tabs t;
    float kap;
    const float *snap;
    long long snap_stride;
    float *grad;               // 5 accumulators [5][shot][plane]
    long long grad_stride;
    const long long *src_f;
    const float *mt;
    float *gwav;
    int nt, k;
    float src_scale;
};

struct El2RecArgs {
    int nshots, nrec, nt, k;
    const long long *rec_f;    // [shot][nrec] frame index
    long long plane;
    const float *vx, *vz;
    float *seis;               // [shot][2][nt][nrec]
    // adjoint injection: unique cells per shot
    const int *uoff;           // [shot][nuniq_max + 1] offsets into uid
    const int *uid;            // receiver ids grouped by cell
    int nuniq_max;
    const float *dJdd;
    float *ax, *az;
};

void launch_el2_vel(const El2Args &a, hipStream_t s);
void launch_el2_str(const El2Args &a, hipStream_t s);
void launch_el2_record(const El2RecArgs &a, hipStream_t s);
void launch_el2_inject(const El2RecArgs &a, hipStream_t s);
void launch_el2_adj1(const El2AdjArgs &a, hipStream_t s);
void launch_el2_adj2(const El2AdjArgs &a, hipStream_t s);
void launch_el2_adj3(const El2AdjArgs &a, hipStream_t s);
void launch_el2_prep(const Grid2 &g, int nmodels, const float *vp, const float *vs, const float *rho,
                     float *const *model, float *const *phys_pad, hipStream_t s);
void launch_el2_finalize(const Grid2 &g, int nmodels, int spm, const float *grad, long long grad_stride,
                         float *acc, const float *const *model, const float *const *phys_pad,
                         float *g_vp, float *g_vs, float *g_rho, hipStream_t s);

} // namespace sg
