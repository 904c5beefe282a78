// ac3_internal.h -- launch arguments of the 3-D acoustic kernels (not part
// of the public ABI).
#pragma once
#include "sg_internal.h"

namespace sg {

// ---------------------------------------------------------------- 3-D
// Tile of the 3-D kernels: TX3 x TY3 columns (one thread each), marching in
// z over chunks of planes with register windows along z.  The chunk lengths
// are run-time settings of a model (set_tuning; Grid3.zcf, zca and the
// layer work list), between TZC_MIN and TZC planes; the defaults are below:
// the forward passes and the layer work items take shorter chunks than the
// adjoint, whose longer march re-reads fewer window planes.
constexpr int TX3 = 32;
constexpr int TY3 = 16;
constexpr int NTH3 = TX3 * TY3;
constexpr int TZC = 64;    // the longest chunk (bounds every chunk's 32-bit plane offsets)
constexpr int TZC_MIN = 16;
constexpr int TZCA_DEF = 64;   // the adjoint tile passes
constexpr int TZCF_DEF = 32;   // the forward tile passes
constexpr int TZCI_DEF = 32;   // the layer work items
static_assert(TZCF_DEF <= TZC && TZCI_DEF <= TZC && TZCA_DEF <= TZC && TZC_MIN <= TZCF_DEF, "chunk bounds");
constexpr int OX3 = 32;  // x offset (128-byte aligned rows)
constexpr int OY3 = 4;
constexpr int OZ3 = 4;
constexpr int CELL3_BITS = 9;   // local cell of a TX3 x TY3 plane tile
static_assert(TX3 * TY3 <= (1 << CELL3_BITS) && CELL3_BITS <= 11, "tile cells fit the receiver entries");

struct Grid3 {
    int NX, NY, NZ;
    int P, nx, ny, nz;
    int SX, SY, SZ;
    long long sy, sz, plane;   // strides: sy = SX, sz = SX*SY, plane = sz*SZ
    int ntx, nty, nzc;         // tiles in x, y; adjoint z chunks
    int zcf, zca;              // planes per chunk: forward and adjoint tile passes
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
    int nfree;                 // the first nfree items have no cell with two axes in the layer
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

} // namespace sg
