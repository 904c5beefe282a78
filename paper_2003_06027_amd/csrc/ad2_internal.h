// ad2_internal.h -- launch arguments of the 2-D divergence-form acoustic
// kernels (not part of the public ABI).  Fields live in the 2-D frame of
// sg_internal.h; half-node fields are stored at the index of the node below
// (x: (ix + 1/2, iz) at (ix, iz); z: (ix, iz + 1/2) at (ix, iz)).
#pragma once
#include "sg_internal.h"

namespace sg {

// CPML coefficients by padded index: a, b at the nodes (0) and at the half
// nodes (h) of each axis.
struct Ad2Cpml {
    const float *a0x, *b0x, *ahx, *bhx;
    const float *a0z, *b0z, *ahz, *bhz;
};

// Forward step k over (tile, shot) pairs.
struct Ad2FwdArgs {
    Grid2 g;
    int nshots, shots_per_model;
    const float *u;           // u^k [shot][plane]
    const float *um;          // u^{k-1}
    float *un;                // u^{k+1} (aliases um: each node reads um before writing)
    const float *psx, *psz;   // psi'^k at the half nodes (layer memory, x and z)
    float *psxn, *pszn;       // psi'^{k+1}
    float *xix, *xiz;         // xi' at the nodes, updated in place
    const float *chat;        // dt^2 c^2 / dx^2 [model][plane], replicated one node beyond the grid
    Ad2Cpml t;
    const float *wav;         // [shot][nsrc][nt]
    int nt, k, nsrc;
    float src_scale;          // dt^2 / (dx dz)
    const int *src_off;       // [shot][ntiles + 1] CSR over tiles
    const int *src_ent;       // src_pack(local cell, node), sorted per tile
    const int *rec_off, *rec_ent;
    float *seis;              // [shot][nt][nrec] or null
    int nrec;
    float *snx, *snz;         // S' = G' + psi'^{k+1} of this step [shot][plane], or null
};

// Adjoint launch k: lambda^k from lambda^{k+1}, lambda^{k+2}.
struct Ad2AdjArgs {
    Grid2 g;
    int nshots, shots_per_model;
    const float *l1;          // lambda^{k+1}
    const float *l2;          // lambda^{k+2}
    float *l0;                // lambda^k (aliases l2)
    const float *yx, *yz;     // Y^{k+2} = a * adjoint of xi' (nodes)
    float *yxn, *yzn;         // Y^{k+1}
    const float *zx, *zz;     // Z^{k+2} = ah * adjoint of psi' (half nodes)
    float *zxn, *zzn;         // Z^{k+1}
    const float *chat;
    Ad2Cpml t;
    int nt, k;
    const int *rec_off, *rec_ent;
    const float *dJdd;        // [shot][nt][nrec]; sample k-1 joins lambda^k
    int nrec;
    const float *snx, *snz;   // S' of forward step k, or null (no gradient term)
    float *gn;                // dJ/dchat at the nodes [shot][plane], accumulated
};

void launch_ad2_fwd(const Ad2FwdArgs &a, hipStream_t s);
void launch_ad2_adj(const Ad2AdjArgs &a, hipStream_t s);
void launch_ad2_prep(const Grid2 &g, int nmodels, const float *vp, double dt, double dx, float *chat,
                     float *cpad, hipStream_t s);
void launch_ad2_finalize(const Grid2 &g, int nmodels, int shots_per_model, const float *gn, float *acc,
                         const float *cpad, double dt, double dx, float *g_vp, hipStream_t s);

} // namespace sg
