// el2_internal.h -- launch arguments of the 2-D elastic kernels (not part of
// the public ABI).
#pragma once
#include "sg_internal.h"

namespace sg {

// ---------------------------------------------------------------- elastic 2-D
// Staggered velocity-stress fields on a 2-D frame (same frame as the 2-D
// acoustic fields); one thread per cell, cell blocks of EBX x (256 / EBX),
// EBX = 32 (32 x 8, the default) or 64 (64 x 4), a run-time setting of a
// model (set_tuning).  The forward passes and the adjoint's first two passes
// give each thread a group of gs shots of one model (by default
// el2_group(shots per model)); the forward passes number (cell block, shot
// group) in a 1-D grid, the adjoint passes take the shot group as the grid's
// y index.
constexpr int EBX_DEF = 32;
constexpr long long el2_cell_blocks(int ebx, long long NX, long long NZ)
{
    return (NX + ebx - 1) / ebx * ((NZ + 256 / ebx - 1) / (256 / ebx));
}
constexpr int EL_NS = 13;      // vx vz sxx szz sxz + 8 CPML memory variables
enum { E_VX, E_VZ, E_SXX, E_SZZ, E_SXZ, E_MVXX, E_MVXZ, E_MVZX, E_MVZZ,
       E_MSXXX, E_MSXZZ, E_MSXZX, E_MSZZZ };
enum { M_LAM, M_MU, M_MUXZ, M_BX, M_BZ };

struct El2Tabs {               // CPML a, b at integer (0) and half (1) positions
    const float *ax[2], *bx[2], *az[2], *bz[2];
};

__host__ __device__ constexpr int el2_group(int spm) { return spm % 4 == 0 ? 4 : spm % 2 == 0 ? 2 : 1; }

struct El2Args {
    Grid2 g;                   // NX, NZ, P, nx, nz, SX, SZ, plane (tiles unused)
    int nshots, shots_per_model;
    int gs, ebx;               // shots per thread (divides shots_per_model); cell block width
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
    int gs, ebx;               // as in El2Args
    float *a[EL_NS];           // adjoint state
    float *tmp[8];             // e1..e4 then d1..d4
    const float *m[5];
    El2Tabs t;
    float kap;
    const float *snap;
    long long snap_stride;
    float *grad;               // 5 accumulators [5][shot group][plane]
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
// pass 3 of step k with pass 1 of step k - 1 (a: the arguments of step k - 1)
void launch_el2_adj31(const El2AdjArgs &a, hipStream_t s);
void launch_el2_prep(const Grid2 &g, int nmodels, const float *vp, const float *vs, const float *rho,
                     float *const *model, float *const *phys_pad, hipStream_t s);
void launch_el2_finalize(const Grid2 &g, int nmodels, int spm, int gs, const float *grad, long long grad_stride,
                         float *acc, const float *const *model, const float *const *phys_pad,
                         float *g_vp, float *g_vs, float *g_rho, hipStream_t s);

} // namespace sg
