// seisgrad.hip -- host runtime and C ABI of libseisgrad (see include/seisgrad.h).
//
// The runtime validates arguments, carves all device state from the caller's
// workspace, uploads the acquisition geometry, and drives the per-step
// kernels: the forward sweep with wavefield checkpoints every K steps, and
// the reverse sweep that restores each checkpoint, recomputes its segment
// (storing w~^k snapshots) and runs the adjoint steps backwards in time
// (two-level checkpointing; memory O(nt/K + K) wavefields instead of O(nt)).
#include "../../include/seisgrad.h"
#include "sg_internal.h"
#include "ad2_internal.h"
#include "ac3_internal.h"
#include "el2_internal.h"
#include "sg_error.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstring>
#include <string>
#include <vector>

using namespace sg;

namespace sg {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

} // namespace sg

namespace {

#define HIPCHECK(x)                                                                  \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            return fail(SG_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));     \
    } while (0)

constexpr double L8_SYMBOL_MAX = 6.501587301587301; // max |1-D 8th-order symbol| * dx^2
constexpr size_t ALIGN = 256;
constexpr int TABPAD = 4;   // damping tables carry 4 neutral entries on each side

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    int ndim;
    Grid2 g2;
    Grid3 g3;
    long long plane;   // floats per field per shot
    int ntiles;        // 2-D tiles, or 3-D xy tiles
    int nf;            // wavefield state fields (checkpointed)
    int K, nseg;
    long long field;   // floats of one field over max_shots
    int n[3];          // padded extents x, y, z (y = 1 in 2-D)
    bool elastic;
    bool ad2;          // 2-D acoustic in divergence form (staggered grid, CPML)
    int nsnap, ngrad, nmod; // snapshot fields per step, gradient accumulators, model fields
    int nxs;           // extra wavefield slots (2-D acoustic: u and s rotate over 4 slots, the layer
                       // auxiliaries over 2 pairs)
    size_t off_chat, off_cpad, off_tab, off_fwd, off_adj, off_ckpt, off_snap,
        off_grad, off_src, off_recoff, off_recent, off_part, off_tmp, off_acc, off_uoff, off_uid, off_mt,
        off_tiles, off_soff, off_sent, off_nodef, off_items, off_flag, total;
};

int check_desc(const sg_desc *d)
{
    if (!d) return fail(SG_EINVAL, "descriptor is NULL");
    if (d->physics != SG_ACOUSTIC && d->physics != SG_ELASTIC && d->physics != SG_ACOUSTIC_DIV)
        return fail(SG_EUNSUPPORTED, "physics %d is not provided by this build", d->physics);
    if (d->ndim != 2 && d->ndim != 3) return fail(SG_EUNSUPPORTED, "ndim %d is not provided by this build", d->ndim);
    if (d->physics == SG_ELASTIC && d->ndim != 2) return fail(SG_EUNSUPPORTED, "elastic modelling is 2-D in this build");
    if (d->physics == SG_ACOUSTIC_DIV && d->ndim != 2)
        return fail(SG_EUNSUPPORTED, "the divergence-form acoustic equation is 2-D in this build");
    const int ny = d->ndim == 3 ? d->ny : 1;
    if (d->nx < 1 || d->nz < 1 || ny < 1 || d->npml < 0 || d->nt < 1 || d->nmodels < 1)
        return fail(SG_EINVAL, "bad grid: nx=%d ny=%d nz=%d npml=%d nt=%d nmodels=%d", d->nx, d->ny, d->nz,
                    d->npml, d->nt, d->nmodels);
    if (!(d->dx > 0) || !(d->dt > 0)) return fail(SG_EINVAL, "dx and dt must be positive");
    if (d->npml > 0 && (!(d->pml_R > 0 && d->pml_R < 1) || !(d->pml_vmax > 0)))
        return fail(SG_EINVAL, "absorbing layer needs 0 < pml_R < 1 and pml_vmax > 0");
    const long long cells = (long long)(d->nx + 2 * d->npml) * (ny + (d->ndim == 3 ? 2 * d->npml : 0)) *
                            (d->nz + 2 * d->npml);
    if (cells > (1LL << 33)) return fail(SG_EINVAL, "grid too large");
    if (d->ndim == 3) {
        // the 3-D tile passes address a z chunk and its window planes with
        // 32-bit byte offsets
        const long long NX = d->nx + 2LL * d->npml, NY = d->ny + 2LL * d->npml;
        const long long SX = OX3 + (NX + TX3 - 1) / TX3 * TX3 + 32, SY = OY3 + (NY + TY3 - 1) / TY3 * TY3 + 4;
        if ((TZC + 12) * SX * SY * 4 >= (1LL << 32))
            return fail(SG_EUNSUPPORTED, "3-D grid planes of %lld x %lld cells exceed this build's limit", NX, NY);
        // receiver entries are sorted by (tile, plane) with a 12-bit plane field
        if (d->nz + 2LL * d->npml >= 4096)
            return fail(SG_EUNSUPPORTED, "3-D grids are limited to %d padded planes in z", 4095);
    }
    return SG_OK;
}

// Shot-count limits of the elastic launches: the adjoint passes take the shot
// (group) as the grid's y index (at most 65535); the forward passes number
// (cell block, shot group) in a 1-D grid of int work ids, at most
// el2_cell_blocks * max_shots of them (shot groups of one, either block width).
int check_shots(const sg_desc *d, int max_shots)
{
    if (d->physics != SG_ELASTIC) return SG_OK;
    const long long NX = d->nx + 2LL * d->npml, NZ = d->nz + 2LL * d->npml;
    const long long nblk = std::max(el2_cell_blocks(32, NX, NZ), el2_cell_blocks(64, NX, NZ));
    if (max_shots > 65535 || nblk * max_shots >= (1LL << 31))
        return fail(SG_EINVAL, "too many elastic shots (%d) for a %lld x %lld grid", max_shots, NX, NZ);
    return SG_OK;
}

// Entries of the 3-D layer pass's work list: per xy tile at most one item
// per TZC_MIN planes plus one for each of the three z ranges (slab, interior,
// slab) an item may not straddle, and, in each of the list's two parts, the
// padding of one group per distinct first plane (see build_items3).
size_t items3_cap(int ntiles, int NZ)
{
    const size_t per_col = (size_t)(NZ + TZC_MIN - 1) / TZC_MIN + 3;
    return (size_t)ntiles * per_col + 2 * per_col * (NXCD - 1);
}

Layout make_layout(const sg_desc *d, int max_shots, int max_rec, int ckpt)
{
    Layout L{};
    L.ndim = d->ndim;
    L.elastic = d->physics == SG_ELASTIC;
    L.ad2 = d->physics == SG_ACOUSTIC_DIV;
    L.nsnap = 1;
    L.ngrad = 1;
    L.nmod = 2;            // chat, padded velocity
    const int P = d->npml;
    if (L.elastic) {
        Grid2 &g = L.g2;
        g.P = P; g.nx = d->nx; g.nz = d->nz;
        g.NX = d->nx + 2 * P; g.NZ = d->nz + 2 * P;
        g.ntx = g.ntz = 0;
        g.SX = OX + (g.NX + 31) / 32 * 32 + 32;
        g.SZ = OZ + g.NZ + 8;
        g.plane = (long long)g.SX * g.SZ;
        L.plane = g.plane;
        L.ntiles = 0;
        L.nf = EL_NS;
        L.nsnap = 5;
        L.ngrad = 5;
        L.nmod = 8;        // lam, mu, muxz, bx, bz + padded vp, vs, rho
        L.n[0] = g.NX; L.n[1] = 1; L.n[2] = g.NZ;
    } else if (d->ndim == 2) {
        Grid2 &g = L.g2;
        g.P = P; g.nx = d->nx; g.nz = d->nz;
        g.NX = d->nx + 2 * P; g.NZ = d->nz + 2 * P;
        g.ntx = (g.NX + TX - 1) / TX; g.ntz = (g.NZ + TZ - 1) / TZ;
        g.SX = OX + g.ntx * TX + 32;
        g.SZ = OZ + g.ntz * TZ + 8;
        g.plane = (long long)g.SX * g.SZ;
        L.plane = g.plane;
        L.ntiles = g.ntx * g.ntz;
        L.nf = 4;
        L.nxs = 4;
        if (L.ad2) {
            // state u^k, u^{k-1}, psi'x, psi'z, xi'x, xi'z; the second psi' buffers
            // (forward) and the adjoint's 10 fields use the extra slots
            L.nf = 6;
            L.nxs = 4;
            L.nsnap = 2;   // S'x, S'z per step
        }
        L.n[0] = g.NX; L.n[1] = 1; L.n[2] = g.NZ;
    } else {
        Grid3 &g = L.g3;
        g.P = P; g.nx = d->nx; g.ny = d->ny; g.nz = d->nz;
        g.NX = d->nx + 2 * P; g.NY = d->ny + 2 * P; g.NZ = d->nz + 2 * P;
        g.ntx = (g.NX + TX3 - 1) / TX3; g.nty = (g.NY + TY3 - 1) / TY3;
        g.zcf = TZCF_DEF;
        g.zca = TZCA_DEF;
        g.nzc = (g.NZ + g.zca - 1) / g.zca;
        g.SX = OX3 + g.ntx * TX3 + 32;
        g.SY = OY3 + g.nty * TY3 + 4;
        g.SZ = OZ3 + g.NZ + 4;
        g.sy = g.SX;
        g.sz = (long long)g.SX * g.SY;
        g.plane = g.sz * g.SZ;
        L.plane = g.plane;
        L.ntiles = g.ntx * g.nty;
        L.nf = 6;
        L.n[0] = g.NX; L.n[1] = g.NY; L.n[2] = g.NZ;
    }
    L.K = ckpt > 0 ? ckpt : (int)std::ceil(std::sqrt((double)d->nt));
    if (L.K > d->nt) L.K = d->nt;
    L.nseg = (d->nt + L.K - 1) / L.K;
    L.field = (long long)max_shots * L.plane;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.off_chat = take(sizeof(float) * (size_t)L.nmod * d->nmodels * L.plane);   // model fields
    L.off_cpad = L.off_chat + sizeof(float) * (size_t)d->nmodels * L.plane;
    L.off_tab = take(sizeof(float) * 4 * (L.n[0] + L.n[1] + L.n[2] + 6 * TABPAD));
    L.off_fwd = take(sizeof(float) * (L.nf + L.nxs) * L.field);
    L.off_adj = take(sizeof(float) * (L.nf + L.nxs) * L.field);
    L.off_ckpt = take(sizeof(float) * (size_t)L.nseg * L.nf * L.field);
    L.off_snap = take(sizeof(float) * (size_t)L.K * L.nsnap * L.field);
    L.off_grad = take(sizeof(float) * (size_t)L.ngrad * L.field);
    L.off_src = take(sizeof(long long) * max_shots);
    L.off_recoff = take(sizeof(int) * (size_t)max_shots * (L.ntiles + 1));
    L.off_recent = take(std::max(sizeof(int2), sizeof(long long)) * std::max<size_t>(1, (size_t)max_shots * max_rec));
    L.off_part = take(sizeof(double) * NOALLOC_PARTS);
    L.off_tmp = take(L.elastic ? sizeof(float) * 8 * L.field : 0);
    L.off_acc = take(sizeof(float) * 8 * (size_t)d->nmodels * L.plane);
    L.off_uoff = take(sizeof(int) * (size_t)max_shots * (max_rec + 1));
    L.off_uid = take(sizeof(int) * std::max<size_t>(1, (size_t)max_shots * max_rec));
    L.off_mt = take(sizeof(float) * 3 * max_shots);
    L.off_tiles = take(sizeof(int) * 2 * std::max(1, L.ntiles));
    L.off_soff = take(sizeof(int) * (size_t)max_shots * (L.ntiles + 1));
    L.off_sent = take(sizeof(int) * (size_t)max_shots * SG_MAX_SRC);
    L.off_nodef = take(sizeof(long long) * (size_t)max_shots * SG_MAX_SRC);
    L.off_items = take(L.ndim == 3 ? sizeof(int4) * 2 * items3_cap(L.ntiles, L.g3.NZ) : 0);
    L.off_flag = take(sizeof(int));
    L.total = o;
    return L;
}

} // namespace

struct sg_model {
    sg_desc d;
    Layout L;
    int max_shots, max_rec;
    char *ws;
    float *chat, *cpad;
    float *h[3], *p[3], *ih[3];   // damping tables per axis (x, y, z)
    float *fwd[EL_NS], *adj[EL_NS], *tmp[8];
    // 2-D acoustic: u^t lives in slot u4[t % 4], the adjoint s^t in s4[t % 4]
    float *u4[4], *s4[4];
    // 2-D acoustic tiles advanced one step per launch ("near": the layer within
    // reach, or receivers within 4 cells) and two steps per launch ("blocked")
    int *tiles_near = nullptr, *tiles_blk = nullptr;
    // several source nodes per shot (2-D acoustic): per-tile CSR and node frame indices
    int *src_off = nullptr, *src_ent = nullptr;
    long long *node_f = nullptr;
    int geom_nsrc = 1;
    std::vector<int> h_soff, h_sent;
    std::vector<long long> h_nodef;
    int n_near = 0, n_blk = 0;      // one-step tiles (the first n_layer_near by the layer), blocked tiles
    int n_layer_near = 0;
    std::vector<int> h_tiles;
    // tiles holding layer cells (the layer pass of the constant-density form)
    int *tiles_layer = nullptr;
    int n_layer = 0;
    std::vector<int> h_layer;
    // 3-D acoustic layer pass: (xy tile, first plane, end plane) work items
    int4 *items3 = nullptr;
    int n_items3 = 0;
    int n_items3_free = 0;        // the leading items whose cells have at most one axis in the layer
    int4 *items3a = nullptr;      // the adjoint's list
    int n_items3a = 0;
    std::vector<int4> h_items3a;
    int zci = 0;                  // planes per layer work item
    // elastic launch settings: shots per thread (0: el2_group of the shots per
    // model) and cell block width
    int el_gs = 0, el_ebx = EBX_DEF;
    std::vector<int4> h_items3;
    // 3-D xy tiles, those within the stencil reach of the layer in x or y first
    int *tiles3 = nullptr;
    int n_near3 = 0;
    std::vector<int> h_tiles3;
    int steps_per_launch = 2;
    bool pair = true;             // 2-D: near step k and blocked steps k, k+1 in one launch
    // snapshots of the last n_store checkpoint segments, written by a
    // checkpointed forward into the workspace beyond its minimum size
    float *store = nullptr;
    int n_store = 0;
    bool have_store = false;
    float *model[8];              // elastic: lam, mu, muxz, bx, bz, vp, vs, rho (padded)
    float *ckpt, *snap, *grad, *acc;
    int *uoff, *uid;
    float *mt;
    float *cpml[2][4];            // elastic CPML tables: [x|z][a0, b0, a1, b1]
    int nuniq_max = 0;
    std::vector<int> h_uoff, h_uid;
    std::vector<long long> h_recf;
    std::vector<float> h_mt;
    long long *src_f;
    int *rec_off;
    void *rec_ent;
    double *partials;
    int *numeric_flag;            // set on the device by a non-finite misfit
    std::vector<float> h_tab;
    std::vector<long long> h_src;
    std::vector<int> h_off, h_ent;
    std::vector<int2> h_ent3;
    std::vector<int32_t> geom_src, geom_rec;  // geometry as uploaded
    int geom_nshots = -1, geom_nrec = -1;
    bool have_ckpt = false;
    // optional device timing of the step loops: one event pair per segment
    struct Span { int phase; int steps; hipEvent_t a, b; };
    bool profiling = false;
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    // graph mode: one executable graph per checkpoint segment and sweep
    // (forward; restore + recompute + adjoint), captured on a stream of the
    // model and replayed on the caller's while the arguments they hold match
    struct SegGraph { uint64_t key = 0; hipGraphExec_t exec = nullptr; };
    bool graphs = false;
    hipStream_t cap = nullptr;
    std::vector<SegGraph> gfwd[2], gadj;   // forward: without / with checkpoints
    uint64_t epoch = 1;           // bumped by every change of launch settings or geometry
    ~sg_model()
    {
        for (auto &sp : spans) { pool.push_back(sp.a); pool.push_back(sp.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (auto *v : {&gfwd[0], &gfwd[1], &gadj})
            for (auto &g : *v)
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

bool same_geometry(const sg_model *m, const sg_shots *sh)
{
    const int nd = m->d.ndim, ns = sh->nshots;
    if (m->L.elastic) {
        if (!sh->mt || m->h_mt.size() != (size_t)3 * ns) return false;
        for (int i = 0; i < 3 * ns; ++i)
            if (m->h_mt[i] != sh->mt[i]) return false;
    }
    const int nsrc = sh->nsrc < 1 ? 1 : sh->nsrc;
    return m->geom_nshots == ns && m->geom_nrec == sh->nrec && m->geom_nsrc == nsrc &&
           std::equal(sh->src, sh->src + (size_t)nd * ns * nsrc, m->geom_src.begin()) &&
           (sh->nrec == 0 || std::equal(sh->rec, sh->rec + (size_t)nd * ns * sh->nrec, m->geom_rec.begin()));
}

// The 3-D layer pass's work list (host copy): every plane of the xy tiles
// that touch the layer in x or y, the two z slabs of the others, in items of
// at most zci planes.  The items are grouped by their first plane, and each
// group is laid out in launch order: the hardware deals consecutive
// workgroups to the XCDs in turn, so the group's n items are padded to a
// multiple of NXCD (entries with tile -1, which return at once) and placed
// so that XCD x takes the contiguous run x * per .. x * per + per - 1 of
// them (per = ceil(n / NXCD)).  All XCDs then work on the same planes, each
// on neighbouring tiles.  Two lists: the forward's, in two parts (the items
// without psi terms first, each part grouped as above; the tiles by the
// layer split at the z-slab boundaries so that an item is wholly in one
// part), and the adjoint's, one list as above.  Returns nonzero, leaving the
// model's lists as they were, if a list would overflow its workspace slot.
int build_items3(sg_model *m, int zci)
{
    const Layout &L = m->L;
    const Grid3 &g = L.g3;
    // forward: items whose cells have at most one axis in the layer (no psi
    // term) first, then the others; adjoint (no psi): one list in which the
    // tiles by the layer take whole columns
    std::vector<int4> raw[2], rawa;
    for (int t = 0; t < L.ntiles; ++t) {
        const int x0 = (t % g.ntx) * TX3, y0 = (t / g.ntx) * TY3;
        const bool lx = x0 < g.P || x0 + TX3 > g.P + g.nx, ly = y0 < g.P || y0 + TY3 > g.P + g.ny;
        auto add = [&](int za, int zb) {
            for (int z = za; z < zb; z += zci) {
                const int ze = std::min(z + zci, zb);
                const bool lz = z < g.P || ze > g.P + g.nz;
                const bool two = (lx && ly) || ((lx || ly) && lz);
                raw[two].push_back(make_int4(t, z, ze, 0));
            }
        };
        auto adda = [&](int za, int zb) {
            for (int z = za; z < zb; z += zci) rawa.push_back(make_int4(t, z, std::min(z + zci, zb), 0));
        };
        if (lx || ly) {
            add(0, g.P);                 // items never straddle a z-slab boundary
            add(g.P, g.P + g.nz);
            add(g.P + g.nz, g.NZ);
            adda(0, g.NZ);
        } else {
            add(0, g.P);
            add(g.P + g.nz, g.NZ);
            adda(0, g.P);
            adda(g.P + g.nz, g.NZ);
        }
    }
    // each list grouped by first plane, each group in launch order
    auto order = [](std::vector<int4> &r, std::vector<int4> &out) {
        std::stable_sort(r.begin(), r.end(), [](const int4 &a, const int4 &b) { return a.y < b.y; });
        for (size_t b = 0; b < r.size();) {
            size_t e = b;
            while (e < r.size() && r[e].y == r[b].y) ++e;
            const size_t n = e - b, per = (n + NXCD - 1) / NXCD;
            for (size_t sl = 0; sl < per * NXCD; ++sl) {
                const size_t i = (sl % NXCD) * per + sl / NXCD;
                out.push_back(i < n ? r[b + i] : make_int4(-1, 0, 0, 0));
            }
            b = e;
        }
    };
    std::vector<int4> out, outa;
    order(raw[0], out);
    const size_t nfree = out.size();
    order(raw[1], out);
    order(rawa, outa);
    const size_t cap = items3_cap(L.ntiles, g.NZ);
    if (out.size() > cap || outa.size() > cap) return 1;    // the model keeps its lists
    m->h_items3.swap(out);
    m->n_items3 = (int)m->h_items3.size();
    m->n_items3_free = (int)nfree;
    m->h_items3a.swap(outa);
    m->n_items3a = (int)m->h_items3a.size();
    m->zci = zci;
    return 0;
}

// Shots per thread of the elastic passes for spm shots per model: the
// model's setting if it divides spm, else el2_group(spm).
int el_group(const sg_model *m, int spm)
{
    return m->el_gs > 0 && spm % m->el_gs == 0 ? m->el_gs : el2_group(spm);
}

int upload_geometry(sg_model *m, const sg_shots *sh, hipStream_t s)
{
    const Layout &L = m->L;
    const int nd = m->d.ndim, ns = sh->nshots, nrec = sh->nrec, P = m->d.npml;
    const int phys[3] = {m->d.nx, nd == 3 ? m->d.ny : 1, m->d.nz};
    if (!sh->src || (nrec > 0 && !sh->rec)) return fail(SG_EINVAL, "source/receiver arrays are NULL");
    auto inside = [&](const int32_t *q) {
        for (int c = 0; c < nd; ++c) {
            const int axis = nd == 2 && c == 1 ? 2 : c;   // 2-D points are (ix, iz)
            if (q[c] < 0 || q[c] >= phys[axis]) return false;
        }
        return true;
    };
    const int nsrc = sh->nsrc < 1 ? 1 : sh->nsrc;
    for (int i = 0; i < ns; ++i) {
        for (int j = 0; j < nsrc; ++j)
            if (!inside(sh->src + ((size_t)i * nsrc + j) * nd))
                return fail(SG_EINVAL, "shot %d: source node %d outside the %dx%dx%d grid", i, j, phys[0], phys[1],
                            phys[2]);
        for (int r = 0; r < nrec; ++r)
            if (!inside(sh->rec + ((size_t)i * nrec + r) * nd))
                return fail(SG_EINVAL, "shot %d receiver %d outside the grid", i, r);
    }
    if (same_geometry(m, sh)) return SG_OK;
    ++m->epoch;                       // captured segment graphs hold the old lists and counts
    // the previous upload may still be reading the host vectors
    HIPCHECK(hipStreamSynchronize(s));
    if (L.elastic) {
        if (!sh->mt) return fail(SG_EINVAL, "elastic shots need moment tensors (mt)");
        const Grid2 &g = L.g2;
        auto frame = [&](const int32_t *q) { return (long long)(q[1] + P + OZ) * g.SX + q[0] + P + OX; };
        m->h_src.assign(ns, 0);
        m->h_recf.assign((size_t)std::max(1, ns * nrec), 0);
        m->h_mt.assign(sh->mt, sh->mt + 3 * ns);
        std::vector<std::vector<int>> groups(ns);
        int nu = 0;
        for (int i = 0; i < ns; ++i) {
            m->h_src[i] = frame(sh->src + 2 * i);
            std::vector<std::pair<long long, int>> byc;
            for (int r = 0; r < nrec; ++r) {
                const long long f = frame(sh->rec + ((size_t)i * nrec + r) * 2);
                m->h_recf[(size_t)i * nrec + r] = f;
                byc.push_back({f, r});
            }
            std::sort(byc.begin(), byc.end());
            int cnt = 0;
            for (size_t j = 0; j < byc.size(); ++j) cnt += (j == 0 || byc[j].first != byc[j - 1].first);
            nu = std::max(nu, cnt);
            for (auto &pr : byc) groups[i].push_back(pr.second);   // receiver ids by cell
        }
        m->nuniq_max = nu;
        m->h_uoff.assign((size_t)ns * (nu + 1), 0);
        m->h_uid.clear();
        for (int i = 0; i < ns; ++i) {
            int *off = m->h_uoff.data() + (size_t)i * (nu + 1);
            int u = 0;
            long long prev = -1;
            const size_t base = m->h_uid.size();
            for (size_t j = 0; j < groups[i].size(); ++j) {
                const int r = groups[i][j];
                const long long f = m->h_recf[(size_t)i * nrec + r];
                if (j == 0 || f != prev) off[u++] = (int)(base + j);
                prev = f;
                m->h_uid.push_back(r);
            }
            for (; u <= nu; ++u) off[u] = (int)m->h_uid.size();
        }
        HIPCHECK(hipMemcpyAsync(m->src_f, m->h_src.data(), sizeof(long long) * ns, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->mt, m->h_mt.data(), sizeof(float) * 3 * ns, hipMemcpyHostToDevice, s));
        if (nrec > 0) {
            HIPCHECK(hipMemcpyAsync(m->rec_ent, m->h_recf.data(), sizeof(long long) * ns * nrec, hipMemcpyHostToDevice, s));
            HIPCHECK(hipMemcpyAsync(m->uoff, m->h_uoff.data(), sizeof(int) * m->h_uoff.size(), hipMemcpyHostToDevice, s));
            HIPCHECK(hipMemcpyAsync(m->uid, m->h_uid.data(), sizeof(int) * m->h_uid.size(), hipMemcpyHostToDevice, s));
        }
        m->geom_src.assign(sh->src, sh->src + (size_t)nd * ns);
        if (nrec > 0) m->geom_rec.assign(sh->rec, sh->rec + (size_t)nd * ns * nrec);
        else m->geom_rec.clear();
        m->geom_nshots = ns;
        m->geom_nrec = nrec;
        m->geom_nsrc = 1;
        m->have_ckpt = false;
        return SG_OK;
    }
    const int ntiles = L.ntiles;
    m->h_src.assign(ns, 0);
    m->h_off.assign((size_t)ns * (ntiles + 1), 0);
    m->h_ent.clear();
    m->h_ent3.clear();
    std::vector<std::pair<long long, int>> keyed;
    if (nsrc > 1 || L.ad2) {
        // several source nodes per shot (and every divergence-form shot): no
        // fused point source; per (shot, tile)
        // lists of (local cell, node) and the frame index of every node
        const Grid2 &g = L.g2;
        m->h_soff.assign((size_t)ns * (ntiles + 1), 0);
        m->h_sent.clear();
        m->h_nodef.assign((size_t)ns * nsrc, 0);
        for (int i = 0; i < ns; ++i) {
            std::vector<std::pair<int, int>> byt;   // (tile, packed entry)
            for (int j = 0; j < nsrc; ++j) {
                const int32_t *q = sh->src + ((size_t)i * nsrc + j) * 2;
                const int px = q[0] + P, pz = q[1] + P;
                m->h_nodef[(size_t)i * nsrc + j] = (long long)(pz + OZ) * g.SX + px + OX;
                byt.push_back({(pz / TZ) * g.ntx + px / TX, src_pack((pz % TZ) * TX + px % TX, j)});
            }
            std::sort(byt.begin(), byt.end());
            int *off = m->h_soff.data() + (size_t)i * (ntiles + 1);
            size_t e = 0;
            for (int tl = 0; tl < ntiles; ++tl) {
                off[tl] = (int)m->h_sent.size();
                while (e < byt.size() && byt[e].first == tl) m->h_sent.push_back(byt[e++].second);
            }
            off[ntiles] = (int)m->h_sent.size();
        }
        HIPCHECK(hipMemcpyAsync(m->src_off, m->h_soff.data(), sizeof(int) * m->h_soff.size(), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->src_ent, m->h_sent.data(), sizeof(int) * m->h_sent.size(), hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->node_f, m->h_nodef.data(), sizeof(long long) * m->h_nodef.size(),
                                hipMemcpyHostToDevice, s));
    }
    for (int i = 0; i < ns; ++i) {
        const int32_t *q = sh->src + (size_t)nd * nsrc * i;
        if (nsrc > 1 || L.ad2) {
            m->h_src[i] = -1;
        } else if (nd == 2) {
            const Grid2 &g = L.g2;
            m->h_src[i] = (long long)(q[1] + P + OZ) * g.SX + q[0] + P + OX;
        } else {
            const Grid3 &g = L.g3;
            m->h_src[i] = (long long)(q[2] + P + OZ3) * g.sz + (long long)(q[1] + P + OY3) * g.sy + q[0] + P + OX3;
        }
        keyed.clear();
        for (int r = 0; r < nrec; ++r) {
            const int32_t *e = sh->rec + ((size_t)i * nrec + r) * nd;
            if (nd == 2) {
                const int px = e[0] + P, pz = e[1] + P;
                const int tile = (pz / TZ) * L.g2.ntx + px / TX;
                const int cell = (pz % TZ) * TX + px % TX;
                keyed.push_back({(long long)tile << 42 | (long long)cell << 21 | r, rec_pack(cell, r)});
            } else {
                const int px = e[0] + P, py = e[1] + P, pz = e[2] + P;
                const int tile = (py / TY3) * L.g3.ntx + px / TX3;
                const int cell = (py % TY3) * TX3 + px % TX3;
                // key: tile (bits 44..), plane (32..43), cell (21..31), receiver (0..20)
                keyed.push_back({(long long)tile << 44 | (long long)pz << 32 | (long long)cell << 21 | r, r});
            }
        }
        std::sort(keyed.begin(), keyed.end());
        int *off = m->h_off.data() + (size_t)i * (ntiles + 1);
        const size_t base = nd == 2 ? m->h_ent.size() : m->h_ent3.size();
        size_t e = 0;
        for (int tl = 0; tl < ntiles; ++tl) {
            off[tl] = (int)(base + e);
            while (e < keyed.size() && (int)(keyed[e].first >> (nd == 2 ? 42 : 44)) == tl) {
                if (nd == 2) {
                    m->h_ent.push_back(keyed[e].second);
                } else {
                    const long long k = keyed[e].first;
                    const int pz = (int)((k >> 32) & 0xFFF), cell = (int)((k >> 21) & 0x7FF);
                    m->h_ent3.push_back(make_int2((pz << CELL3_BITS) | cell, keyed[e].second));
                }
                ++e;
            }
        }
        off[ntiles] = (int)(base + e);
    }
    if (nd == 2) {
        // blocked tiles: the tile and its BLK_HALO-cell halo are physical cells,
        // and no receiver of any shot lies within 4 cells of the tile
        const Grid2 &g = L.g2;
        std::vector<char> rec_near(ntiles, 0);
        const int nnode = nsrc > 1 ? nsrc : 0;     // source nodes handled by the one-step kernel
        for (int i = 0; i < ns; ++i)
            for (int r = 0; r < nrec + nnode; ++r) {
                const int32_t *e = r < nrec ? sh->rec + ((size_t)i * nrec + r) * nd
                                            : sh->src + ((size_t)i * nsrc + (r - nrec)) * nd;
                const int px = e[0] + P, pz = e[1] + P;
                for (int tz = std::max(0, (pz - 4) / TZ - 1); tz <= std::min(g.ntz - 1, (pz + 4) / TZ); ++tz)
                    for (int tx = std::max(0, (px - 4) / TX - 1); tx <= std::min(g.ntx - 1, (px + 4) / TX); ++tx)
                        if (px >= tx * TX - 4 && px < tx * TX + TX + 4 && pz >= tz * TZ - 4 && pz < tz * TZ + TZ + 4)
                            rec_near[tz * g.ntx + tx] = 1;
            }
        // one-step tiles: those within 4 cells of the layer (their kernel folds
        // the layer pass in) first, then the others; then the blocked tiles
        std::vector<int> near, other, blk;
        for (int t = 0; t < ntiles; ++t) {
            const int x0 = (t % g.ntx) * TX, z0 = (t / g.ntx) * TZ;
            const bool inner = x0 - BLK_HALO >= P && x0 + TX + BLK_HALO <= P + g.nx &&
                               z0 - BLK_HALO >= P && z0 + TZ + BLK_HALO <= P + g.nz;
            const bool by_layer = P > 0 && (x0 - 4 < P || x0 + TX + 4 > P + g.nx ||
                                            z0 - 4 < P || z0 + TZ + 4 > P + g.nz);
            (by_layer ? near : inner && !rec_near[t] ? blk : other).push_back(t);
        }
        m->n_layer_near = (int)near.size();
        m->n_near = (int)(near.size() + other.size());
        m->n_blk = (int)blk.size();
        m->h_tiles = near;
        m->h_tiles.insert(m->h_tiles.end(), other.begin(), other.end());
        m->h_tiles.insert(m->h_tiles.end(), blk.begin(), blk.end());
        HIPCHECK(hipMemcpyAsync(m->tiles_near, m->h_tiles.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice, s));
        m->tiles_blk = m->tiles_near + m->n_near;
    }
    HIPCHECK(hipMemcpyAsync(m->src_f, m->h_src.data(), sizeof(long long) * ns, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(m->rec_off, m->h_off.data(), sizeof(int) * m->h_off.size(), hipMemcpyHostToDevice, s));
    if (nd == 2 && !m->h_ent.empty())
        HIPCHECK(hipMemcpyAsync(m->rec_ent, m->h_ent.data(), sizeof(int) * m->h_ent.size(), hipMemcpyHostToDevice, s));
    if (nd == 3 && !m->h_ent3.empty())
        HIPCHECK(hipMemcpyAsync(m->rec_ent, m->h_ent3.data(), sizeof(int2) * m->h_ent3.size(), hipMemcpyHostToDevice, s));
    m->geom_src.assign(sh->src, sh->src + (size_t)nd * ns * nsrc);
    if (nrec > 0) m->geom_rec.assign(sh->rec, sh->rec + (size_t)nd * ns * nrec);
    else m->geom_rec.clear();
    m->geom_nshots = ns;
    m->geom_nrec = nrec;
    m->geom_nsrc = nsrc;
    m->have_ckpt = false;
    return SG_OK;
}

// The runtime's view of where p lives, when it has one: the attribute query
// fails on plain pageable host memory on some runtimes; that failure is
// cleared so later launch checks do not report it, and the pointer is then
// taken as host memory.
hipMemoryType memory_type(const void *p)
{
    hipPointerAttribute_t a;
    if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return hipMemoryTypeUnregistered;
    }
    return a.type;
}

int check_shots(const sg_model *m, const sg_shots *sh)
{
    if (!sh) return fail(SG_EINVAL, "shots is NULL");
    // src, rec and mt are read by the host while the geometry is uploaded: a
    // device address there would fault the host process, so it is refused
    if (memory_type(sh->src) == hipMemoryTypeDevice || memory_type(sh->rec) == hipMemoryTypeDevice ||
        memory_type(sh->mt) == hipMemoryTypeDevice)
        return fail(SG_EINVAL, "src, rec and mt are HOST arrays; a device pointer was passed");
    if (m->L.elastic && !sh->mt) return fail(SG_EINVAL, "elastic shots need moment tensors (mt)");
    if (sh->nshots < 1 || sh->nshots > m->max_shots)
        return fail(SG_EINVAL, "nshots %d outside [1, %d]", sh->nshots, m->max_shots);
    if (sh->nshots % m->d.nmodels)
        return fail(SG_EINVAL, "nshots %d is not a multiple of nmodels %d", sh->nshots, m->d.nmodels);
    if (sh->nrec < 0 || sh->nrec > m->max_rec)
        return fail(SG_EINVAL, "nrec %d outside [0, %d]", sh->nrec, m->max_rec);
    if (!sh->wavelet) return fail(SG_EINVAL, "wavelet is NULL");
    if (sh->nsrc < 0 || sh->nsrc > SG_MAX_SRC) return fail(SG_EINVAL, "nsrc %d outside [0, %d]", sh->nsrc, SG_MAX_SRC);
    if (sh->nsrc > 1 && (m->L.elastic || m->d.ndim != 2))
        return fail(SG_EUNSUPPORTED, "several source nodes per shot are provided for the 2-D acoustic equation only");
    return SG_OK;
}

hipEvent_t take_event(sg_model *m)
{
    if (!m->pool.empty()) {
        hipEvent_t e = m->pool.back();
        m->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Record the start of a timed loop of `steps` steps of `phase`
// (0 forward, 1 recompute, 2 adjoint); returns the span index or -1.
int span_begin(sg_model *m, int phase, int steps, hipStream_t s)
{
    if (!m->profiling) return -1;
    sg_model::Span sp{phase, steps, take_event(m), take_event(m)};
    if (!sp.a || !sp.b) return -1;
    (void)hipEventRecord(sp.a, s);
    m->spans.push_back(sp);
    return (int)m->spans.size() - 1;
}

void span_end(sg_model *m, int i, hipStream_t s)
{
    if (i >= 0) (void)hipEventRecord(m->spans[i].b, s);
}

float src_scale(const sg_model *m)
{
    const double dx = m->d.dx;
    return (float)(m->d.dt * m->d.dt / (m->d.ndim == 2 ? dx * dx : dx * dx * dx));
}

Ac3Tabs tabs3(const sg_model *m)
{
    Ac3Tabs t;
    for (int j = 0; j < 3; ++j) { t.h[j] = m->h[j]; t.p[j] = m->p[j]; t.ih[j] = m->ih[j]; }
    return t;
}

El2Tabs el_tabs(const sg_model *m)
{
    El2Tabs t;
    for (int h = 0; h < 2; ++h) {
        t.ax[h] = m->cpml[0][2 * h];
        t.bx[h] = m->cpml[0][2 * h + 1];
        t.az[h] = m->cpml[1][2 * h];
        t.bz[h] = m->cpml[1][2 * h + 1];
    }
    return t;
}

// One elastic step: velocity update, receiver record, stress update (+ source).
void el_fwd_step(const sg_model *m, int ns, const float *wav, int k, float *seis, float *snap, hipStream_t s)
{
    El2Args a{};
    a.g = m->L.g2;
    a.nshots = ns;
    a.shots_per_model = ns / m->d.nmodels;
    a.gs = el_group(m, a.shots_per_model);
    a.ebx = m->el_ebx;
    for (int i = 0; i < EL_NS; ++i) a.f[i] = m->fwd[i];
    for (int i = 0; i < 5; ++i) a.m[i] = m->model[i];
    a.t = el_tabs(m);
    a.kap = (float)(m->d.dt / m->d.dx);
    a.snap = snap;
    a.snap_stride = m->L.field;
    a.src_f = m->src_f;
    a.mt = m->mt;
    a.wav = wav;
    a.nt = m->d.nt;
    a.k = k;
    a.src_scale = (float)(m->d.dt / (m->d.dx * m->d.dx));
    launch_el2_vel(a, s);
    if (seis && m->geom_nrec > 0) {
        El2RecArgs r{};
        r.nshots = ns; r.nrec = m->geom_nrec; r.nt = m->d.nt; r.k = k;
        r.rec_f = static_cast<const long long *>(m->rec_ent);
        r.plane = m->L.plane;
        r.vx = m->fwd[E_VX]; r.vz = m->fwd[E_VZ];
        r.seis = seis;
        launch_el2_record(r, s);
    }
    launch_el2_str(a, s);
}

// Elastic adjoint step k: pass 1 (unless the previous launch ran it: first =
// false), the receiver injection, pass 2, and pass 3 -- with the next step's
// pass 1 when that step's snapshots are at hand (snap_next, step k - 1 of
// the same segment).
void el_adj_step(const sg_model *m, int ns, int k, const float *dJdd, float *gwav, const float *snap, hipStream_t s,
                 bool first = true, const float *snap_next = nullptr)
{
    El2AdjArgs a{};
    a.g = m->L.g2;
    a.nshots = ns;
    a.shots_per_model = ns / m->d.nmodels;
    a.gs = el_group(m, a.shots_per_model);
    a.ebx = m->el_ebx;
    for (int i = 0; i < EL_NS; ++i) a.a[i] = m->adj[i];
    for (int i = 0; i < 8; ++i) a.tmp[i] = m->tmp[i];
    for (int i = 0; i < 5; ++i) a.m[i] = m->model[i];
    a.t = el_tabs(m);
    a.kap = (float)(m->d.dt / m->d.dx);
    a.snap = snap;
    a.snap_stride = m->L.field;
    a.grad = m->grad;
    a.grad_stride = m->L.field;
    a.src_f = m->src_f;
    a.mt = m->mt;
    a.gwav = gwav;
    a.nt = m->d.nt;
    a.k = k;
    a.src_scale = (float)(m->d.dt / (m->d.dx * m->d.dx));
    if (first) launch_el2_adj1(a, s);
    if (m->geom_nrec > 0) {
        El2RecArgs r{};
        r.nshots = ns; r.nrec = m->geom_nrec; r.nt = m->d.nt; r.k = k;
        r.rec_f = static_cast<const long long *>(m->rec_ent);
        r.plane = m->L.plane;
        r.uoff = m->uoff; r.uid = m->uid; r.nuniq_max = m->nuniq_max;
        r.dJdd = dJdd;
        r.ax = m->adj[E_VX]; r.az = m->adj[E_VZ];
        launch_el2_inject(r, s);
    }
    launch_el2_adj2(a, s);
    if (snap_next) {
        El2AdjArgs b = a;
        b.k = k - 1;
        b.snap = snap_next;
        launch_el2_adj31(b, s);
    } else {
        launch_el2_adj3(a, s);
    }
}

// 2-D divergence form.  Forward: u^k in fwd[k & 1] (u^{k+1} overwrites
// u^{k-1}), psi'x^k, psi'z^k in fwd[2 + (k & 1)], fwd[4 + (k & 1)], xi'x, xi'z
// in fwd[6], fwd[7].  Adjoint: lambda^k in adj[k & 1], Y^k (x, z) in
// adj[2 + (k & 1)], adj[4 + (k & 1)], Z^k in adj[6 + (k & 1)], adj[8 + (k & 1)].
Ad2Cpml ad2_tabs(const sg_model *m)
{
    Ad2Cpml t;
    t.a0x = m->cpml[0][0]; t.b0x = m->cpml[0][1]; t.ahx = m->cpml[0][2]; t.bhx = m->cpml[0][3];
    t.a0z = m->cpml[1][0]; t.b0z = m->cpml[1][1]; t.ahz = m->cpml[1][2]; t.bhz = m->cpml[1][3];
    return t;
}

// Field i of the checkpointed state at the start of step k:
// (u^k, u^{k-1}, psi'x^k, psi'z^k, xi'x, xi'z).
float *ad2_state(const sg_model *m, int k, int i)
{
    switch (i) {
    case 0: return m->fwd[k & 1];
    case 1: return m->fwd[(k + 1) & 1];
    case 2: return m->fwd[2 + (k & 1)];
    case 3: return m->fwd[4 + (k & 1)];
    default: return m->fwd[i + 2];
    }
}

void ad2_fwd_step(const sg_model *m, int ns, const float *wav, int k, float *seis, float *snap, hipStream_t s)
{
    Ad2FwdArgs a{};
    a.g = m->L.g2;
    a.nshots = ns;
    a.shots_per_model = ns / m->d.nmodels;
    a.u = m->fwd[k & 1];
    a.um = m->fwd[(k + 1) & 1];
    a.un = m->fwd[(k + 1) & 1];
    a.psx = m->fwd[2 + (k & 1)];
    a.psxn = m->fwd[2 + ((k + 1) & 1)];
    a.psz = m->fwd[4 + (k & 1)];
    a.pszn = m->fwd[4 + ((k + 1) & 1)];
    a.xix = m->fwd[6];
    a.xiz = m->fwd[7];
    a.chat = m->chat;
    a.t = ad2_tabs(m);
    a.wav = wav;
    a.nt = m->d.nt;
    a.k = k;
    a.nsrc = m->geom_nsrc;
    a.src_scale = src_scale(m);
    a.src_off = m->src_off;
    a.src_ent = m->src_ent;
    a.rec_off = m->rec_off;
    a.rec_ent = static_cast<const int *>(m->rec_ent);
    a.seis = seis;
    a.nrec = m->geom_nrec;
    a.snx = snap;
    a.snz = snap ? snap + m->L.field : nullptr;
    launch_ad2_fwd(a, s);
}

// Adjoint launch k (k = nt: lambda^nt from the last sample alone, no
// gradient term); then dJ/dr_j(t_k) = dt^2/(dx dz) lambda^{k+1} at node j.
void ad2_adj_step(const sg_model *m, int ns, int k, const float *dJdd, float *gwav, const float *snap,
                  hipStream_t s)
{
    Ad2AdjArgs a{};
    a.g = m->L.g2;
    a.nshots = ns;
    a.shots_per_model = ns / m->d.nmodels;
    a.l1 = m->adj[(k + 1) & 1];
    a.l2 = m->adj[k & 1];
    a.l0 = m->adj[k & 1];
    a.yx = m->adj[2 + (k & 1)];
    a.yxn = m->adj[2 + ((k + 1) & 1)];
    a.yz = m->adj[4 + (k & 1)];
    a.yzn = m->adj[4 + ((k + 1) & 1)];
    a.zx = m->adj[6 + (k & 1)];
    a.zxn = m->adj[6 + ((k + 1) & 1)];
    a.zz = m->adj[8 + (k & 1)];
    a.zzn = m->adj[8 + ((k + 1) & 1)];
    a.chat = m->chat;
    a.t = ad2_tabs(m);
    a.nt = m->d.nt;
    a.k = k;
    a.rec_off = m->rec_off;
    a.rec_ent = static_cast<const int *>(m->rec_ent);
    a.dJdd = dJdd;
    a.nrec = m->geom_nrec;
    a.snx = snap;
    a.snz = snap ? snap + m->L.field : nullptr;
    a.gn = m->grad;
    launch_ad2_adj(a, s);
    if (gwav && k < m->d.nt)
        launch_ac2_src_gather(ns, m->geom_nsrc, m->L.plane, m->node_f, m->adj[(k + 1) & 1], gwav, m->d.nt, k,
                              src_scale(m), s);
}

// 2-D acoustic: u^t is slot u4[t % 4] and s^t is slot s4[t % 4], so one
// launch can write u^{k+1} and u^{k+2} while another still reads u^k and
// u^{k-1} (the one- and two-step launches of a double step never touch a
// slot another one reads).  The layer auxiliaries alternate over two pairs
// of fields: phi~^t (forward) and c^t (adjoint) in fields 2, 3 for even t
// and 6, 7 for odd t, so a step reads one pair and writes the other.
inline float *ac2_aux(float *const *f, int t, int j)
{
    return f[((t & 1) ? 6 : 2) + j];
}

// The tile lists of a step: the one-step tiles within 4 cells of the layer
// (pass A folded in), the other one-step tiles, the blocked tiles.
enum TileSet { TS_LAYER, TS_OTHER, TS_BLOCKED };
inline const int *tile_set(const sg_model *m, TileSet t, int &n)
{
    n = t == TS_LAYER ? m->n_layer_near : t == TS_OTHER ? m->n_near - m->n_layer_near : m->n_blk;
    return t == TS_LAYER ? m->tiles_near : t == TS_OTHER ? m->tiles_near + m->n_layer_near : m->tiles_blk;
}

// One forward step k on a tile set.
Ac2FwdArgs ac2_args(const sg_model *m, int ns, const float *wav, int k, TileSet ts, float *seis, float *snap)
{
    Ac2FwdArgs a{};
    a.g = m->L.g2;
    a.nshots = ns;
    a.tiles = tile_set(m, ts, a.ntl);
    a.u = m->u4[k & 3];
    a.um = m->u4[(k + 3) & 3];
    a.un = m->u4[(k + 1) & 3];
    a.chat = m->chat;
    a.shots_per_model = ns / m->d.nmodels;
    a.phx0 = ac2_aux(m->fwd, k - 1, 0);
    a.phz0 = ac2_aux(m->fwd, k - 1, 1);
    a.phx = ac2_aux(m->fwd, k, 0);
    a.phz = ac2_aux(m->fwd, k, 1);
    a.hx = m->h[0]; a.hz = m->h[2]; a.px = m->p[0]; a.pz = m->p[2]; a.ihx = m->ih[0]; a.ihz = m->ih[2];
    a.src_f = m->src_f;
    a.wav = wav;
    a.nt = m->d.nt;
    a.k = k;
    a.src_scale = src_scale(m);
    a.rec_off = m->rec_off;
    a.rec_ent = static_cast<const int *>(m->rec_ent);
    a.nrec = m->geom_nrec;
    a.seis = seis;
    a.snap = snap;
    a.nsrc = m->geom_nsrc;
    a.src_off = m->src_off;
    a.src_ent = m->src_ent;
    return a;
}

void ac2_tiles(const sg_model *m, int ns, const float *wav, int k, TileSet ts, float *seis, float *snap,
               hipStream_t s)
{
    launch_ac2_fwd(ac2_args(m, ns, wav, k, ts, seis, snap), ts == TS_LAYER, s);
}

// Forward step k, or steps k and k+1 when `two`: the one-step list step by
// step, blocked tiles both steps in one launch (between the two one-step
// launches, whose second step reads the blocked tiles' u^{k+1} in its halo).
void ac2_forward(const sg_model *m, int ns, const float *wav, int k, bool two, float *seis, float *snap0,
                 float *snap1, hipStream_t s)
{
    if (!two) {
        for (TileSet ts : {TS_LAYER, TS_OTHER, TS_BLOCKED}) ac2_tiles(m, ns, wav, k, ts, seis, snap0, s);
        return;
    }
    Ac2Fwd2Args b{};
    b.g = m->L.g2;
    b.nshots = ns;
    b.tiles = m->tiles_blk;
    b.ntl = m->n_blk;
    b.u0 = m->u4[k & 3];
    b.um = m->u4[(k + 3) & 3];
    b.u1 = m->u4[(k + 1) & 3];
    b.u2 = m->u4[(k + 2) & 3];
    b.chat = m->chat;
    b.shots_per_model = ns / m->d.nmodels;
    b.src_f = m->src_f;
    b.wav = wav;
    b.nt = m->d.nt;
    b.k = k;
    b.src_scale = src_scale(m);
    b.snap0 = snap0;
    b.snap1 = snap1;
    int n_other = 0;
    (void)tile_set(m, TS_OTHER, n_other);
    if (m->pair && n_other == 0 && (!seis || m->geom_nrec == 0)) {
        // the near tiles' step k and the blocked tiles' double step in one
        // grid (sweeps that record seismograms keep them apart: paired, the
        // C2 forward ran 2 % slower while the recompute gained 4 %)
        launch_ac2_fwd_pair(ac2_args(m, ns, wav, k, TS_LAYER, seis, snap0), b, s);
    } else {
        ac2_tiles(m, ns, wav, k, TS_LAYER, seis, snap0, s);
        ac2_tiles(m, ns, wav, k, TS_OTHER, seis, snap0, s);
        launch_ac2_fwd2(b, s);
    }
    ac2_tiles(m, ns, wav, k + 1, TS_LAYER, seis, snap1, s);
    ac2_tiles(m, ns, wav, k + 1, TS_OTHER, seis, snap1, s);
}

// One forward step of the 3-D acoustic or 2-D elastic recursion.
// cu selects u^k = fwd[cu], u^{k-1} = fwd[1-cu].
void fwd_step(const sg_model *m, int ns, const float *wav, int cu, int k, float *seis, float *snap,
              hipStream_t s)
{
    if (m->L.elastic) {
        el_fwd_step(m, ns, wav, k, seis, snap, s);
    } else if (m->d.ndim == 2) {
        ac2_forward(m, ns, wav, k, false, seis, snap, nullptr, s);
    } else {
        Ac3PhiArgs p{};
        p.g = m->L.g3;
        p.items = m->items3;
        p.nitems = m->n_items3;
        p.nfree = m->n_items3_free;
        p.u = m->fwd[cu];
        p.psi = m->fwd[5];
        for (int j = 0; j < 3; ++j) p.ph[j] = m->fwd[2 + j];
        p.t = tabs3(m);
        p.inv_dt = (float)(1.0 / m->d.dt);
        launch_ac3_phi(p, ns, s);
        Ac3FwdArgs a{};
        a.g = m->L.g3;
        a.nshots = ns;
        a.u = m->fwd[cu];
        a.um = m->fwd[1 - cu];
        a.chat = m->chat;
        a.shots_per_model = ns / m->d.nmodels;
        for (int j = 0; j < 3; ++j) a.ph[j] = m->fwd[2 + j];
        a.psi = m->fwd[5];
        a.t = tabs3(m);
        a.dt = (float)m->d.dt;
        a.inv_dt = (float)(1.0 / m->d.dt);
        a.src_f = m->src_f;
        a.wav = wav;
        a.nt = m->d.nt;
        a.k = k;
        a.src_scale = src_scale(m);
        a.rec_off = m->rec_off;
        a.rec_ent = static_cast<const int2 *>(m->rec_ent);
        a.nrec = m->geom_nrec;
        a.seis = seis;
        a.snap = snap;
        a.tiles = m->tiles3;
        a.nnear = m->n_near3;
        launch_ac3_fwd(a, s);
    }
}

// One adjoint step k (s^{k+1} from s^{k+2}, s^{k+3}) on a tile set.
void ac2_adj_tiles(const sg_model *m, int ns, int k, TileSet ts, const float *dJdd, float *gwav,
                   const float *snap, hipStream_t s)
{
    Ac2AdjArgs b{};
    b.g = m->L.g2;
    b.nshots = ns;
    b.tiles = tile_set(m, ts, b.ntl);
    b.s2 = m->s4[(k + 2) & 3];
    b.s3 = m->s4[(k + 3) & 3];
    b.s1 = m->s4[(k + 1) & 3];
    b.chat = m->chat;
    b.shots_per_model = ns / m->d.nmodels;
    b.cx0 = ac2_aux(m->adj, k + 2, 0);
    b.cz0 = ac2_aux(m->adj, k + 2, 1);
    b.cx = ac2_aux(m->adj, k + 1, 0);
    b.cz = ac2_aux(m->adj, k + 1, 1);
    b.hx = m->h[0]; b.hz = m->h[2]; b.px = m->p[0]; b.pz = m->p[2]; b.ihx = m->ih[0]; b.ihz = m->ih[2];
    b.src_f = m->src_f;
    b.gwav = gwav;
    b.nt = m->d.nt;
    b.k = k;
    b.src_scale = src_scale(m);
    b.rec_off = m->rec_off;
    b.rec_ent = static_cast<const int *>(m->rec_ent);
    b.dJdd = dJdd;
    b.nrec = m->geom_nrec;
    b.snap = snap;
    b.grad = m->grad;
    launch_ac2_adj(b, ts == TS_LAYER, s);
}

// Adjoint step k, or steps k and k-1 when `two` (snap1 = w~^k, snap0 = w~^{k-1}).
void ac2_adjoint(const sg_model *m, int ns, int k, bool two, const float *dJdd, float *gwav, const float *snap1,
                 const float *snap0, hipStream_t s)
{
    const bool nodes = gwav && m->geom_nsrc > 1;
    auto gather = [&](int kk) {
        launch_ac2_src_gather(ns, m->geom_nsrc, m->L.plane, m->node_f, m->s4[(kk + 1) & 3], gwav, m->d.nt, kk,
                              src_scale(m), s);
    };
    if (!two) {
        for (TileSet ts : {TS_LAYER, TS_OTHER, TS_BLOCKED}) ac2_adj_tiles(m, ns, k, ts, dJdd, gwav, snap1, s);
        if (nodes) gather(k);
        return;
    }
    ac2_adj_tiles(m, ns, k, TS_LAYER, dJdd, gwav, snap1, s);
    ac2_adj_tiles(m, ns, k, TS_OTHER, dJdd, gwav, snap1, s);
    if (nodes) gather(k);
    Ac2Adj2Args b{};
    b.g = m->L.g2;
    b.nshots = ns;
    b.tiles = m->tiles_blk;
    b.ntl = m->n_blk;
    b.s2 = m->s4[(k + 2) & 3];
    b.s3 = m->s4[(k + 3) & 3];
    b.o1 = m->s4[(k + 1) & 3];
    b.o0 = m->s4[k & 3];
    b.chat = m->chat;
    b.shots_per_model = ns / m->d.nmodels;
    b.src_f = m->src_f;
    b.gwav = gwav;
    b.nt = m->d.nt;
    b.k = k;
    b.src_scale = src_scale(m);
    b.snap1 = snap1;
    b.snap0 = snap0;
    b.grad = m->grad;
    launch_ac2_adj2(b, s);
    ac2_adj_tiles(m, ns, k - 1, TS_LAYER, dJdd, gwav, snap0, s);
    ac2_adj_tiles(m, ns, k - 1, TS_OTHER, dJdd, gwav, snap0, s);
    if (nodes) gather(k - 1);
}

// One adjoint step k of the 3-D acoustic or 2-D elastic recursion:
// s^{k+2} = adj[ca], s^{k+3} = adj[1-ca] (in) / s^{k+1} (out).
void adj_step(const sg_model *m, int ns, int ca, int k, const float *dJdd, float *gwav,
              const float *snap, hipStream_t s)
{
    const int spm = ns / m->d.nmodels;
    if (m->L.elastic) {
        el_adj_step(m, ns, k, dJdd, gwav, snap, s);
    } else if (m->d.ndim == 2) {
        ac2_adjoint(m, ns, k, false, dJdd, gwav, snap, nullptr, s);
    } else {
        Ac3PhiAdjArgs pa{};
        pa.g = m->L.g3;
        pa.items = m->items3a;
        pa.nitems = m->n_items3a;
        pa.s2 = m->adj[ca];
        pa.chat = m->chat;
        pa.shots_per_model = spm;
        for (int j = 0; j < 3; ++j) pa.b[j] = m->adj[2 + j];
        pa.t = tabs3(m);
        launch_ac3_phi_adj(pa, ns, s);
        Ac3AdjArgs b{};
        b.g = m->L.g3;
        b.nshots = ns;
        b.s2 = m->adj[ca];
        b.s3 = m->adj[1 - ca];
        b.chat = m->chat;
        b.shots_per_model = spm;
        for (int j = 0; j < 3; ++j) b.b[j] = m->adj[2 + j];
        b.e = m->adj[5];
        b.t = tabs3(m);
        b.dt = (float)m->d.dt;
        b.inv_dt = (float)(1.0 / m->d.dt);
        b.src_f = m->src_f;
        b.gwav = gwav;
        b.nt = m->d.nt;
        b.k = k;
        b.src_scale = src_scale(m);
        b.rec_off = m->rec_off;
        b.rec_ent = static_cast<const int2 *>(m->rec_ent);
        b.dJdd = dJdd;
        b.nrec = m->geom_nrec;
        b.snap = snap;
        b.grad = m->grad;
        b.tiles = m->tiles3;
        b.nnear = m->n_near3;
        launch_ac3_adj(b, s);
    }
}

// FNV-1a over the arguments a segment's launches hold
struct KeyHash {
    uint64_t h = 1469598103934665603ull;
    template <class T> KeyHash &add(T v)
    {
        uint64_t x = 0;
        static_assert(sizeof(T) <= sizeof(x), "scalar key parts");
        std::memcpy(&x, &v, sizeof(T));
        for (int i = 0; i < 8; ++i) { h ^= (x >> (8 * i)) & 0xff; h *= 1099511628211ull; }
        return *this;
    }
};

// Issues one segment's work on s, or in graph mode launches the segment's
// cached executable graph on s, capturing it first (on the model's capture
// stream, so that the caller's stream may be the null stream) when there is
// none or it was made for other arguments.
template <class F>
int run_segment(sg_model *m, std::vector<sg_model::SegGraph> &cache, int seg, uint64_t key, hipStream_t s,
                F &&issue)
{
    if (!m->graphs) return issue(s);
    if ((int)cache.size() <= seg) cache.resize(seg + 1);
    sg_model::SegGraph &slot = cache[seg];
    if (!slot.exec || slot.key != key) {
        if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        slot.exec = nullptr;
        if (!m->cap) HIPCHECK(hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking));
        HIPCHECK(hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
        const int rc = issue(m->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(m->cap, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : fail(SG_EDEVICE, "segment capture failed: %s", hipGetErrorString(e));
        }
        const hipError_t e2 = hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            slot.exec = nullptr;
            return fail(SG_EDEVICE, "segment graph instantiation failed: %s", hipGetErrorString(e2));
        }
        slot.key = key;
    }
    HIPCHECK(hipGraphLaunch(slot.exec, s));
    return SG_OK;
}

} // namespace

extern "C" {

const char *last_error(void) { return g_err.c_str(); }

size_t workspace_bytes(const sg_desc *d, int32_t max_shots, int32_t max_rec, int32_t ckpt_every)
{
    if (check_desc(d) != SG_OK) return 0;
    if (max_shots < 1 || max_rec < 0 || ckpt_every < 0) {
        fail(SG_EINVAL, "max_shots >= 1, max_rec >= 0 and ckpt_every >= 0 required");
        return 0;
    }
    if ((long long)max_rec >= (1LL << REC_ID_BITS)) {     // as init_model
        fail(SG_EINVAL, "at most %d receivers per shot", (1 << REC_ID_BITS) - 1);
        return 0;
    }
    if (check_shots(d, max_shots) != SG_OK) return 0;
    return make_layout(d, max_shots, max_rec, ckpt_every).total;
}

size_t snapshot_segment_bytes(const sg_desc *d, int32_t max_shots, int32_t ckpt_every)
{
    g_err.clear();
    if (check_desc(d) != SG_OK) return 0;
    if (max_shots < 1 || ckpt_every < 0) {
        fail(SG_EINVAL, "max_shots >= 1 and ckpt_every >= 0 required");
        return 0;
    }
    const Layout L = make_layout(d, max_shots, 0, ckpt_every);
    return sizeof(float) * (size_t)L.K * L.nsnap * L.field;
}

// Stability of the velocities (read back from the device; one
// synchronisation of s): positive and finite, 0 < vs < vp and rho > 0 for
// elastic models, the leapfrog limit of the scheme with a 5 % margin, and
// the damping limit of the acoustic layer.
int check_velocities(const sg_desc *d, const Layout &L, const float *vp, const float *vs, const float *rho,
                     hipStream_t s)
{
    const bool elastic = d->physics == SG_ELASTIC;
    // stability: velocity range from the device copy
    const size_t nphys = (size_t)d->nmodels * d->nx * (d->ndim == 3 ? d->ny : 1) * d->nz;
    std::vector<float> hv(nphys);
    HIPCHECK(hipMemcpyAsync(hv.data(), vp, sizeof(float) * nphys, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    float vmax = hv[0];
    for (float v : hv) {
        if (!(v > 0) || !std::isfinite(v)) return fail(SG_EINVAL, "velocity must be positive and finite");
        vmax = std::max(vmax, v);
    }
    if (elastic) {
        std::vector<float> hs(nphys), hr(nphys);
        HIPCHECK(hipMemcpyAsync(hs.data(), vs, sizeof(float) * nphys, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipMemcpyAsync(hr.data(), rho, sizeof(float) * nphys, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        for (size_t i = 0; i < nphys; ++i)
            if (!(hs[i] > 0) || !(hs[i] < hv[i]) || !(hr[i] > 0) || !std::isfinite(hr[i]))
                return fail(SG_EINVAL, "elastic model needs 0 < vs < vp and rho > 0");
    }
    if (elastic || L.ad2) {
        // 4th-order staggered leapfrog: v dt/dx <= 1/(sqrt(ndim) (9/8 + 1/24))
        // (divergence form: the half-node coefficient never exceeds vmax^2)
        const double limit = 1.0 / (std::sqrt((double)d->ndim) * (9.0 / 8.0 + 1.0 / 24.0));
        const double cfl = vmax * d->dt / d->dx;
        if (cfl > 0.95 * limit) return fail(SG_EUNSTABLE, "CFL number %.4f above 0.95 x %.4f", cfl, limit);
    } else {
        const double limit = 2.0 / std::sqrt(L8_SYMBOL_MAX * d->ndim);
        const double cfl = vmax * d->dt / d->dx;
        if (cfl > 0.95 * limit) return fail(SG_EUNSTABLE, "CFL number %.4f above 0.95 x %.4f", cfl, limit);
    }
    const double zmax = d->npml > 0 ? 3.0 * d->pml_vmax * std::log(1.0 / d->pml_R) / (2.0 * d->npml * d->dx) : 0.0;
    if (!elastic && !L.ad2 && zmax * d->dt > 0.3) return fail(SG_EUNSTABLE, "zeta_max*dt = %.3f above 0.3", zmax * d->dt);
    return SG_OK;
}

int init_model(const sg_desc *d, const float *vp, const float *vs, const float *rho,
               int32_t max_shots, int32_t max_rec, int32_t ckpt_every, void *ws, size_t ws_bytes,
               sg_stream_t stream, sg_model **out)
{
    g_err.clear();
    if (!out) return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_desc(d);
    if (rc) return rc;
    const bool elastic = d->physics == SG_ELASTIC;
    if (!elastic && (vs || rho)) return fail(SG_EINVAL, "vs and rho must be NULL for acoustic models");
    if (elastic && (!vs || !rho)) return fail(SG_EINVAL, "elastic models need vs and rho");
    if (!vp || !ws) return fail(SG_EINVAL, "vp and ws must be device pointers");
    if (max_shots < 1 || max_rec < 0 || ckpt_every < 0)
        return fail(SG_EINVAL, "max_shots >= 1, max_rec >= 0 and ckpt_every >= 0 required");
    if (max_shots % d->nmodels) return fail(SG_EINVAL, "max_shots must be a multiple of nmodels");
    if ((long long)max_rec >= (1LL << REC_ID_BITS)) return fail(SG_EINVAL, "at most %d receivers per shot", (1 << REC_ID_BITS) - 1);
    if (const int e = check_shots(d, max_shots)) return e;
    if (d->ndim == 3 && d->nz + 2 * d->npml >= (1 << 12)) return fail(SG_EINVAL, "3-D grids are limited to 4095 padded planes in z");
    const Layout L = make_layout(d, max_shots, max_rec, ckpt_every);
    if (ws_bytes < L.total) return fail(SG_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if ((uintptr_t)ws % ALIGN) return fail(SG_EINVAL, "workspace must be %zu-byte aligned", ALIGN);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    if (const int e = check_velocities(d, L, vp, vs, rho, s)) return e;
    const double zmax = d->npml > 0 ? 3.0 * d->pml_vmax * std::log(1.0 / d->pml_R) / (2.0 * d->npml * d->dx) : 0.0;

    sg_model *m = new sg_model();
    m->d = *d;
    if (d->ndim == 2) m->d.ny = 1;
    m->L = L;
    m->max_shots = max_shots;
    m->max_rec = max_rec;
    m->ws = static_cast<char *>(ws);
    m->chat = reinterpret_cast<float *>(m->ws + L.off_chat);
    m->cpad = reinterpret_cast<float *>(m->ws + L.off_cpad);
    for (int i = 0; i < L.nf + L.nxs; ++i) {
        m->fwd[i] = reinterpret_cast<float *>(m->ws + L.off_fwd) + i * L.field;
        m->adj[i] = reinterpret_cast<float *>(m->ws + L.off_adj) + i * L.field;
    }
    if (!L.elastic && d->ndim == 2) {
        if (!L.ad2) {
            float *fb = reinterpret_cast<float *>(m->ws + L.off_fwd), *ab = reinterpret_cast<float *>(m->ws + L.off_adj);
            const int slot[4] = {0, 1, 4, 5};   // fields 2, 3 and 6, 7 hold the layer auxiliaries
            for (int i = 0; i < 4; ++i) {
                m->u4[i] = fb + slot[i] * L.field;
                m->s4[i] = ab + slot[i] * L.field;
            }
        }
        m->tiles_near = reinterpret_cast<int *>(m->ws + L.off_tiles);
        m->tiles_blk = m->tiles_near + L.ntiles;
        m->tiles_layer = m->tiles_near + L.ntiles;   // the second half of the tile lists
        const Grid2 &g = L.g2;
        for (int t = 0; t < L.ntiles && d->npml > 0; ++t) {
            const int x0 = (t % g.ntx) * TX, z0 = (t / g.ntx) * TZ;
            if (x0 < g.P || x0 + TX > g.P + g.nx || z0 < g.P || z0 + TZ > g.P + g.nz) m->h_layer.push_back(t);
        }
        m->n_layer = (int)m->h_layer.size();
    }
    {
        const size_t per = sizeof(float) * (size_t)L.K * L.nsnap * L.field;
        const size_t extra = ws_bytes - L.total;
        m->n_store = (int)std::min<size_t>(extra / per, (size_t)L.nseg);
        m->store = m->n_store > 0 ? reinterpret_cast<float *>(m->ws + L.total) : nullptr;
    }
    m->src_off = reinterpret_cast<int *>(m->ws + L.off_soff);
    m->src_ent = reinterpret_cast<int *>(m->ws + L.off_sent);
    m->node_f = reinterpret_cast<long long *>(m->ws + L.off_nodef);
    m->ckpt = reinterpret_cast<float *>(m->ws + L.off_ckpt);
    m->snap = reinterpret_cast<float *>(m->ws + L.off_snap);
    m->grad = reinterpret_cast<float *>(m->ws + L.off_grad);
    m->src_f = reinterpret_cast<long long *>(m->ws + L.off_src);
    m->rec_off = reinterpret_cast<int *>(m->ws + L.off_recoff);
    m->rec_ent = m->ws + L.off_recent;
    m->partials = reinterpret_cast<double *>(m->ws + L.off_part);
    m->numeric_flag = reinterpret_cast<int *>(m->ws + L.off_flag);
    for (int i = 0; i < 8; ++i) {
        m->model[i] = reinterpret_cast<float *>(m->ws + L.off_chat) + (size_t)i * d->nmodels * L.plane;
        m->tmp[i] = L.elastic ? reinterpret_cast<float *>(m->ws + L.off_tmp) + i * L.field : nullptr;
    }
    m->acc = reinterpret_cast<float *>(m->ws + L.off_acc);
    m->uoff = reinterpret_cast<int *>(m->ws + L.off_uoff);
    m->uid = reinterpret_cast<int *>(m->ws + L.off_uid);
    m->mt = reinterpret_cast<float *>(m->ws + L.off_mt);

    // damping tables per axis, FP64 rounded once: h = zeta dt / 2,
    // p = (1-h)/(1+h), 1/(1+h); TABPAD neutral entries (h = 0) on each side
    const int phys[3] = {d->nx, d->ndim == 3 ? d->ny : 1, d->nz};
    const bool cpml = elastic || L.ad2;   // the staggered-grid forms
    size_t tot = 0;
    if (cpml) tot = 4 * (L.n[0] + L.n[2] + 4 * TABPAD);
    else for (int a = 0; a < 3; ++a) tot += 3 * (L.n[a] + 2 * TABPAD);
    m->h_tab.assign(tot, 0.f);
    float *dev_tab = reinterpret_cast<float *>(m->ws + L.off_tab);
    size_t o = 0;
    for (int a = 0; a < (cpml ? 0 : 3); ++a) {
        const int N = L.n[a] + 2 * TABPAD;
        float *h = m->h_tab.data() + o, *p = h + N, *ih = p + N;
        for (int i = 0; i < N; ++i) {
            const int c = i - TABPAD;   // padded-grid index
            int depth = 0;
            if (c >= 0 && c < L.n[a] && !(d->ndim == 2 && a == 1))
                depth = c < d->npml ? d->npml - c : (c >= d->npml + phys[a] ? c - (d->npml + phys[a] - 1) : 0);
            const double r = d->npml > 0 ? (double)depth / d->npml : 0.0;
            const double hv = 0.5 * d->dt * zmax * r * r;
            h[i] = (float)hv;
            p[i] = (float)((1.0 - hv) / (1.0 + hv));
            ih[i] = (float)(1.0 / (1.0 + hv));
        }
        m->h[a] = dev_tab + o + TABPAD;
        m->p[a] = dev_tab + o + N + TABPAD;
        m->ih[a] = dev_tab + o + 2 * N + TABPAD;
        o += 3 * N;
    }
    if (cpml) {
        // CPML (kappa = 1): b = exp(-(d + al) dt), a = d (b - 1)/(d + al),
        // d = d0 (x/L)^2, al = pi f0 (1 - x/L), d0 = 3 vmax ln(1/R)/(2L), at
        // integer and half positions; x = distance into the layer
        const double Lw = d->npml * d->dx;
        const double d0 = d->npml > 0 ? 3.0 * d->pml_vmax * std::log(1.0 / d->pml_R) / (2.0 * Lw) : 0.0;
        o = 0;
        for (int ax = 0; ax < 2; ++ax) {
            const int a = ax == 0 ? 0 : 2, N = L.n[a] + 2 * TABPAD, n = phys[a];
            for (int h = 0; h < 2; ++h) {
                float *ta = m->h_tab.data() + o, *tb = ta + N;
                for (int i = 0; i < N; ++i) {
                    const double x = (i - TABPAD) + 0.5 * h;
                    double dist = 0.0;
                    if (i - TABPAD >= 0 && i - TABPAD < L.n[a]) {
                        if (x < d->npml) dist = d->npml - x;
                        else if (x > d->npml + n - 1) dist = x - (d->npml + n - 1);
                    }
                    double av = 0.0, bv = 1.0;
                    if (d->npml > 0 && dist > 0.0) {
                        const double r = std::min(dist / d->npml, 1.0);
                        const double dd = d0 * r * r, al = M_PI * d->f0_pml * (1.0 - r);
                        bv = std::exp(-(dd + al) * d->dt);
                        av = dd * (bv - 1.0) / (dd + al);
                    }
                    ta[i] = (float)av;
                    tb[i] = (float)bv;
                }
                m->cpml[ax][2 * h] = dev_tab + o + TABPAD;
                m->cpml[ax][2 * h + 1] = dev_tab + o + N + TABPAD;
                o += 2 * N;
            }
        }
    }
    if (d->ndim == 3) {
        const Grid3 &g = L.g3;
        m->tiles3 = reinterpret_cast<int *>(m->ws + L.off_tiles);
        std::vector<int> rest;
        for (int t = 0; t < L.ntiles; ++t) {
            const int x0 = (t % g.ntx) * TX3, y0 = (t / g.ntx) * TY3;
            const bool near = g.P > 0 && (x0 - 4 < g.P || x0 + TX3 + 4 > g.P + g.nx ||
                                          y0 - 4 < g.P || y0 + TY3 + 4 > g.P + g.ny);
            (near ? m->h_tiles3 : rest).push_back(t);
        }
        m->n_near3 = (int)m->h_tiles3.size();
        m->h_tiles3.insert(m->h_tiles3.end(), rest.begin(), rest.end());
    }
    if (d->ndim == 3 && d->npml > 0) {
        m->items3 = reinterpret_cast<int4 *>(m->ws + L.off_items);
        m->items3a = m->items3 + items3_cap(L.ntiles, L.g3.NZ);
        if (build_items3(m, TZCI_DEF)) {
            delete m;
            return fail(SG_EINVAL, "layer work list overflows its buffer");
        }
    }
    // the numeric flag starts clear (a fill kernel: the int 0 is the float 0.f)
    launch_fill(reinterpret_cast<float *>(m->numeric_flag), 1, 0.f, s);
    hipError_t e = hipMemcpyAsync(dev_tab, m->h_tab.data(), sizeof(float) * tot, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && m->n_items3 > 0)
        e = hipMemcpyAsync(m->items3, m->h_items3.data(), sizeof(int4) * m->n_items3, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && m->n_items3a > 0)
        e = hipMemcpyAsync(m->items3a, m->h_items3a.data(), sizeof(int4) * m->n_items3a, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && m->n_layer > 0)
        e = hipMemcpyAsync(m->tiles_layer, m->h_layer.data(), sizeof(int) * m->n_layer, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !m->h_tiles3.empty())
        e = hipMemcpyAsync(m->tiles3, m->h_tiles3.data(), sizeof(int) * m->h_tiles3.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        delete m;
        return fail(SG_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    if (elastic) launch_el2_prep(L.g2, d->nmodels, vp, vs, rho, m->model, m->model + 5, s);
    else if (L.ad2) launch_ad2_prep(L.g2, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    else if (d->ndim == 2) launch_ac2_prep(L.g2, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    else launch_ac3_prep(L.g3, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete m;
        return fail(SG_EDEVICE, "model preparation failed: %s", hipGetErrorString(e));
    }
    *out = m;
    return SG_OK;
}

int update_model(sg_model *m, const float *vp, const float *vs, const float *rho, sg_stream_t stream)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    const sg_desc *d = &m->d;
    const Layout &L = m->L;
    const bool elastic = L.elastic;
    if (!elastic && (vs || rho)) return fail(SG_EINVAL, "vs and rho must be NULL for acoustic models");
    if (elastic && (!vs || !rho)) return fail(SG_EINVAL, "elastic models need vs and rho");
    if (!vp) return fail(SG_EINVAL, "vp must be a device pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (const int e = check_velocities(d, L, vp, vs, rho, s)) return e;
    if (elastic) launch_el2_prep(L.g2, d->nmodels, vp, vs, rho, m->model, m->model + 5, s);
    else if (L.ad2) launch_ad2_prep(L.g2, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    else if (d->ndim == 2) launch_ac2_prep(L.g2, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    else launch_ac3_prep(L.g3, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SG_EDEVICE, "model preparation failed: %s", hipGetErrorString(e));
    // the checkpoints and stored snapshots belong to the old parameters
    m->have_ckpt = false;
    m->have_store = false;
    return SG_OK;
}

int forward_shots(sg_model *m, const sg_shots *sh, float *seis, int32_t save_ckpt, sg_stream_t stream)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    int rc = check_shots(m, sh);
    if (rc) return rc;
    if (!seis && sh->nrec > 0) return fail(SG_EINVAL, "seis is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = upload_geometry(m, sh, s);
    if (rc) return rc;
    const Layout &L = m->L;
    const int ns = sh->nshots, nt = m->d.nt, K = L.K, nf = L.nf;
    const long long fs = (long long)ns * L.plane;  // floats of one field over the batch
    const bool ad2 = L.ad2;
    const bool ac2 = !L.elastic && !ad2 && m->d.ndim == 2;
    for (int i = 0; i < (ad2 || ac2 ? nf + L.nxs : nf); ++i) launch_fill(m->fwd[i], fs, 0.f, s);
    float *sp = sh->nrec > 0 ? seis : nullptr;
    // segments >= seg0 keep their adjoint snapshots (checkpointed forwards only)
    const int seg0 = save_ckpt ? L.nseg - m->n_store : L.nseg;
    auto stored = [&](int k) -> float * {
        const int seg = k / K;
        if (seg < seg0) return nullptr;
        return m->store + ((size_t)(seg - seg0) * K + (k - seg * K)) * L.nsnap * L.field;
    };
    // one checkpoint segment: the checkpoint of its first state, then its steps
    auto issue = [&](int seg, hipStream_t st) -> int {
        const int k0 = seg * K, k1 = std::min(k0 + K, nt);
        int cu = k0 & 1;                  // 3-D / elastic: u^k in fwd[cu]
        if (save_ckpt) {
            // state at the start of step k0: u^k, u^{k-1}, then the layer fields
            // (acoustic: u^k, u^{k-1} first; elastic: the fields in order)
            float *ck = m->ckpt + (size_t)seg * nf * L.field;
            for (int i = 0; i < nf; ++i) {
                const float *src = ad2 ? ad2_state(m, k0, i)
                                 : ac2 ? (i < 2 ? m->u4[(k0 + 4 - i) & 3] : ac2_aux(m->fwd, k0 - 1, i - 2))
                                 : L.elastic || i >= 2 ? m->fwd[i]
                                       : (i == 0 ? m->fwd[cu] : m->fwd[1 - cu]);
                HIPCHECK(hipMemcpyAsync(ck + i * L.field, src, sizeof(float) * fs, hipMemcpyDeviceToDevice, st));
            }
        }
        for (int k = k0; k < k1;) {
            if (ac2) {
                // two steps per launch on the blocked tiles, within one checkpoint segment
                const bool two = m->steps_per_launch == 2 && m->n_blk > 0 && k + 1 < k1;
                ac2_forward(m, ns, sh->wavelet, k, two, sp, stored(k), two ? stored(k + 1) : nullptr, st);
                k += two ? 2 : 1;
            } else if (ad2) {
                ad2_fwd_step(m, ns, sh->wavelet, k, sp, stored(k), st);
                ++k;
            } else {
                fwd_step(m, ns, sh->wavelet, cu, k, sp, stored(k), st);
                cu = 1 - cu;
                ++k;
            }
        }
        return SG_OK;
    };
    const uint64_t key = KeyHash().add(m->epoch).add(sp).add(sh->wavelet).add(save_ckpt).add(seg0).add(ns)
                             .add(sh->nrec).h;
    for (int seg = 0; seg < L.nseg; ++seg) {
        const int steps = std::min(K, nt - seg * K);
        const int span = m->graphs ? -1 : span_begin(m, 0, steps, s);
        rc = run_segment(m, m->gfwd[save_ckpt != 0], seg, key, s, [&](hipStream_t st) { return issue(seg, st); });
        if (rc) return rc;
        span_end(m, span, s);
    }
    HIPCHECK(hipGetLastError());
    m->have_ckpt = save_ckpt != 0;
    m->have_store = save_ckpt != 0 && m->n_store > 0;
    return SG_OK;
}

int misfit(sg_model *m, const float *pred, const float *obs, int64_t n, double *J_dev,
           float *resid, sg_stream_t stream)
{
    g_err.clear();
    if (!J_dev || n < 0 || (n > 0 && (!pred || !obs))) return fail(SG_EINVAL, "bad misfit arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    launch_misfit(pred, obs, n, resid, m ? m->partials : nullptr, m ? NOALLOC_PARTS : 1, J_dev,
                  m ? m->numeric_flag : nullptr, s);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int adjoint_gradient(sg_model *m, const sg_shots *sh, const float *dJ_dd, float *g_vp,
                     float *g_vs, float *g_rho, float *g_wavelet, sg_stream_t stream)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    int rc = check_shots(m, sh);
    if (rc) return rc;
    if (!m->L.elastic && (g_vs || g_rho)) return fail(SG_EINVAL, "g_vs and g_rho must be NULL for acoustic models");
    if (m->L.elastic && (!g_vs || !g_rho)) return fail(SG_EINVAL, "elastic gradients need g_vs and g_rho");
    if (!g_vp || (!dJ_dd && sh->nrec > 0)) return fail(SG_EINVAL, "g_vp / dJ_dd is NULL");
    if (!sh->src || (sh->nrec > 0 && !sh->rec)) return fail(SG_EINVAL, "source/receiver arrays are NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!m->have_ckpt || !same_geometry(m, sh))
        return fail(SG_ESTATE, "no checkpointed forward of these shots precedes the adjoint");
    const Layout &L = m->L;
    const int ns = sh->nshots, nt = m->d.nt, K = L.K, nf = L.nf;
    const long long fs = (long long)ns * L.plane;
    const bool ad2 = L.ad2;
    const bool ac2 = !L.elastic && !ad2 && m->d.ndim == 2;
    for (int i = 0; i < (ad2 || ac2 ? nf + L.nxs : nf); ++i) launch_fill(m->adj[i], fs, 0.f, s);
    for (int q = 0; q < L.ngrad; ++q) launch_fill(m->grad + q * L.field, fs, 0.f, s);
    if (L.elastic)
        for (int i = 0; i < 8; ++i) launch_fill(m->tmp[i], fs, 0.f, s);
    if (ad2) ad2_adj_step(m, ns, nt, dJ_dd, nullptr, nullptr, s);   // lambda^nt
    const int seg0 = m->have_store ? L.nseg - m->n_store : L.nseg;
    const bool blk = ac2 && m->steps_per_launch == 2 && m->n_blk > 0;
    // one checkpoint segment: restore and recompute its snapshots (unless the
    // forward kept them), then its adjoint steps; with `spans` (eager runs)
    // the recompute and adjoint loops are timed apart
    auto issue = [&](int seg, hipStream_t st, bool spans) -> int {
        const int k0 = seg * K, k1 = std::min(k0 + K, nt);
        const bool kept = seg >= seg0;   // snapshots written by the forward
        float *sbase = kept ? m->store + (size_t)(seg - seg0) * K * L.nsnap * L.field : m->snap;
        auto snap = [&](int k) { return sbase + (size_t)(k - k0) * L.nsnap * L.field; };
        int span = -1;
        if (!kept) {
            const float *ck = m->ckpt + (size_t)seg * nf * L.field;
            for (int i = 0; i < nf; ++i) {
                float *dst = ad2 ? ad2_state(m, k0, i)
                           : ac2 ? (i < 2 ? m->u4[(k0 + 4 - i) & 3] : ac2_aux(m->fwd, k0 - 1, i - 2))
                                 : m->fwd[i];
                HIPCHECK(hipMemcpyAsync(dst, ck + i * L.field, sizeof(float) * fs, hipMemcpyDeviceToDevice, st));
            }
            int cu = 0;
            if (spans) span = span_begin(m, 1, k1 - k0, st);
            for (int k = k0; k < k1;) {
                if (ac2) {
                    const bool two = blk && k + 1 < k1;
                    ac2_forward(m, ns, sh->wavelet, k, two, nullptr, snap(k), two ? snap(k + 1) : nullptr, st);
                    k += two ? 2 : 1;
                } else if (ad2) {
                    ad2_fwd_step(m, ns, sh->wavelet, k, nullptr, snap(k), st);
                    ++k;
                } else {
                    fwd_step(m, ns, sh->wavelet, cu, k, nullptr, snap(k), st);
                    cu = 1 - cu;
                    ++k;
                }
            }
            span_end(m, span, st);
        }
        int ca = (nt - k1) & 1;          // 3-D / elastic: s^{k+2} in adj[ca]
        span = spans ? span_begin(m, 2, k1 - k0, st) : -1;
        for (int k = k1 - 1; k >= k0;) {
            if (ac2) {
                const bool two = blk && k - 1 >= k0;
                ac2_adjoint(m, ns, k, two, dJ_dd, g_wavelet, snap(k), two ? snap(k - 1) : nullptr, st);
                k -= two ? 2 : 1;
            } else if (ad2) {
                ad2_adj_step(m, ns, k, dJ_dd, g_wavelet, snap(k), st);
                --k;
            } else if (L.elastic) {
                // pass 3 of step k and pass 1 of step k - 1 share a launch within the segment
                el_adj_step(m, ns, k, dJ_dd, g_wavelet, snap(k), st, k == k1 - 1, k > k0 ? snap(k - 1) : nullptr);
                --k;
            } else {
                adj_step(m, ns, ca, k, dJ_dd, g_wavelet, snap(k), st);
                ca = 1 - ca;
                --k;
            }
        }
        span_end(m, span, st);
        return SG_OK;
    };
    const uint64_t key = KeyHash().add(m->epoch).add(dJ_dd).add(g_wavelet).add(sh->wavelet).add(seg0).add(ns)
                             .add(sh->nrec).h;
    for (int seg = L.nseg - 1; seg >= 0; --seg) {
        rc = run_segment(m, m->gadj, seg, key, s, [&](hipStream_t st) { return issue(seg, st, !m->graphs); });
        if (rc) return rc;
    }
    if (L.elastic)
        launch_el2_finalize(L.g2, m->d.nmodels, ns / m->d.nmodels, el_group(m, ns / m->d.nmodels), m->grad,
                            L.field, m->acc, m->model,
                            m->model + 5, g_vp, g_vs, g_rho, s);
    else if (ad2)
        launch_ad2_finalize(L.g2, m->d.nmodels, ns / m->d.nmodels, m->grad, m->acc, m->cpad, m->d.dt, m->d.dx,
                            g_vp, s);
    else if (m->d.ndim == 2)
        launch_ac2_finalize(L.g2, m->d.nmodels, ns / m->d.nmodels, m->grad, m->acc, m->cpad, m->d.dt, m->d.dx, g_vp, s);
    else
        launch_ac3_finalize(L.g3, m->d.nmodels, ns / m->d.nmodels, m->grad, m->acc, m->cpad, m->d.dt, m->d.dx, g_vp, s);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int misfit_noalloc(const float *pred, const float *obs, int64_t n, double *J_dev, float *resid,
                   sg_stream_t stream)
{
    g_err.clear();
    if (!J_dev || n < 0 || (n > 0 && (!pred || !obs))) return fail(SG_EINVAL, "bad misfit arguments");
    if (n > (int64_t(1) << 40)) return fail(SG_EINVAL, "n = %lld above the limit 2^40", (long long)n);
    double *partials = nullptr;
    if (noalloc_scratch(&partials)) return fail(SG_EDEVICE, "no address for the static partial-sum array");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    launch_misfit(pred, obs, n, resid, partials, NOALLOC_PARTS, J_dev, nullptr, s);
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int numeric_status(sg_model *m, sg_stream_t stream)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHECK(hipStreamSynchronize(s));
    int flag = 0;
    HIPCHECK(hipMemcpy(&flag, m->numeric_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (!flag) return SG_OK;
    const int zero = 0;
    HIPCHECK(hipMemcpy(m->numeric_flag, &zero, sizeof(int), hipMemcpyHostToDevice));
    return fail(SG_ENUMERIC, "a misfit on this model was not finite (NaN or Inf in the seismograms)");
}

int set_tuning(sg_model *m, int32_t key, int32_t value, sg_stream_t stream)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    const bool three = !m->L.elastic && m->d.ndim == 3;
    ++m->epoch;                       // segment graphs captured under the old settings are stale
    switch (key) {
    case SG_TUNE_TIME_BLOCKING:
        return set_time_blocking(m, value);
    case SG_TUNE_GRAPHS:
        if (value != 0 && value != 1) return fail(SG_EINVAL, "graphs: 0 or 1");
        m->graphs = value != 0;
        return SG_OK;
    case SG_TUNE_CHUNK_FWD3:
    case SG_TUNE_CHUNK_ADJ3:
    case SG_TUNE_CHUNK_LAYER3: {
        if (!three) return fail(SG_EINVAL, "3-D chunk lengths apply to 3-D acoustic models");
        if (value < TZC_MIN || value > TZC || value % 8)
            return fail(SG_EINVAL, "chunk of %d planes outside [%d, %d] or not a multiple of 8", value, TZC_MIN, TZC);
        Grid3 &g = m->L.g3;
        if (key == SG_TUNE_CHUNK_FWD3) g.zcf = value;
        if (key == SG_TUNE_CHUNK_ADJ3) {
            g.zca = value;
            g.nzc = (g.NZ + value - 1) / value;
        }
        if (key == SG_TUNE_CHUNK_LAYER3 && m->items3 && value != m->zci) {
            if (build_items3(m, value)) return fail(SG_EINVAL, "layer work list overflows its buffer");
            // the list is read by launches already enqueued: wait for them first
            hipStream_t s = reinterpret_cast<hipStream_t>(stream);
            HIPCHECK(hipStreamSynchronize(s));
            HIPCHECK(hipMemcpyAsync(m->items3, m->h_items3.data(), sizeof(int4) * m->n_items3,
                                    hipMemcpyHostToDevice, s));
            HIPCHECK(hipMemcpyAsync(m->items3a, m->h_items3a.data(), sizeof(int4) * m->n_items3a,
                                    hipMemcpyHostToDevice, s));
            HIPCHECK(hipStreamSynchronize(s));
        }
        return SG_OK;
    }
    case SG_TUNE_PAIR:
        if (m->L.elastic || m->L.ad2 || m->d.ndim != 2) return fail(SG_EINVAL, "launch pairing applies to 2-D acoustic models");
        if (value != 0 && value != 1) return fail(SG_EINVAL, "launch pairing: 0 or 1");
        m->pair = value != 0;
        return SG_OK;
    case SG_TUNE_SHOT_GROUP:
        if (!m->L.elastic) return fail(SG_EINVAL, "shot groups apply to elastic models");
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return fail(SG_EINVAL, "shot group %d: 0 (automatic), 1, 2 or 4", value);
        m->el_gs = value;
        return SG_OK;
    case SG_TUNE_BLOCK_X:
        if (!m->L.elastic) return fail(SG_EINVAL, "cell block width applies to elastic models");
        if (value != 32 && value != 64) return fail(SG_EINVAL, "cell block width %d: 32 or 64", value);
        m->el_ebx = value;
        return SG_OK;
    default:
        return fail(SG_EINVAL, "unknown tuning key %d", key);
    }
}

int set_time_blocking(sg_model *m, int32_t steps)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    if (steps != 1 && steps != 2) return fail(SG_EINVAL, "steps per launch must be 1 or 2, got %d", steps);
    m->steps_per_launch = steps;
    ++m->epoch;
    return SG_OK;
}

int set_profiling(sg_model *m, int32_t enable)
{
    g_err.clear();
    if (!m) return fail(SG_EINVAL, "model is NULL");
    m->profiling = enable != 0;
    return SG_OK;
}

int phase_times(sg_model *m, double *ms, int64_t *steps)
{
    g_err.clear();
    if (!m || !ms || !steps) return fail(SG_EINVAL, "bad phase_times arguments");
    for (int i = 0; i < 3; ++i) { ms[i] = 0.0; steps[i] = 0; }
    for (auto &sp : m->spans) {
        HIPCHECK(hipEventSynchronize(sp.b));
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, sp.a, sp.b));
        ms[sp.phase] += t;
        steps[sp.phase] += sp.steps;
        m->pool.push_back(sp.a);
        m->pool.push_back(sp.b);
    }
    m->spans.clear();
    return SG_OK;
}

int free_model(sg_model *m)
{
    delete m;
    return SG_OK;
}

int ricker(double f0, double t0, double dt, int32_t nt, float *out, sg_stream_t stream)
{
    g_err.clear();
    if (!out || nt < 1 || !(dt > 0) || !(f0 > 0)) return fail(SG_EINVAL, "bad ricker arguments");
    launch_ricker(f0, t0, dt, nt, out, reinterpret_cast<hipStream_t>(stream));
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

int dot_f64(const float *x, const float *y, int64_t n, double *out, sg_stream_t stream)
{
    g_err.clear();
    if (!x || !y || !out || n < 0) return fail(SG_EINVAL, "bad dot arguments");
    launch_dot(x, y, n, out, reinterpret_cast<hipStream_t>(stream));
    HIPCHECK(hipGetLastError());
    return SG_OK;
}

} // extern "C"
