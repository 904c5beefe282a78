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

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace sg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
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

#define HIPCHECK(x)                                                                  \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            return fail(SG_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));     \
    } while (0)

constexpr double L8_SYMBOL_MAX = 6.501587301587301; // max |1-D 8th-order symbol| * dx^2
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    Grid2 g;
    int K, nseg;
    size_t off_chat, off_cpad, off_tab, off_fwd, off_adj, off_ckpt, off_snap,
        off_grad, off_src, off_recoff, off_recent, off_part, total;
    int ntiles;
    long long field;   // floats per field over max_shots
};

int check_desc(const sg_desc *d)
{
    if (!d) return fail(SG_EINVAL, "descriptor is NULL");
    if (d->physics != SG_ACOUSTIC) return fail(SG_EUNSUPPORTED, "physics %d is not provided by this build", d->physics);
    if (d->ndim != 2) return fail(SG_EUNSUPPORTED, "ndim %d is not provided by this build", d->ndim);
    if (d->nx < 1 || d->nz < 1 || d->npml < 0 || d->nt < 1 || d->nmodels < 1)
        return fail(SG_EINVAL, "bad grid: nx=%d nz=%d npml=%d nt=%d nmodels=%d", d->nx, d->nz, d->npml, d->nt, d->nmodels);
    if (!(d->dx > 0) || !(d->dt > 0)) return fail(SG_EINVAL, "dx and dt must be positive");
    if (d->npml > 0 && (!(d->pml_R > 0 && d->pml_R < 1) || !(d->pml_vmax > 0)))
        return fail(SG_EINVAL, "absorbing layer needs 0 < pml_R < 1 and pml_vmax > 0");
    if ((long long)(d->nx + 2 * d->npml) * (d->nz + 2 * d->npml) > (1LL << 31))
        return fail(SG_EINVAL, "grid too large");
    return SG_OK;
}

Layout make_layout(const sg_desc *d, int max_shots, int max_rec, int ckpt)
{
    Layout L{};
    Grid2 &g = L.g;
    g.P = d->npml; g.nx = d->nx; g.nz = d->nz;
    g.NX = d->nx + 2 * d->npml; g.NZ = d->nz + 2 * d->npml;
    g.ntx = (g.NX + TX - 1) / TX; g.ntz = (g.NZ + TZ - 1) / TZ;
    g.SX = OX + g.ntx * TX + 32;
    g.SZ = OZ + g.ntz * TZ + 8;
    g.plane = (long long)g.SX * g.SZ;
    L.ntiles = g.ntx * g.ntz;
    L.K = ckpt > 0 ? ckpt : (int)std::ceil(std::sqrt((double)d->nt));
    if (L.K > d->nt) L.K = d->nt;
    L.nseg = (d->nt + L.K - 1) / L.K;
    L.field = (long long)max_shots * g.plane;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    L.off_chat = take(sizeof(float) * d->nmodels * g.plane);
    L.off_cpad = take(sizeof(float) * d->nmodels * g.plane);
    L.off_tab = take(sizeof(float) * 3 * (g.NX + g.NZ));  // h, (1-h)/(1+h), 1/(1+h) per axis
    L.off_fwd = take(sizeof(float) * 4 * L.field);        // u[2], phx, phz
    L.off_adj = take(sizeof(float) * 4 * L.field);        // s[2], cx, cz
    L.off_ckpt = take(sizeof(float) * (size_t)L.nseg * 4 * L.field);
    L.off_snap = take(sizeof(float) * (size_t)L.K * L.field);
    L.off_grad = take(sizeof(float) * L.field);
    L.off_src = take(sizeof(int) * max_shots);
    L.off_recoff = take(sizeof(int) * (size_t)max_shots * (L.ntiles + 1));
    L.off_recent = take(sizeof(int) * std::max<size_t>(1, (size_t)max_shots * max_rec));
    L.off_part = take(sizeof(double) * 4096);
    L.total = o;
    return L;
}

} // namespace

struct sg_model {
    sg_desc d;
    Layout L;
    int max_shots, max_rec;
    char *ws;
    float *chat, *cpad, *hx, *hz, *px, *pz, *ihx, *ihz;
    float *fwd[4], *adj[4];
    float *ckpt, *snap, *grad;
    int *src_cell, *rec_off, *rec_ent;
    double *partials;
    std::vector<float> h_tab;
    std::vector<int> h_src, h_off, h_ent;
    std::vector<int32_t> geom_src, geom_rec;  // geometry as uploaded
    int geom_nshots = -1, geom_nrec = -1;
    bool have_ckpt = false;
    int ckpt_nshots = 0;
    // optional device timing of the step loops: one event pair per segment
    struct Span { int phase; int steps; hipEvent_t a, b; };
    bool profiling = false;
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    ~sg_model()
    {
        for (auto &sp : spans) { pool.push_back(sp.a); pool.push_back(sp.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

int upload_geometry(sg_model *m, const sg_shots *sh, hipStream_t s)
{
    const Grid2 &g = m->L.g;
    const int ns = sh->nshots, nrec = sh->nrec;
    if (!sh->src || (nrec > 0 && !sh->rec)) return fail(SG_EINVAL, "source/receiver arrays are NULL");
    for (int i = 0; i < ns; ++i) {
        const int ix = sh->src[2 * i], iz = sh->src[2 * i + 1];
        if (ix < 0 || ix >= g.nx || iz < 0 || iz >= g.nz)
            return fail(SG_EINVAL, "shot %d: source (%d, %d) outside the %dx%d grid", i, ix, iz, g.nx, g.nz);
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = sh->rec + ((size_t)i * nrec + r) * 2;
            if (q[0] < 0 || q[0] >= g.nx || q[1] < 0 || q[1] >= g.nz)
                return fail(SG_EINVAL, "shot %d receiver %d: (%d, %d) outside the grid", i, r, q[0], q[1]);
        }
    }
    const bool same = m->geom_nshots == ns && m->geom_nrec == nrec &&
                      std::equal(sh->src, sh->src + 2 * ns, m->geom_src.begin()) &&
                      (nrec == 0 || std::equal(sh->rec, sh->rec + (size_t)2 * ns * nrec, m->geom_rec.begin()));
    if (same) return SG_OK;
    // the previous upload may still be reading the host vectors
    HIPCHECK(hipStreamSynchronize(s));
    const int ntiles = m->L.ntiles;
    m->h_src.assign(ns, 0);
    m->h_off.assign((size_t)ns * (ntiles + 1), 0);
    m->h_ent.clear();
    std::vector<std::pair<long long, int>> keyed;
    for (int i = 0; i < ns; ++i) {
        const int ix = sh->src[2 * i] + g.P, iz = sh->src[2 * i + 1] + g.P;
        m->h_src[i] = (iz + OZ) * g.SX + ix + OX;
        keyed.clear();
        for (int r = 0; r < nrec; ++r) {
            const int32_t *q = sh->rec + ((size_t)i * nrec + r) * 2;
            const int px = q[0] + g.P, pz = q[1] + g.P;
            const int tile = (pz / TZ) * g.ntx + px / TX;
            const int cell = (pz % TZ) * TX + px % TX;
            keyed.push_back({(long long)tile << 32 | (long long)cell << 20 | r, rec_pack(cell, r)});
        }
        std::sort(keyed.begin(), keyed.end());
        int *off = m->h_off.data() + (size_t)i * (ntiles + 1);
        size_t base = m->h_ent.size();
        int e = 0;
        for (int tl = 0; tl < ntiles; ++tl) {
            off[tl] = (int)(base + e);
            while (e < (int)keyed.size() && (int)(keyed[e].first >> 32) == tl) {
                m->h_ent.push_back(keyed[e].second);
                ++e;
            }
        }
        off[ntiles] = (int)(base + e);
    }
    HIPCHECK(hipMemcpyAsync(m->src_cell, m->h_src.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(m->rec_off, m->h_off.data(), sizeof(int) * m->h_off.size(), hipMemcpyHostToDevice, s));
    if (!m->h_ent.empty())
        HIPCHECK(hipMemcpyAsync(m->rec_ent, m->h_ent.data(), sizeof(int) * m->h_ent.size(), hipMemcpyHostToDevice, s));
    m->geom_src.assign(sh->src, sh->src + 2 * ns);
    m->geom_rec.assign(sh->rec ? sh->rec : sh->src, sh->rec ? sh->rec + (size_t)2 * ns * nrec : sh->src);
    m->geom_nshots = ns;
    m->geom_nrec = nrec;
    m->have_ckpt = false;
    return SG_OK;
}

int check_shots(const sg_model *m, const sg_shots *sh)
{
    if (!sh) return fail(SG_EINVAL, "shots is NULL");
    if (sh->nshots < 1 || sh->nshots > m->max_shots)
        return fail(SG_EINVAL, "nshots %d outside [1, %d]", sh->nshots, m->max_shots);
    if (sh->nshots % m->d.nmodels)
        return fail(SG_EINVAL, "nshots %d is not a multiple of nmodels %d", sh->nshots, m->d.nmodels);
    if (sh->nrec < 0 || sh->nrec > m->max_rec)
        return fail(SG_EINVAL, "nrec %d outside [0, %d]", sh->nrec, m->max_rec);
    if (!sh->wavelet) return fail(SG_EINVAL, "wavelet is NULL");
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

Ac2FwdArgs fwd_args(const sg_model *m, int ns, const float *wav, int cu)
{
    Ac2FwdArgs a{};
    a.g = m->L.g;
    a.nshots = ns;
    a.u = m->fwd[cu];
    a.um = m->fwd[1 - cu];
    a.chat = m->chat;
    a.shots_per_model = ns / m->d.nmodels;
    a.phx = m->fwd[2];
    a.phz = m->fwd[3];
    a.hx = m->hx;
    a.hz = m->hz;
    a.src_cell = m->src_cell;
    a.wav = wav;
    a.nt = m->d.nt;
    a.src_scale = (float)(m->d.dt * m->d.dt / (m->d.dx * m->d.dx));
    a.rec_off = m->rec_off;
    a.rec_ent = m->rec_ent;
    a.nrec = m->geom_nrec;
    return a;
}

// One forward step: layer auxiliary fields from u^k, then the tile update.
void fwd_step(const sg_model *m, Ac2FwdArgs a, int k, float *seis, float *snap, hipStream_t s)
{
    Ac2PhiArgs p{};
    p.g = a.g;
    p.u = a.u;
    p.phx = m->fwd[2];
    p.phz = m->fwd[3];
    p.hx = m->hx; p.hz = m->hz; p.px = m->px; p.pz = m->pz; p.ihx = m->ihx; p.ihz = m->ihz;
    launch_ac2_phi(p, a.nshots, s);
    a.k = k;
    a.seis = seis;
    a.snap = snap;
    launch_ac2_fwd(a, s);
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
    return make_layout(d, max_shots, max_rec, ckpt_every).total;
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
    if (vs || rho) return fail(SG_EINVAL, "vs and rho must be NULL for acoustic models");
    if (!vp || !ws) return fail(SG_EINVAL, "vp and ws must be device pointers");
    if (max_shots < 1 || max_rec < 0 || ckpt_every < 0)
        return fail(SG_EINVAL, "max_shots >= 1, max_rec >= 0 and ckpt_every >= 0 required");
    if (max_shots % d->nmodels) return fail(SG_EINVAL, "max_shots must be a multiple of nmodels");
    if ((long long)max_rec >= (1LL << REC_ID_BITS)) return fail(SG_EINVAL, "at most %d receivers per shot", (1 << REC_ID_BITS) - 1);
    const Layout L = make_layout(d, max_shots, max_rec, ckpt_every);
    if (ws_bytes < L.total) return fail(SG_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if ((uintptr_t)ws % ALIGN) return fail(SG_EINVAL, "workspace must be %zu-byte aligned", ALIGN);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // stability: velocity range from the device copy
    const size_t nphys = (size_t)d->nmodels * d->nx * d->nz;
    std::vector<float> hv(nphys);
    HIPCHECK(hipMemcpyAsync(hv.data(), vp, sizeof(float) * nphys, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    float vmin = hv[0], vmax = hv[0];
    for (float v : hv) {
        if (!(v > 0) || !std::isfinite(v)) return fail(SG_EINVAL, "velocity must be positive and finite");
        vmin = std::min(vmin, v);
        vmax = std::max(vmax, v);
    }
    const double limit = 2.0 / std::sqrt(L8_SYMBOL_MAX * d->ndim);
    const double cfl = vmax * d->dt / d->dx;
    if (cfl > 0.95 * limit)
        return fail(SG_EUNSTABLE, "CFL number %.4f above 0.95 x %.4f", cfl, limit);
    const Grid2 &g = L.g;
    const double zmax = d->npml > 0 ? 3.0 * d->pml_vmax * std::log(1.0 / d->pml_R) / (2.0 * d->npml * d->dx) : 0.0;
    if (zmax * d->dt > 0.3) return fail(SG_EUNSTABLE, "zeta_max*dt = %.3f above 0.3", zmax * d->dt);

    sg_model *m = new sg_model();
    m->d = *d;
    m->L = L;
    m->max_shots = max_shots;
    m->max_rec = max_rec;
    m->ws = static_cast<char *>(ws);
    m->chat = reinterpret_cast<float *>(m->ws + L.off_chat);
    m->cpad = reinterpret_cast<float *>(m->ws + L.off_cpad);
    float *tab = reinterpret_cast<float *>(m->ws + L.off_tab);
    m->hx = tab;
    m->px = tab + g.NX;
    m->ihx = tab + 2 * g.NX;
    m->hz = tab + 3 * g.NX;
    m->pz = m->hz + g.NZ;
    m->ihz = m->hz + 2 * g.NZ;
    for (int i = 0; i < 4; ++i) {
        m->fwd[i] = reinterpret_cast<float *>(m->ws + L.off_fwd) + i * L.field;
        m->adj[i] = reinterpret_cast<float *>(m->ws + L.off_adj) + i * L.field;
    }
    m->ckpt = reinterpret_cast<float *>(m->ws + L.off_ckpt);
    m->snap = reinterpret_cast<float *>(m->ws + L.off_snap);
    m->grad = reinterpret_cast<float *>(m->ws + L.off_grad);
    m->src_cell = reinterpret_cast<int *>(m->ws + L.off_src);
    m->rec_off = reinterpret_cast<int *>(m->ws + L.off_recoff);
    m->rec_ent = reinterpret_cast<int *>(m->ws + L.off_recent);
    m->partials = reinterpret_cast<double *>(m->ws + L.off_part);

    // damping tables per axis, FP64 rounded once: h = zeta dt / 2,
    // p = (1-h)/(1+h), 1/(1+h)
    auto profile = [&](int n, float *h, float *p, float *ih) {
        for (int i = 0; i < n + 2 * d->npml; ++i) {
            int depth = i < d->npml ? d->npml - i : (i >= d->npml + n ? i - (d->npml + n - 1) : 0);
            const double r = d->npml > 0 ? (double)depth / d->npml : 0.0;
            const double hv = 0.5 * d->dt * zmax * r * r;
            h[i] = (float)hv;
            p[i] = (float)((1.0 - hv) / (1.0 + hv));
            ih[i] = (float)(1.0 / (1.0 + hv));
        }
    };
    m->h_tab.assign(3 * (g.NX + g.NZ), 0.f);
    float *ht = m->h_tab.data();
    profile(d->nx, ht, ht + g.NX, ht + 2 * g.NX);
    profile(d->nz, ht + 3 * g.NX, ht + 3 * g.NX + g.NZ, ht + 3 * g.NX + 2 * g.NZ);
    hipError_t e = hipMemcpyAsync(tab, ht, sizeof(float) * m->h_tab.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        delete m;
        return fail(SG_EDEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    launch_ac2_prep(g, d->nmodels, vp, d->dt, d->dx, m->chat, m->cpad, s);
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete m;
        return fail(SG_EDEVICE, "model preparation failed: %s", hipGetErrorString(e));
    }
    *out = m;
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
    const int ns = sh->nshots, nt = m->d.nt, K = m->L.K;
    const Grid2 &g = m->L.g;
    const long long fs = (long long)ns * g.plane;  // floats of one field over the batch
    for (int i = 0; i < 4; ++i) launch_fill(m->fwd[i], fs, 0.f, s);
    int cu = 0;
    int span = -1;
    for (int k = 0; k < nt; ++k) {
        if (k % K == 0) {
            span_end(m, span, s);
            span = span_begin(m, 0, std::min(K, nt - k), s);
        }
        if (save_ckpt && k % K == 0) {
            float *ck = m->ckpt + (size_t)(k / K) * 4 * m->L.field;
            HIPCHECK(hipMemcpyAsync(ck, m->fwd[cu], sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
            HIPCHECK(hipMemcpyAsync(ck + m->L.field, m->fwd[1 - cu], sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
            HIPCHECK(hipMemcpyAsync(ck + 2 * m->L.field, m->fwd[2], sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
            HIPCHECK(hipMemcpyAsync(ck + 3 * m->L.field, m->fwd[3], sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
        }
        fwd_step(m, fwd_args(m, ns, sh->wavelet, cu), k, sh->nrec > 0 ? seis : nullptr, nullptr, s);
        cu = 1 - cu;
    }
    span_end(m, span, s);
    HIPCHECK(hipGetLastError());
    m->have_ckpt = save_ckpt != 0;
    m->ckpt_nshots = ns;
    return SG_OK;
}

int misfit(sg_model *m, const float *pred, const float *obs, int64_t n, double *J_dev,
           float *resid, sg_stream_t stream)
{
    g_err.clear();
    if (!pred || !obs || !J_dev || n < 0) return fail(SG_EINVAL, "bad misfit arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    launch_misfit(pred, obs, n, resid, m ? m->partials : nullptr, m ? 4096 : 1, J_dev, s);
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
    if (g_vs || g_rho) return fail(SG_EINVAL, "g_vs and g_rho must be NULL for acoustic models");
    if (!g_vp || (!dJ_dd && sh->nrec > 0)) return fail(SG_EINVAL, "g_vp / dJ_dd is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // geometry must be the one of the checkpointed forward
    const int ns = sh->nshots;
    const bool same = m->have_ckpt && m->geom_nshots == ns && m->geom_nrec == sh->nrec &&
                      std::equal(sh->src, sh->src + 2 * ns, m->geom_src.begin()) &&
                      (sh->nrec == 0 || std::equal(sh->rec, sh->rec + (size_t)2 * ns * sh->nrec, m->geom_rec.begin()));
    if (!same) return fail(SG_ESTATE, "no checkpointed forward of these shots precedes the adjoint");
    const int nt = m->d.nt, K = m->L.K;
    const Grid2 &g = m->L.g;
    const long long fs = (long long)ns * g.plane;
    for (int i = 0; i < 4; ++i) launch_fill(m->adj[i], fs, 0.f, s);
    launch_fill(m->grad, fs, 0.f, s);

    Ac2AdjArgs b{};
    b.g = g;
    b.nshots = ns;
    b.cx = m->adj[2];
    b.cz = m->adj[3];
    b.chat = m->chat;
    b.shots_per_model = ns / m->d.nmodels;
    b.hx = m->hx;
    b.hz = m->hz;
    b.src_cell = m->src_cell;
    b.gwav = g_wavelet;
    b.nt = nt;
    b.src_scale = (float)(m->d.dt * m->d.dt / (m->d.dx * m->d.dx));
    b.rec_off = m->rec_off;
    b.rec_ent = m->rec_ent;
    b.dJdd = dJ_dd;
    b.nrec = sh->nrec;
    b.grad = m->grad;
    Ac2PhiAdjArgs pa{};
    pa.g = g;
    pa.chat = m->chat;
    pa.shots_per_model = b.shots_per_model;
    pa.cx = m->adj[2];
    pa.cz = m->adj[3];
    pa.hx = m->hx; pa.hz = m->hz; pa.px = m->px; pa.pz = m->pz; pa.ihx = m->ihx; pa.ihz = m->ihz;
    int ca = 0;   // s^{k+2} = adj[ca], s^{k+3} = adj[1-ca]
    for (int seg = m->L.nseg - 1; seg >= 0; --seg) {
        const int k0 = seg * K, k1 = std::min(k0 + K, nt);
        const float *ck = m->ckpt + (size_t)seg * 4 * m->L.field;
        HIPCHECK(hipMemcpyAsync(m->fwd[0], ck, sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->fwd[1], ck + m->L.field, sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->fwd[2], ck + 2 * m->L.field, sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipMemcpyAsync(m->fwd[3], ck + 3 * m->L.field, sizeof(float) * fs, hipMemcpyDeviceToDevice, s));
        int cu = 0;
        int span = span_begin(m, 1, k1 - k0, s);
        for (int k = k0; k < k1; ++k) {
            float *snap = m->snap + (size_t)(k - k0) * m->L.field;
            fwd_step(m, fwd_args(m, ns, sh->wavelet, cu), k, nullptr, snap, s);
            cu = 1 - cu;
        }
        span_end(m, span, s);
        span = span_begin(m, 2, k1 - k0, s);
        for (int k = k1 - 1; k >= k0; --k) {
            b.k = k;
            b.snap = m->snap + (size_t)(k - k0) * m->L.field;
            b.s2 = m->adj[ca];
            b.s3 = m->adj[1 - ca];
            pa.s2 = b.s2;
            launch_ac2_phi_adj(pa, ns, s);
            launch_ac2_adj(b, s);
            ca = 1 - ca;
        }
        span_end(m, span, s);
    }
    // the snapshot buffer (free now) holds the per-model shot sums
    launch_ac2_finalize(g, m->d.nmodels, ns / m->d.nmodels, m->grad, m->snap, m->cpad, m->d.dt, m->d.dx, g_vp, s);
    HIPCHECK(hipGetLastError());
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
