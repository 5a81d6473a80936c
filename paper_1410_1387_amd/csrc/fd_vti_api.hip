// fd_vti_api.hip -- host side of the VTI part of the C ABI declared in
// include/fdwave.h: the per-plane z weights (Fornberg's recursion), the stability
// limit, the padded layout and workspace plan, model preparation, the
// source/receiver event tables, launch dispatch and state copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fdwave.h"
#include "fd_host.h"
#include "fd_util.h"
#include "fd_vti.h"

using namespace fdw;

#define fail fdw::host_fail

#define HIP_TRY(ctxp, expr)                                                                      \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            if (ctxp) (ctxp)->poisoned = true;                                                   \
            return fail(FD_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                               \
        }                                                                                        \
    } while (0)

namespace {

constexpr int64_t kRowAlignBytes = 128;  // byte offset of each row's interior
constexpr int kMaxRz = 8;

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool radii_ok(int rxy, int rz)
{
    const bool xy = rxy == 2 || rxy == 4 || rxy == 8 || rxy == 12;
    const bool z = rz == 1 || rz == 2 || rz == 4 || rz == 8;
    return xy && z && rz <= rxy;
}

enum { F_P0, F_P1, F_Q0, F_Q1, F_AX, F_AN, F_AZ, F_COUNT };

struct VtiLayout {
    size_t esize;
    int rxy, rz;
    int64_t nx, ny, nz;
    int64_t px, py, planes, pxy, off0;
    size_t field_bytes;
    size_t o_field[F_COUNT], o_wz, o_partial, o_out, o_evptr, o_ev, o_src, total;
    int64_t ncol;
};

bool make_vti_layout(const fd_grid *g, int rxy, int rz, fd_dtype dt, int64_t max_src, int64_t max_rec,
                     VtiLayout *L)
{
    if (!g || g->ndim != 3 || !radii_ok(rxy, rz)) return false;
    if (dt != FD_F32 && dt != FD_F64) return false;
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 1 || g->n[a] > (1 << 30)) return false;
    if (max_src < 0 || max_rec < 0) return false;
    L->esize = dt == FD_F32 ? 4 : 8;
    L->rxy = rxy;
    L->rz = rz;
    L->nx = g->n[0];
    L->ny = g->n[1];
    L->nz = g->n[2];
    const int64_t xo = kRowAlignBytes / (int64_t)L->esize;  // >= 16 >= the largest x halo (12)
    L->px = align_up(xo + align_up(L->nx, 256) + 16, kRowAlignBytes / (int64_t)L->esize);
    L->py = rxy + align_up(L->ny, 64) + rxy;
    L->planes = L->nz + 2 * rz;
    L->pxy = L->px * L->py;
    L->off0 = (int64_t)rz * L->pxy + (int64_t)rxy * L->px + xo;
    L->field_bytes = (size_t)align_up(L->pxy * L->planes * (int64_t)L->esize, 256);
    L->ncol = L->nx * L->ny;
    if (L->ncol + 1 > INT32_MAX || max_src + max_rec > INT32_MAX / 2) return false;
    if (L->pxy * (int64_t)L->esize >= ((int64_t)1 << 31)) return false;  // 32-bit in-plane offsets
    size_t o = 0;
    for (int f = 0; f < F_COUNT; ++f) {
        L->o_field[f] = o;
        o += L->field_bytes;
    }
    L->o_wz = o;
    o += align_up(L->nz * (2 * rz + 1) * (int64_t)L->esize, 256);
    L->o_partial = o;
    o += align_up(3 * kPrepBlocks * sizeof(double), 256);
    L->o_out = o;
    o += 256;
    L->o_evptr = o;
    o += align_up((L->ncol + 1) * (int64_t)sizeof(int32_t), 256);
    L->o_ev = o;
    o += align_up(std::max<int64_t>(1, max_src + max_rec) * (int64_t)sizeof(Event), 256);
    L->o_src = o;
    o += align_up(std::max<int64_t>(1, max_src) * (int64_t)sizeof(VtiSource), 256);
    L->total = o;
    return true;
}

// Second-derivative weights at the origin for the nodes x[0..n-1] (offsets from the
// evaluation point), by Fornberg's recursion (Math. Comp. 51, 1988): the weights of
// the derivatives of order 0..2 for the first i+1 nodes are updated from those for the
// first i nodes as each node is added, which is the Lagrange-basis construction done
// incrementally.  d2[j] receives the weight of node j.
void fornberg_d2(const double *x, int n, double *d2)
{
    double C[2 * kMaxRz + 1][3];
    for (int j = 0; j < n; ++j) C[j][0] = C[j][1] = C[j][2] = 0.0;
    C[0][0] = 1.0;
    double c1 = 1.0, c4 = x[0];
    for (int i = 1; i < n; ++i) {
        const int mn = std::min(i, 2);
        double c2 = 1.0;
        const double c5 = c4;
        c4 = x[i];
        for (int j = 0; j < i; ++j) {
            const double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int m = mn; m >= 1; --m) C[i][m] = c1 * ((double)m * C[i - 1][m - 1] - c5 * C[i - 1][m]) / c2;
                C[i][0] = -c1 * c5 * C[i - 1][0] / c2;
            }
            for (int m = mn; m >= 1; --m) C[j][m] = (c4 * C[j][m] - (double)m * C[j][m - 1]) / c3;
            C[j][0] = c4 * C[j][0] / c3;
        }
        c1 = c2;
    }
    for (int j = 0; j < n; ++j) d2[j] = C[j][2];
}

// Plane coordinates (planes -rz .. nz+rz-1): the caller's, or uniform with spacing h.
bool plane_coords(const double *zc, int64_t nz, int rz, double h, std::vector<double> *out)
{
    out->resize((size_t)(nz + 2 * rz));
    for (int64_t i = 0; i < nz + 2 * rz; ++i) (*out)[(size_t)i] = zc ? zc[i] : (double)(i - rz) * h;
    for (size_t i = 0; i < out->size(); ++i) {
        if (!std::isfinite((*out)[i])) return false;
        if (i > 0 && !((*out)[i] > (*out)[i - 1])) return false;
    }
    return true;
}

void z_weight_table(const std::vector<double> &z, int64_t nz, int rz, std::vector<double> *w)
{
    const int n = 2 * rz + 1;
    w->assign((size_t)(nz * n), 0.0);
    double off[2 * kMaxRz + 1];
    for (int64_t k = 0; k < nz; ++k) {
        for (int j = 0; j < n; ++j) off[j] = z[(size_t)(k + j)] - z[(size_t)(k + rz)];
        fornberg_d2(off, n, w->data() + k * n);
    }
}

// Mode-matrix factors: a = 2 S_xy / h^2 (x and y at Nyquist), b = largest row sum of |Dzz|.
void mode_factors(int rxy, double h, const std::vector<double> &w, int rz, double *a, double *b)
{
    double wx[13];
    fd_weights(rxy, wx);
    double S = -wx[0];
    for (int l = 1; l <= rxy; ++l) S += 2.0 * std::fabs(wx[l]);
    *a = 2.0 * S / (h * h);
    const int n = 2 * rz + 1;
    double bm = 0.0;
    for (size_t k = 0; k < w.size() / (size_t)n; ++k) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += std::fabs(w[k * n + j]);
        bm = std::max(bm, r);
    }
    *b = bm;
}

double perron(double A, double B, double C) { return 0.5 * ((A + B) + std::sqrt((A - B) * (A - B) + 4.0 * B * C)); }

struct Tuning {
    int config;
    int zchunk;
};
std::mutex g_vtune_mu;
std::map<std::tuple<int, int, int>, Tuning> g_vtuning;

const VtiEntry *vti_table(fd_dtype dt, int rxy, int rz, int *count)
{
    return dt == FD_F32 ? vti_configs_f32(rxy, rz, count) : vti_configs_f64(rxy, rz, count);
}

struct VtiSourceRec {
    int64_t pos[3];
    const void *wav;
    int64_t nsamp;
    double amp_p, amp_q;
};

}  // namespace

struct fd_vti_ctx {
    fd_grid g;
    int rxy, rz;
    double h, dt;
    fd_dtype dtype;
    hipStream_t stream;
    VtiLayout L;
    char *ws;
    int64_t max_src, max_rec;
    const VtiEntry *kv;
    int zch;
    int64_t tiles_x, tiles_y, chunks_z;
    std::string cfg_name;
    std::vector<double> dzc;  // z extent of each plane's cell
    VtiDesc desc;
    std::vector<VtiSourceRec> sources;
    std::vector<int32_t> rec_pos;
    int64_t nrec;
    void *traces_p, *traces_q;
    int64_t rec_cap, rec_base;
    std::vector<int32_t> h_evptr;
    std::vector<Event> h_ev;
    std::vector<VtiSource> h_src;
    int64_t step;
    bool poisoned;

    void *field(int f) const { return ws + L.o_field[f]; }
    Geom geom() const
    {
        Geom gm;
        gm.nx = L.nx;
        gm.ny = L.ny;
        gm.nz = L.nz;
        gm.px = L.px;
        gm.pxy = L.pxy;
        gm.off0 = L.off0;
        return gm;
    }
};

static int check_vctx(const fd_vti_ctx *c)
{
    if (!c) return fail(FD_E_INVAL, "null VTI context");
    if (c->poisoned) return fail(FD_E_STATE, "VTI context is poisoned by an earlier device error");
    return FD_OK;
}

static int upload_vti_tables(fd_vti_ctx *c)
{
    const VtiLayout &L = c->L;
    struct Tmp {
        int64_t col;
        int32_t z, code;
    };
    std::vector<Tmp> all;
    c->h_src.clear();
    for (size_t s = 0; s < c->sources.size(); ++s) {
        const VtiSourceRec &sr = c->sources[s];
        all.push_back(Tmp{sr.pos[1] * L.nx + sr.pos[0], (int32_t)sr.pos[2], ~(int32_t)s});
        const double k = c->dt * c->dt / (c->h * c->h * c->dzc[(size_t)sr.pos[2]]);
        c->h_src.push_back(VtiSource{sr.wav, sr.nsamp, sr.amp_p * k, sr.amp_q * k});
    }
    for (int64_t j = 0; j < c->nrec; ++j)
        all.push_back(Tmp{(int64_t)c->rec_pos[3 * j + 1] * L.nx + c->rec_pos[3 * j], c->rec_pos[3 * j + 2], (int32_t)j});
    // sources sort before receivers at the same point (negative codes first)
    std::sort(all.begin(), all.end(), [](const Tmp &a, const Tmp &b) {
        if (a.col != b.col) return a.col < b.col;
        if (a.z != b.z) return a.z < b.z;
        return a.code < b.code;
    });
    c->h_ev.resize(all.size());
    c->h_evptr.assign((size_t)L.ncol + 1, 0);
    for (size_t i = 0; i < all.size(); ++i) {
        c->h_ev[i] = Event{all[i].z, all[i].code};
        c->h_evptr[(size_t)all[i].col + 1]++;
    }
    for (int64_t i = 0; i < L.ncol; ++i) c->h_evptr[(size_t)i + 1] += c->h_evptr[(size_t)i];
    VtiDesc &d = c->desc;
    const bool any = !all.empty();
    d.ev_ptr = any ? reinterpret_cast<const int32_t *>(c->ws + L.o_evptr) : nullptr;
    d.ev = reinterpret_cast<const Event *>(c->ws + L.o_ev);
    d.src = reinterpret_cast<const VtiSource *>(c->ws + L.o_src);
    d.traces_p = c->traces_p;
    d.traces_q = c->traces_q;
    d.nrec = c->nrec;
    d.rec_base = c->rec_base;
    d.rec_cap = c->rec_cap;
    if (any) {
        HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_evptr, c->h_evptr.data(), c->h_evptr.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_ev, c->h_ev.data(), c->h_ev.size() * sizeof(Event),
                                  hipMemcpyHostToDevice, c->stream));
        if (!c->h_src.empty())
            HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_src, c->h_src.data(), c->h_src.size() * sizeof(VtiSource),
                                      hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FD_OK;
}

// ------------------------------------------------------------------ weights and limits

extern "C" int fd_vti_z_weights(const double *zc, int64_t nz, int rz, double *w)
{
    if (!zc || !w || nz < 1 || rz < 1 || rz > kMaxRz) return fail(FD_E_INVAL, "fd_vti_z_weights: bad arguments");
    std::vector<double> z, tab;
    if (!plane_coords(zc, nz, rz, 1.0, &z))
        return fail(FD_E_INVAL, "fd_vti_z_weights: coordinates must be finite and strictly increasing");
    z_weight_table(z, nz, rz, &tab);
    std::memcpy(w, tab.data(), tab.size() * sizeof(double));
    return FD_OK;
}

extern "C" double fd_vti_dt_max(int rxy, int rz, double h, const double *zc, int64_t nz, double vz_max,
                                double eps_max, double delta_max)
{
    if (!radii_ok(rxy, rz) || !(h > 0) || !std::isfinite(h) || nz < 1 || !(vz_max > 0) || !std::isfinite(vz_max) ||
        !(1.0 + 2.0 * eps_max > 0) || !(1.0 + 2.0 * delta_max >= 0) || !std::isfinite(eps_max) ||
        !std::isfinite(delta_max))
        return -1.0;
    std::vector<double> z, tab;
    if (!plane_coords(zc, nz, rz, h, &z)) return -1.0;
    z_weight_table(z, nz, rz, &tab);
    double a, b;
    mode_factors(rxy, h, tab, rz, &a, &b);
    const double z2 = vz_max * vz_max;
    const double lam = perron(z2 * (1.0 + 2.0 * eps_max) * a, z2 * b, z2 * (1.0 + 2.0 * delta_max) * a);
    return 2.0 / std::sqrt(lam);
}

extern "C" int fd_vti_workspace_bytes(const fd_grid *g, int rxy, int rz, fd_dtype dtype, int64_t max_sources,
                                      int64_t max_receivers, size_t *bytes)
{
    VtiLayout L;
    if (!bytes || !make_vti_layout(g, rxy, rz, dtype, max_sources, max_receivers, &L))
        return fail(FD_E_INVAL, "fd_vti_workspace_bytes: bad grid (3-D), radius pair, dtype or maxima");
    *bytes = L.total;
    return FD_OK;
}

extern "C" int fd_vti_set_tuning(fd_dtype dtype, int rxy, int rz, int config, int zchunk)
{
    int count = 0;
    if ((dtype != FD_F32 && dtype != FD_F64) || !radii_ok(rxy, rz))
        return fail(FD_E_INVAL, "fd_vti_set_tuning: bad dtype or radius pair");
    vti_table(dtype, rxy, rz, &count);
    if (config < 0 || config >= count || zchunk < 0)
        return fail(FD_E_RANGE, "fd_vti_set_tuning: config %d of %d, zchunk %d", config, count, zchunk);
    std::lock_guard<std::mutex> lk(g_vtune_mu);
    g_vtuning[std::make_tuple((int)dtype, rxy, rz)] = Tuning{config, zchunk};
    return FD_OK;
}

// ------------------------------------------------------------------ lifecycle

extern "C" int fd_vti_create(fd_vti_ctx **out, const fd_grid *g, int rxy, int rz, double h, const double *zc,
                             double dt, const void *vz, const void *eps, const void *delta, fd_dtype dtype,
                             void *workspace, size_t ws_bytes, int64_t max_sources, int64_t max_receivers,
                             void *stream)
{
    if (!out) return fail(FD_E_INVAL, "fd_vti_create: null out");
    *out = nullptr;
    VtiLayout L;
    if (!make_vti_layout(g, rxy, rz, dtype, max_sources, max_receivers, &L))
        return fail(FD_E_INVAL, "fd_vti_create: bad grid (3-D, n >= 1), radius pair (rxy in {2,4,8,12}, rz in "
                                "{1,2,4,8}, rz <= rxy), dtype or maxima");
    if (!(h > 0) || !(dt > 0) || !std::isfinite(h) || !std::isfinite(dt))
        return fail(FD_E_INVAL, "fd_vti_create: h and dt must be positive");
    if (!vz || !eps || !delta || !workspace) return fail(FD_E_INVAL, "fd_vti_create: null model or workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(FD_E_INVAL, "fd_vti_create: workspace not 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(FD_E_NOMEM, "fd_vti_create: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    std::vector<double> z, wtab;
    if (!plane_coords(zc, L.nz, rz, h, &z))
        return fail(FD_E_INVAL, "fd_vti_create: z coordinates must be finite and strictly increasing");
    z_weight_table(z, L.nz, rz, &wtab);
    double fa, fb;
    mode_factors(rxy, h, wtab, rz, &fa, &fb);

    int count = 0;
    const VtiEntry *tab = vti_table(dtype, rxy, rz, &count);
    if (!tab || count == 0) return fail(FD_E_INVAL, "fd_vti_create: no kernel for this dtype and radius pair");
    Tuning tu{0, 0};
    {
        std::lock_guard<std::mutex> lk(g_vtune_mu);
        auto it = g_vtuning.find(std::make_tuple((int)dtype, rxy, rz));
        if (it != g_vtuning.end()) tu = it->second;
    }

    fd_vti_ctx *c = new fd_vti_ctx();
    c->g = *g;
    c->rxy = rxy;
    c->rz = rz;
    c->h = h;
    c->dt = dt;
    c->dtype = dtype;
    c->stream = (hipStream_t)stream;
    c->L = L;
    c->ws = (char *)workspace;
    c->max_src = max_sources;
    c->max_rec = max_receivers;
    c->kv = &tab[tu.config];
    c->tiles_x = (L.nx + c->kv->bx - 1) / c->kv->bx;
    c->tiles_y = (L.ny + c->kv->by - 1) / c->kv->by;
    c->zch = tu.zchunk > 0 ? (int)std::min<int64_t>(tu.zchunk, L.nz)
                           : choose_zch(c->tiles_x * c->tiles_y, L.nz, rz, resident_slots(c->kv->kernel, c->kv->nt));
    c->chunks_z = (L.nz + c->zch - 1) / c->zch;
    c->dzc.resize((size_t)L.nz);
    for (int64_t k = 0; k < L.nz; ++k) c->dzc[(size_t)k] = 0.5 * (z[(size_t)(k + rz + 1)] - z[(size_t)(k + rz - 1)]);
    c->nrec = 0;
    c->traces_p = c->traces_q = nullptr;
    c->rec_cap = c->rec_base = 0;
    c->step = 0;
    c->poisoned = false;
    char nm[256];
    snprintf(nm, sizeof(nm), "%s, zchunk %d, grid %lld wg", c->kv->name, c->zch,
             (long long)(c->tiles_x * c->tiles_y * c->chunks_z));
    c->cfg_name = nm;

    // the z weights in units of h (times h^2), in the working precision
    const int nw = 2 * rz + 1;
    std::vector<float> wf;
    std::vector<double> wd;
    if (dtype == FD_F32) {
        wf.resize(wtab.size());
        for (size_t i = 0; i < wtab.size(); ++i) wf[i] = (float)(wtab[i] * h * h);
    } else {
        wd.resize(wtab.size());
        for (size_t i = 0; i < wtab.size(); ++i) wd[i] = wtab[i] * h * h;
    }
    double red[3] = {0, 0, 0};
    hipError_t e = hipMemsetAsync(workspace, 0, L.total, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.o_wz, dtype == FD_F32 ? (const void *)wf.data() : (const void *)wd.data(),
                           (size_t)(L.nz * nw) * L.esize, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_vti_prep((int)dtype, c->geom(), vz, eps, delta, c->field(F_AX), c->field(F_AN), c->field(F_AZ),
                            (dt / h) * (dt / h), fa, fb, (double *)(c->ws + L.o_partial), (double *)(c->ws + L.o_out),
                            c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(red, c->ws + L.o_out, sizeof(red), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(FD_E_DEVICE, "fd_vti_create: %s", hipGetErrorString(e));
    }
    if (red[1] != 0.0) {
        delete c;
        return fail(FD_E_INVAL, "fd_vti_create: model must have vz > 0, 1 + 2 eps > 0, 1 + 2 delta >= 0, all finite");
    }
    if (red[2] != 0.0) {
        delete c;
        return fail(FD_E_UNSTABLE, "fd_vti_create: delta > eps somewhere: the coupled system has a growing mode");
    }
    const double dtm = 2.0 / std::sqrt(red[0]);
    if (dt > dtm * (1.0 + 1e-12)) {
        delete c;
        return fail(FD_E_UNSTABLE, "fd_vti_create: dt %.6g exceeds the stability limit %.6g", dt, dtm);
    }

    VtiDesc &d = c->desc;
    std::memset(&d, 0, sizeof(d));
    d.pbuf[0] = c->field(F_P0);
    d.pbuf[1] = c->field(F_P1);
    d.qbuf[0] = c->field(F_Q0);
    d.qbuf[1] = c->field(F_Q1);
    d.ax = c->field(F_AX);
    d.an = c->field(F_AN);
    d.az = c->field(F_AZ);
    d.wz = c->ws + L.o_wz;
    d.nx = (int32_t)L.nx;
    d.ny = (int32_t)L.ny;
    d.nz = (int32_t)L.nz;
    d.tiles_x = (int32_t)c->tiles_x;
    d.tiles_y = (int32_t)c->tiles_y;
    d.chunks_z = (int32_t)c->chunks_z;
    d.zch = c->zch;
    d.xcd_remap = 1;
    d.px = L.px;
    d.pxy = L.pxy;
    d.off0 = L.off0;
    int st = upload_vti_tables(c);
    if (st != FD_OK) {
        delete c;
        return st;
    }
    *out = c;
    return FD_OK;
}

extern "C" int fd_vti_destroy(fd_vti_ctx *ctx)
{
    if (!ctx) return fail(FD_E_INVAL, "fd_vti_destroy: null context");
    if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return FD_OK;
}

extern "C" const char *fd_vti_kernel_config(const fd_vti_ctx *ctx) { return ctx ? ctx->cfg_name.c_str() : ""; }

// ------------------------------------------------------------------ sources and receivers

static bool vti_in_grid(const fd_vti_ctx *c, const int64_t *p)
{
    for (int a = 0; a < 3; ++a)
        if (p[a] < 0 || p[a] >= c->g.n[a]) return false;
    return true;
}

extern "C" int fd_vti_inject(fd_vti_ctx *ctx, const void *wavelet, int64_t nsamp, const int64_t pos[3], double amp_p,
                             double amp_q)
{
    int st = check_vctx(ctx);
    if (st) return st;
    if (!pos || nsamp < 0 || (nsamp > 0 && !wavelet) || !std::isfinite(amp_p) || !std::isfinite(amp_q))
        return fail(FD_E_INVAL, "fd_vti_inject: bad wavelet, nsamp or amplitudes");
    if (!vti_in_grid(ctx, pos))
        return fail(FD_E_RANGE, "fd_vti_inject: position (%lld, %lld, %lld) outside the grid", (long long)pos[0],
                    (long long)pos[1], (long long)pos[2]);
    if ((int64_t)ctx->sources.size() >= ctx->max_src)
        return fail(FD_E_RANGE, "fd_vti_inject: more than max_sources = %lld", (long long)ctx->max_src);
    VtiSourceRec sr;
    std::memcpy(sr.pos, pos, sizeof(sr.pos));
    sr.wav = wavelet;
    sr.nsamp = nsamp;
    sr.amp_p = amp_p;
    sr.amp_q = amp_q;
    ctx->sources.push_back(sr);
    return upload_vti_tables(ctx);
}

extern "C" int fd_vti_record(fd_vti_ctx *ctx, const int32_t *pos, int64_t nrec, void *traces_p, void *traces_q,
                             int64_t cap)
{
    int st = check_vctx(ctx);
    if (st) return st;
    if (nrec < 0 || (nrec > 0 && (!pos || (!traces_p && !traces_q) || cap < 0)))
        return fail(FD_E_INVAL, "fd_vti_record: bad receiver arguments");
    if (nrec > ctx->max_rec)
        return fail(FD_E_RANGE, "fd_vti_record: %lld receivers > max_receivers = %lld", (long long)nrec,
                    (long long)ctx->max_rec);
    std::vector<int32_t> rp((size_t)nrec * 3);
    for (int64_t j = 0; j < nrec; ++j) {
        const int64_t p[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
        if (!vti_in_grid(ctx, p)) return fail(FD_E_RANGE, "fd_vti_record: receiver %lld outside the grid", (long long)j);
        for (int a = 0; a < 3; ++a) rp[3 * j + a] = (int32_t)p[a];
    }
    ctx->rec_pos.swap(rp);
    ctx->nrec = nrec;
    ctx->traces_p = nrec > 0 ? traces_p : nullptr;
    ctx->traces_q = nrec > 0 ? traces_q : nullptr;
    ctx->rec_cap = nrec > 0 ? cap : 0;
    ctx->rec_base = ctx->step;
    return upload_vti_tables(ctx);
}

// ------------------------------------------------------------------ stepping and state

extern "C" int fd_vti_step(fd_vti_ctx *ctx, int64_t nsteps)
{
    int st = check_vctx(ctx);
    if (st) return st;
    if (nsteps < 0) return fail(FD_E_INVAL, "fd_vti_step: negative nsteps");
    if (ctx->nrec > 0 && ctx->step + nsteps - ctx->rec_base > ctx->rec_cap)
        return fail(FD_E_RANGE, "fd_vti_step: trace capacity %lld exceeded", (long long)ctx->rec_cap);
    const int nwg = (int)(ctx->tiles_x * ctx->tiles_y * ctx->chunks_z);
    for (int64_t i = 0; i < nsteps; ++i) {
        ctx->kv->launch(ctx->desc, ctx->step, nwg, ctx->stream);
        HIP_TRY(ctx, hipGetLastError());
        ctx->step++;
    }
    return FD_OK;
}

extern "C" int fd_vti_sync(fd_vti_ctx *ctx)
{
    int st = check_vctx(ctx);
    if (st) return st;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipGetLastError());
    return FD_OK;
}

extern "C" int fd_vti_get_step(const fd_vti_ctx *ctx, int64_t *step)
{
    if (!ctx || !step) return fail(FD_E_INVAL, "fd_vti_get_step: null argument");
    *step = ctx->step;
    return FD_OK;
}

extern "C" int fd_vti_get_state(fd_vti_ctx *ctx, void *p, void *p_prev, void *q, void *q_prev)
{
    int st = check_vctx(ctx);
    if (st) return st;
    const int cb = (int)(ctx->step & 1), pb = cb ^ 1;
    void *dst[4] = {p, p_prev, q, q_prev};
    const int src[4] = {F_P0 + cb, F_P0 + pb, F_Q0 + cb, F_Q0 + pb};
    for (int i = 0; i < 4; ++i)
        if (dst[i]) HIP_TRY(ctx, launch_pack((int)ctx->dtype, ctx->geom(), ctx->field(src[i]), dst[i], ctx->stream));
    return FD_OK;
}

extern "C" int fd_vti_set_state(fd_vti_ctx *ctx, const void *p, const void *p_prev, const void *q, const void *q_prev,
                                int64_t step)
{
    int st = check_vctx(ctx);
    if (st) return st;
    if (step < 0) return fail(FD_E_INVAL, "fd_vti_set_state: negative step");
    // a step of the other parity swaps the roles of the two buffers of each field
    if ((step & 1) != (ctx->step & 1) && !(p && p_prev && q && q_prev))
        return fail(FD_E_INVAL, "fd_vti_set_state: a step of the other parity needs all four fields");
    const int cb = (int)(step & 1), pb = cb ^ 1;
    const void *srcp[4] = {p, p_prev, q, q_prev};
    const int dst[4] = {F_P0 + cb, F_P0 + pb, F_Q0 + cb, F_Q0 + pb};
    for (int i = 0; i < 4; ++i)
        if (srcp[i]) HIP_TRY(ctx, launch_unpack((int)ctx->dtype, ctx->geom(), srcp[i], ctx->field(dst[i]), ctx->stream));
    ctx->step = step;
    return FD_OK;
}
