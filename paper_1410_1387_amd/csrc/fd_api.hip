// fd_api.hip -- host side of the C ABI declared in include/fdwave.h: argument
// validation, the padded layout and workspace plan, the source/receiver event
// tables, launch dispatch, state copies, the checkpointed adjoint driver and the
// batched (graph-captured) serving step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fdwave.h"
#include "fd_fwd2.h"
#include "fd_stencil.h"
#include "fd_types.h"
#include "fd_util.h"
#include "fd_host.h"

using namespace fdw;

// Byte offset of each row's interior: a multiple of the 128-byte cache line.
#ifndef FD_ROW_ALIGN_BYTES
#define FD_ROW_ALIGN_BYTES 128
#endif

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

namespace fdw {
int host_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
}  // namespace fdw

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

extern "C" const char *fd_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ layout

static inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

namespace {

struct Layout {
    int ndim, r;
    size_t esize;
    int64_t knx, kny, knz;   // kernel-axis interior extent
    int64_t px, py, planes;  // row pitch, rows per plane, planes
    int64_t pxy, off0, elems;
    size_t field_bytes;      // one padded field, rounded to 256 bytes
    // workspace offsets
    size_t o_desc, o_partial, o_minmax, o_buf0, o_buf1, o_c, o_evptr, o_ev, o_src, o_damp, total;
    int64_t ncol;
};

bool make_layout(const fd_grid *g, int r, fd_dtype dt, int64_t max_src, int64_t max_rec, Layout *L)
{
    if (!g || (g->ndim != 2 && g->ndim != 3) || r < 1 || r > 8) return false;
    if (dt != FD_F32 && dt != FD_F64) return false;
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 1) return false;
    if (g->ndim == 2 && g->n[2] != 1) return false;
    if (max_src < 0 || max_rec < 0) return false;
    L->ndim = g->ndim;
    L->r = r;
    L->esize = dt == FD_F32 ? 4 : 8;
    const int64_t xo = FD_ROW_ALIGN_BYTES / (int64_t)L->esize;  // interior starts on a cache line
    L->knx = g->n[0];
    L->kny = g->ndim == 3 ? g->n[1] : 1;
    L->knz = g->ndim == 3 ? g->n[2] : g->n[1];
    if (L->knx > (1 << 30) || L->kny > (1 << 30) || L->knz > (1 << 30)) return false;
    L->px = align_up(xo + align_up(L->knx, 256) + 16, 128 / (int64_t)L->esize);
    L->py = g->ndim == 3 ? r + align_up(L->kny, 64) + r : 1;
    L->planes = L->knz + 2 * r;
    L->pxy = L->px * L->py;
    L->off0 = (int64_t)r * L->pxy + (g->ndim == 3 ? (int64_t)r * L->px : 0) + xo;
    L->elems = L->pxy * L->planes;
    L->field_bytes = (size_t)align_up(L->elems * (int64_t)L->esize, 256);
    L->ncol = L->knx * L->kny;
    if (L->ncol + 1 > INT32_MAX || max_src + max_rec > INT32_MAX / 2) return false;
    // kernels address a plane with 32-bit byte offsets
    if (L->pxy * (int64_t)L->esize >= ((int64_t)1 << 31)) return false;
    size_t o = 0;
    L->o_desc = o;
    o += align_up(sizeof(ShotDesc), 256);
    L->o_partial = o;
    o += align_up(2 * kPrepBlocks * sizeof(double), 256);
    L->o_minmax = o;
    o += 256;
    L->o_buf0 = o;
    o += L->field_bytes;
    L->o_buf1 = o;
    o += L->field_bytes;
    L->o_c = o;
    o += L->field_bytes;
    L->o_evptr = o;
    o += align_up((L->ncol + 1) * (int64_t)sizeof(int32_t), 256);
    L->o_ev = o;
    o += align_up(std::max<int64_t>(1, max_src + max_rec) * (int64_t)sizeof(Event), 256);
    L->o_src = o;
    o += align_up(std::max<int64_t>(1, max_src) * (int64_t)sizeof(SourceInfo), 256);
    L->o_damp = o;
    o += align_up((L->knx + L->kny + L->knz) * (int64_t)L->esize, 256);
    L->total = o;
    return true;
}

Geom geom_of(const Layout &L)
{
    Geom g;
    g.nx = L.knx;
    g.ny = L.kny;
    g.nz = L.knz;
    g.px = L.px;
    g.pxy = L.pxy;
    g.off0 = L.off0;
    return g;
}

// ------------------------------------------------------------------ kernel selection

struct Tuning {
    int config;
    int zchunk;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuning> g_tuning;

const FwdEntry *fwd_table(fd_dtype dt, int r, int ndim, int *count)
{
    return dt == FD_F32 ? fwd_configs_f32(r, ndim, count) : fwd_configs_f64(r, ndim, count);
}

const AdjEntry *adj_table(fd_dtype dt, int r, int ndim, int *count)
{
    return dt == FD_F32 ? adj_configs_f32(r, ndim, count) : adj_configs_f64(r, ndim, count);
}
std::map<std::tuple<int, int, int>, int> g_adj_tuning;

// Default z chunks of [kSmallGridZchMin, kSmallGridZchMax) planes select a radius's
// small-grid tile build (measured: 256^3 and 320^3 gain 5-6 %; 512^3 and 400^3, with
// longer chunks, lose 1-3 %; grids of 160^3 and less, with chunks of a few planes, lose
// up to 6 % when batched).
constexpr int kSmallGridZchMin = 16, kSmallGridZchMax = 64;

// Share of a row's tile lanes that fall past its last point when tiles of width bx cover
// nx points.  The adjoint takes its ragged-row build where that share is more than
// kAdjRaggedMargin below the default tile's (measured: 320^3, 192^3 and 160^3 gain 7-17 %
// with the 64-wide tile; 448^3 is even; 400^3, with 11 points of difference, loses 1 %;
// grids whose rows are a multiple of 128 lose 4-5 %).
double row_waste(int64_t nx, int bx)
{
    const int64_t cover = (nx + bx - 1) / bx * bx;
    return 1.0 - (double)nx / (double)cover;
}
constexpr double kAdjRaggedMargin = 0.12;

// The last x tile and its halo (at most 8 points) stay inside the padded row, which
// holds align_up(nx, 256) + 16 points after the interior start: always true of tiles
// whose width divides 256.
bool tile_fits(const FwdEntry &e, const Layout &L)
{
    const int64_t tiles_x = (L.knx + e.bx - 1) / e.bx;
    return tiles_x * e.bx + 8 <= align_up(L.knx, 256) + 16;
}

}  // namespace

namespace fdw {

// Workgroups of kernel k the whole device runs at once (CUs x resident workgroups per
// CU from the occupancy calculator); 512 if the runtime cannot tell.
int resident_slots(const void *kernel, int nt)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 512;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu <= 0)
        return 512;
    return cus * per_cu;
}

// Planes per z chunk.  More chunks mean more workgroups but each chunk re-reads 2r planes
// of u^n (its prologue).  Workgroups run in waves of `slots`; with equal-length
// workgroups a launch costs about ceil(nwg / slots) x (zch + 2r) plane-times, which is
// minimised over the chunk count, down to one plane per chunk: a small grid has few xy
// tiles, and short chunks are what keeps the GPU busy (64^3: 18.5 -> 5.7 us per step).
int choose_zch(int64_t tiles_xy, int64_t nz, int r, int slots)
{
    const int64_t max_chunks = std::max<int64_t>(1, nz);
    int64_t best_c = 1;
    double best = 1e300;
    for (int64_t c = 1; c <= max_chunks; ++c) {
        const int64_t zch = (nz + c - 1) / c;
        const int64_t waves = (tiles_xy * c + slots - 1) / slots;
        const double cost = (double)waves * (double)(zch + 2 * r);
        if (cost < best - 1e-9) {
            best = cost;
            best_c = c;
        }
    }
    return (int)((nz + best_c - 1) / best_c);
}

}  // namespace fdw

// ------------------------------------------------------------------ context

struct SourceRec {
    int64_t pos[3];
    const void *wav;
    int64_t nsamp;
    double amp;
};

struct fd_ctx {
    fd_grid g;
    int r;
    double h, dt;
    fd_dtype dtype;
    fd_bc bc;
    hipStream_t stream;
    Layout L;
    char *ws;
    int64_t max_src, max_rec;
    // kernels
    const FwdEntry *kf;
    const AdjEntry *ka;
    int zch;
    int64_t tiles_x, tiles_y, chunks_z;
    int slots;  // resident workgroups of the forward kernel on the device
    int64_t adj_tiles_x, adj_tiles_y, adj_chunks_z;
    int adj_zch;
    std::string cfg_name;
    std::string adj_cfg_name;
    // host mirrors
    ShotDesc desc;
    std::vector<SourceRec> sources;
    std::vector<int32_t> rec_pos;  // [nrec][3]
    int64_t nrec;
    void *traces;
    int64_t rec_cap, rec_base;
    std::vector<int32_t> h_evptr;
    std::vector<Event> h_ev;
    std::vector<SourceInfo> h_src;
    int64_t step;
    bool poisoned;
    int xcd_remap;
    // two-step forward (temporal blocking): two caller-provided padded fields
    void *aux[2];
    const Fwd2Entry *k2;
    int zch2;
    int64_t tiles2_x, tiles2_y, chunks2_z;

    void *buf(int i) const { return ws + (i == 0 ? L.o_buf0 : L.o_buf1); }
    void *cfield() const { return ws + L.o_c; }
    ShotDesc *d_desc() const { return reinterpret_cast<ShotDesc *>(ws + L.o_desc); }
};

static int check_ctx(const fd_ctx *c)
{
    if (!c) return fail(FD_E_INVAL, "null context");
    if (c->poisoned) return fail(FD_E_STATE, "context is poisoned by an earlier device error");
    return FD_OK;
}

// Rebuild the column-sorted event list and upload it together with the descriptor.
static int upload_tables(fd_ctx *c)
{
    const Layout &L = c->L;
    struct Tmp {
        int64_t col;
        int32_t z, code;
    };
    std::vector<Tmp> all;
    all.reserve(c->sources.size() + (size_t)c->nrec);
    auto colz = [&](const int64_t *p, int64_t *col, int32_t *z) {
        if (L.ndim == 3) {
            *col = p[1] * L.knx + p[0];
            *z = (int32_t)p[2];
        } else {
            *col = p[0];
            *z = (int32_t)p[1];
        }
    };
    c->h_src.clear();
    for (size_t s = 0; s < c->sources.size(); ++s) {
        const SourceRec &sr = c->sources[s];
        Tmp t;
        colz(sr.pos, &t.col, &t.z);
        t.code = ~(int32_t)s;
        all.push_back(t);
        SourceInfo si;
        si.wav = sr.wav;
        si.nsamp = sr.nsamp;
        si.scale = sr.amp * c->dt * c->dt / std::pow(c->h, (double)L.ndim);
        c->h_src.push_back(si);
    }
    for (int64_t j = 0; j < c->nrec; ++j) {
        int64_t p[3] = {c->rec_pos[3 * j], c->rec_pos[3 * j + 1], c->rec_pos[3 * j + 2]};
        Tmp t;
        colz(p, &t.col, &t.z);
        t.code = (int32_t)j;
        all.push_back(t);
    }
    // sources sort before receivers at the same point (negative codes first)
    std::sort(all.begin(), all.end(), [](const Tmp &a, const Tmp &b) {
        if (a.col != b.col) return a.col < b.col;
        if (a.z != b.z) return a.z < b.z;
        return a.code < b.code;
    });
    c->h_ev.resize(all.size());
    c->h_evptr.assign((size_t)L.ncol + 1, 0);
    for (size_t i = 0; i < all.size(); ++i) {
        c->h_ev[i].z = all[i].z;
        c->h_ev[i].code = all[i].code;
        c->h_evptr[(size_t)all[i].col + 1]++;
    }
    for (int64_t i = 0; i < L.ncol; ++i) c->h_evptr[(size_t)i + 1] += c->h_evptr[(size_t)i];

    ShotDesc &d = c->desc;
    const bool any = !all.empty();
    d.ev_ptr = any ? reinterpret_cast<const int32_t *>(c->ws + L.o_evptr) : nullptr;
    d.ev = reinterpret_cast<const Event *>(c->ws + L.o_ev);
    d.src = reinterpret_cast<const SourceInfo *>(c->ws + L.o_src);
    d.traces = c->traces;
    d.nrec = c->nrec;
    d.rec_base = c->rec_base;
    d.rec_cap = c->rec_cap;
    if (any) {
        HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_evptr, c->h_evptr.data(), c->h_evptr.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_ev, c->h_ev.data(), c->h_ev.size() * sizeof(Event),
                                  hipMemcpyHostToDevice, c->stream));
        if (!c->h_src.empty())
            HIP_TRY(c, hipMemcpyAsync(c->ws + L.o_src, c->h_src.data(), c->h_src.size() * sizeof(SourceInfo),
                                      hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_desc(), &c->desc, sizeof(ShotDesc), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FD_OK;
}

// ------------------------------------------------------------------ stencil, limits, planning

extern "C" int fd_weights(int r, double *w)
{
    if (r < 1 || r > 12 || !w) return fail(FD_E_INVAL, "fd_weights: r must be in [1, 12]");
    double s = 0.0;
    for (int l = 1; l <= r; ++l) {
        w[l] = stencil_weight(r, l);
        s += w[l];
    }
    w[0] = -2.0 * s;
    return FD_OK;
}

extern "C" double fd_dt_max(int ndim, int r, double h, double vmax)
{
    if (ndim < 1 || ndim > 3 || r < 1 || r > 8 || !(h > 0) || !(vmax > 0)) return -1.0;
    // S_r = -w0 + 2 sum |w_l|: the 1-D symbol at theta = pi, where it is largest
    double w[9];
    fd_weights(r, w);
    double S = -w[0];
    for (int l = 1; l <= r; ++l) S += 2.0 * std::fabs(w[l]);
    return 2.0 * h / (vmax * std::sqrt((double)ndim * S));
}

extern "C" int fd_field_bytes(const fd_grid *g, int r, fd_dtype dtype, size_t *bytes)
{
    Layout L;
    if (!bytes || !make_layout(g, r, dtype, 0, 0, &L)) return fail(FD_E_INVAL, "fd_field_bytes: bad grid/r/dtype");
    *bytes = L.field_bytes;
    return FD_OK;
}

extern "C" int fd_workspace_bytes(const fd_grid *g, int r, fd_dtype dtype, int64_t max_sources,
                                  int64_t max_receivers, size_t *bytes)
{
    Layout L;
    if (!bytes || !make_layout(g, r, dtype, max_sources, max_receivers, &L))
        return fail(FD_E_INVAL, "fd_workspace_bytes: bad grid/r/dtype/maxima");
    *bytes = L.total;
    return FD_OK;
}

extern "C" int fd_set_tuning(fd_dtype dtype, int r, int ndim, int config, int zchunk)
{
    int count = 0;
    if ((dtype != FD_F32 && dtype != FD_F64) || r < 1 || r > 8 || (ndim != 2 && ndim != 3))
        return fail(FD_E_INVAL, "fd_set_tuning: bad dtype/r/ndim");
    fwd_table(dtype, r, ndim, &count);
    if (config < -1 || config >= count) return fail(FD_E_RANGE, "fd_set_tuning: config %d of %d", config, count);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (config == -1)
        g_tuning.erase(std::make_tuple((int)dtype, r, ndim));  // back to the library's own choice
    else
        g_tuning[std::make_tuple((int)dtype, r, ndim)] = Tuning{config, zchunk};
    return FD_OK;
}

// ------------------------------------------------------------------ lifecycle

extern "C" int fd_set_adj_tuning(fd_dtype dtype, int r, int ndim, int config)
{
    int count = 0;
    const AdjEntry *tab = (dtype == FD_F32 || dtype == FD_F64) ? adj_table(dtype, r, ndim, &count) : nullptr;
    if (!tab || count == 0) return fail(FD_E_INVAL, "fd_set_adj_tuning: bad dtype/r/ndim");
    if (config < -1 || config >= count) return fail(FD_E_RANGE, "fd_set_adj_tuning: config %d of %d", config, count);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (config < 0)
        g_adj_tuning.erase(std::make_tuple((int)dtype, r, ndim));
    else
        g_adj_tuning[std::make_tuple((int)dtype, r, ndim)] = config;
    return FD_OK;
}

extern "C" int fd_create(fd_ctx **out, const fd_grid *g, int r, double h, double dt, const void *velocity,
                         fd_dtype dtype, fd_bc bc, void *workspace, size_t ws_bytes, int64_t max_sources,
                         int64_t max_receivers, void *stream)
{
    if (!out) return fail(FD_E_INVAL, "fd_create: null out");
    *out = nullptr;
    Layout L;
    if (!make_layout(g, r, dtype, max_sources, max_receivers, &L))
        return fail(FD_E_INVAL, "fd_create: bad grid (ndim 2/3, n >= 1, nz = 1 in 2-D), r in [1,8], dtype or maxima");
    if (!(h > 0) || !(dt > 0) || !std::isfinite(h) || !std::isfinite(dt))
        return fail(FD_E_INVAL, "fd_create: h and dt must be positive");
    if (bc != FD_BC_ZERO && bc != FD_BC_PERIODIC) return fail(FD_E_INVAL, "fd_create: bad boundary");
    if (!velocity || !workspace) return fail(FD_E_INVAL, "fd_create: null velocity or workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(FD_E_INVAL, "fd_create: workspace not 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(FD_E_NOMEM, "fd_create: workspace %zu bytes < %zu needed", ws_bytes, L.total);
    if (bc == FD_BC_PERIODIC) {
        const int64_t ext[3] = {L.knx, L.kny, L.knz};
        for (int a = 0; a < 3; ++a)
            if ((a != 1 || L.ndim == 3) && ext[a] < r)
                return fail(FD_E_INVAL, "fd_create: periodic grid must have at least r points per axis");
    }

    int count = 0, acount = 0;
    const FwdEntry *tab = fwd_table(dtype, r, g->ndim, &count);
    const AdjEntry *atab = adj_table(dtype, r, g->ndim, &acount);
    if (!tab || count == 0 || !atab || acount == 0) return fail(FD_E_INVAL, "fd_create: no kernel for this dtype/r/ndim");
    Tuning tu{0, 0};
    bool tuned = false;
    int acfg = -1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuning.find(std::make_tuple((int)dtype, r, (int)g->ndim));
        if (it != g_tuning.end()) {
            tu = it->second;
            tuned = true;
        }
        auto ia = g_adj_tuning.find(std::make_tuple((int)dtype, r, (int)g->ndim));
        if (ia != g_adj_tuning.end()) acfg = ia->second;
    }
    if (acfg < 0) {
        // The library's own adjoint tile: the default, or its ragged-row build (a narrower
        // tile) where a grid row leaves clearly more of the default tile's lanes idle.
        acfg = 0;
        for (int i = 1; i < acount; ++i)
            if (atab[i].role == ADJ_RAGGED_X) {
                if (row_waste(L.knx, atab[i].bx) + kAdjRaggedMargin < row_waste(L.knx, atab[0].bx)) acfg = i;
                break;
            }
    }
    const AdjEntry *ka = &atab[acfg];

    if (!tile_fits(tab[tu.config], L))
        return fail(FD_E_INVAL, "fd_create: tile %s does not fit a row of %lld points", tab[tu.config].name,
                    (long long)L.knx);
    if (!tuned) {
        // The library's own choice: the default tile, or its small-grid build (more resident
        // waves) where the default's z chunks are short but not tiny, i.e. where
        // workgroups are many and brief and latency rather than streaming sets the pace.
        const FwdEntry &d = tab[0];
        const int64_t txy = ((L.knx + d.bx - 1) / d.bx) * ((L.kny + d.by - 1) / d.by);
        const int zd = choose_zch(txy, L.knz, r, resident_slots(d.kernel, d.nt));
        if (zd >= kSmallGridZchMin && zd < kSmallGridZchMax)
            for (int i = 1; i < count; ++i)
                if (tab[i].role == FWD_SMALL_GRID && tile_fits(tab[i], L)) {
                    tu.config = i;
                    break;
                }
    }

    fd_ctx *c = new fd_ctx();
    c->g = *g;
    c->r = r;
    c->h = h;
    c->dt = dt;
    c->dtype = dtype;
    c->bc = bc;
    c->stream = (hipStream_t)stream;
    c->L = L;
    c->ws = (char *)workspace;
    c->max_src = max_sources;
    c->max_rec = max_receivers;
    c->kf = &tab[tu.config];
    c->ka = ka;
    c->tiles_x = (L.knx + c->kf->bx - 1) / c->kf->bx;
    c->tiles_y = (L.kny + c->kf->by - 1) / c->kf->by;
    c->slots = resident_slots(c->kf->kernel, c->kf->nt);
    c->zch = tu.zchunk > 0 ? (int)std::min<int64_t>(tu.zchunk, L.knz)
                           : choose_zch(c->tiles_x * c->tiles_y, L.knz, r, c->slots);
    c->chunks_z = (L.knz + c->zch - 1) / c->zch;
    c->adj_tiles_x = (L.knx + ka->bx - 1) / ka->bx;
    c->adj_tiles_y = (L.kny + ka->by - 1) / ka->by;
    c->adj_zch = choose_zch(c->adj_tiles_x * c->adj_tiles_y, L.knz, r, resident_slots(ka->kernel, ka->nt));
    c->adj_chunks_z = (L.knz + c->adj_zch - 1) / c->adj_zch;
    c->nrec = 0;
    c->traces = nullptr;
    c->rec_cap = 0;
    c->rec_base = 0;
    c->step = 0;
    c->poisoned = false;
    c->xcd_remap = 1;
    char nm[256];
    snprintf(nm, sizeof(nm), "%s, zchunk %d, grid %lld wg", c->kf->name, c->zch,
             (long long)(c->tiles_x * c->tiles_y * c->chunks_z));
    c->cfg_name = nm;
    snprintf(nm, sizeof(nm), "%s, zchunk %d, grid %lld wg", c->ka->name, c->adj_zch,
             (long long)(c->adj_tiles_x * c->adj_tiles_y * c->adj_chunks_z));
    c->adj_cfg_name = nm;

    // zero the workspace: both wavefields (u^0 = u^-1 = 0), c ghosts, tables
    hipError_t e = hipMemsetAsync(workspace, 0, L.total, c->stream);
    if (e == hipSuccess) {
        const double k = (dt / h) * (dt / h);
        e = launch_prep((int)dtype, geom_of(L), velocity, c->cfield(), k, (double *)(c->ws + L.o_partial),
                        (double *)(c->ws + L.o_minmax), c->stream);
    }
    double mm[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(mm, c->ws + L.o_minmax, sizeof(mm), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(FD_E_DEVICE, "fd_create: %s", hipGetErrorString(e));
    }
    if (!(mm[0] > 0) || !std::isfinite(mm[1])) {
        delete c;
        return fail(FD_E_INVAL, "fd_create: velocity must be finite and positive (min %g, max %g)", mm[0], mm[1]);
    }
    const double dtm = fd_dt_max(g->ndim, r, h, mm[1]);
    if (dt > dtm) {
        delete c;
        return fail(FD_E_UNSTABLE, "fd_create: dt %.6g exceeds the stability limit %.6g for vmax %.6g", dt, dtm, mm[1]);
    }

    ShotDesc &d = c->desc;
    std::memset(&d, 0, sizeof(d));
    d.buf[0] = c->buf(0);
    d.buf[1] = c->buf(1);
    d.c = c->cfield();
    d.nx = (int32_t)L.knx;
    d.ny = (int32_t)L.kny;
    d.nz = (int32_t)L.knz;
    d.tiles_x = (int32_t)c->tiles_x;
    d.tiles_y = (int32_t)c->tiles_y;
    d.chunks_z = (int32_t)c->chunks_z;
    d.zch = c->zch;
    d.px = L.px;
    d.pxy = L.pxy;
    d.off0 = L.off0;
    d.ctr[0] = 0;
    d.ctr[1] = 0;
    d.target = 0;
    int st = upload_tables(c);
    if (st != FD_OK) {
        delete c;
        return st;
    }
    *out = c;
    return FD_OK;
}

extern "C" int fd_destroy(fd_ctx *ctx)
{
    if (!ctx) return fail(FD_E_INVAL, "fd_destroy: null context");
    if (!ctx->poisoned) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return FD_OK;
}

extern "C" int fd_set_stream(fd_ctx *ctx, void *stream)
{
    int st = check_ctx(ctx);
    if (st) return st;
    ctx->stream = (hipStream_t)stream;
    return FD_OK;
}

extern "C" const char *fd_kernel_config(const fd_ctx *ctx) { return ctx ? ctx->cfg_name.c_str() : ""; }
extern "C" const char *fd_adjoint_config(const fd_ctx *ctx) { return ctx ? ctx->adj_cfg_name.c_str() : ""; }

// ------------------------------------------------------------------ sources and receivers

static bool in_grid(const fd_ctx *c, const int64_t *p)
{
    const int nd = c->L.ndim;
    for (int a = 0; a < nd; ++a)
        if (p[a] < 0 || p[a] >= c->g.n[a]) return false;
    return true;
}

extern "C" int fd_inject(fd_ctx *ctx, const void *wavelet, int64_t nsamp, const int64_t pos[3], double amp)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!pos || nsamp < 0 || (nsamp > 0 && !wavelet) || !std::isfinite(amp))
        return fail(FD_E_INVAL, "fd_inject: bad wavelet, nsamp or amp");
    int64_t p[3] = {pos[0], pos[1], ctx->L.ndim == 3 ? pos[2] : 0};
    if (!in_grid(ctx, p)) return fail(FD_E_RANGE, "fd_inject: position (%lld, %lld, %lld) outside the grid",
                                      (long long)p[0], (long long)p[1], (long long)p[2]);
    if ((int64_t)ctx->sources.size() >= ctx->max_src)
        return fail(FD_E_RANGE, "fd_inject: more than max_sources = %lld", (long long)ctx->max_src);
    SourceRec sr;
    std::memcpy(sr.pos, p, sizeof(p));
    sr.wav = wavelet;
    sr.nsamp = nsamp;
    sr.amp = amp;
    ctx->sources.push_back(sr);
    return upload_tables(ctx);
}

extern "C" int fd_clear_sources(fd_ctx *ctx)
{
    int st = check_ctx(ctx);
    if (st) return st;
    ctx->sources.clear();
    return upload_tables(ctx);
}

// Cerjan sponge factors along one axis of n points (distance i from a damped face,
// i < width: exp(-(alpha (width - i))^2); overlapping strips multiply).
static void sponge_profile(int64_t n, int width, double alpha, bool lo, bool hi, double *g)
{
    for (int64_t i = 0; i < n; ++i) g[i] = 1.0;
    for (int64_t i = 0; i < std::min<int64_t>(width, n); ++i) {
        const double a = alpha * (double)(width - i);
        const double f = std::exp(-a * a);
        if (lo) g[i] *= f;
        if (hi) g[n - 1 - i] *= f;
    }
}

extern "C" int fd_set_damping(fd_ctx *ctx, int width, double alpha, int faces)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (width < 0 || !(alpha >= 0) || !std::isfinite(alpha) || faces < 0 || faces > 63)
        return fail(FD_E_INVAL, "fd_set_damping: width >= 0, alpha >= 0, faces a 6-bit mask");
    if (ctx->bc != FD_BC_ZERO && width > 0) return fail(FD_E_STATE, "fd_set_damping: zero boundary only");
    const Layout &L = ctx->L;
    if (width == 0 || faces == 0) {
        ctx->desc.damp = nullptr;
    } else {
        // grid faces -> kernel axes: a 2-D grid's y is the kernel's z, the kernel y is unit
        const bool nd3 = L.ndim == 3;
        const int fz = nd3 ? (faces >> 4) & 3 : (faces >> 2) & 3;
        const int fy = nd3 ? (faces >> 2) & 3 : 0;
        std::vector<double> g((size_t)(L.knx + L.kny + L.knz));
        sponge_profile(L.knx, width, alpha, faces & 1, faces & 2, g.data());
        sponge_profile(L.kny, fy ? width : 0, alpha, fy & 1, fy & 2, g.data() + L.knx);
        sponge_profile(L.knz, width, alpha, fz & 1, fz & 2, g.data() + L.knx + L.kny);
        std::vector<float> gf;
        if (ctx->dtype == FD_F32) gf.assign(g.begin(), g.end());
        HIP_TRY(ctx, hipMemcpyAsync(ctx->ws + L.o_damp, ctx->dtype == FD_F32 ? (const void *)gf.data() : g.data(),
                                    g.size() * L.esize, hipMemcpyHostToDevice, ctx->stream));
        ctx->desc.damp = ctx->ws + L.o_damp;
    }
    return upload_tables(ctx);
}

extern "C" int fd_record(fd_ctx *ctx, const int32_t *pos, int64_t nrec, void *traces, int64_t cap)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (nrec < 0 || (nrec > 0 && (!pos || !traces || cap < 0)))
        return fail(FD_E_INVAL, "fd_record: bad receiver arguments");
    if (nrec > ctx->max_rec)
        return fail(FD_E_RANGE, "fd_record: %lld receivers > max_receivers = %lld", (long long)nrec, (long long)ctx->max_rec);
    std::vector<int32_t> rp((size_t)nrec * 3);
    for (int64_t j = 0; j < nrec; ++j) {
        int64_t p[3] = {pos[3 * j], pos[3 * j + 1], ctx->L.ndim == 3 ? pos[3 * j + 2] : 0};
        if (!in_grid(ctx, p)) return fail(FD_E_RANGE, "fd_record: receiver %lld outside the grid", (long long)j);
        rp[3 * j] = (int32_t)p[0];
        rp[3 * j + 1] = (int32_t)p[1];
        rp[3 * j + 2] = (int32_t)p[2];
    }
    ctx->rec_pos.swap(rp);
    ctx->nrec = nrec;
    ctx->traces = nrec > 0 ? traces : nullptr;
    ctx->rec_cap = nrec > 0 ? cap : 0;
    ctx->rec_base = ctx->step;
    return upload_tables(ctx);
}

extern "C" int fd_ricker(void *out, int64_t nsamp, double dt, double f0, double t0, fd_dtype dtype, void *stream)
{
    if (nsamp < 0 || (nsamp > 0 && !out) || !(dt > 0) || !(f0 > 0) || (dtype != FD_F32 && dtype != FD_F64))
        return fail(FD_E_INVAL, "fd_ricker: bad arguments");
    hipError_t e = launch_ricker((int)dtype, out, nsamp, dt, f0, t0, (hipStream_t)stream);
    if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_ricker: %s", hipGetErrorString(e));
    return FD_OK;
}

// ------------------------------------------------------------------ stepping

static LaunchArgs direct_args(const fd_ctx *c, int64_t step)
{
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.shots = c->d_desc();
    a.wg_prefix = nullptr;
    a.nshots = 1;
    a.slot = 0;
    a.step = step;
    a.record = 1;
    a.xcd_remap = c->xcd_remap;
    return a;
}

static int64_t nwg_of(const fd_ctx *c) { return c->tiles_x * c->tiles_y * c->chunks_z; }

static void launch_two_step(fd_ctx *c, const void *cur, const void *prev, void *out1, void *out2, int64_t step)
{
    Fwd2Args a;
    std::memset(&a, 0, sizeof(a));
    a.shot = c->d_desc();
    a.cur = cur;
    a.prev = prev;
    a.out1 = out1;
    a.out2 = out2;
    a.step = step;
    a.zch = c->zch2;
    a.tiles_x = (int32_t)c->tiles2_x;
    a.tiles_y = (int32_t)c->tiles2_y;
    a.chunks_z = (int32_t)c->chunks2_z;
    a.xcd_remap = c->xcd_remap;
    c->k2->launch(a, (int)(c->tiles2_x * c->tiles2_y * c->chunks2_z), c->stream);
}

extern "C" int fd_set_time_blocking(fd_ctx *ctx, void *aux, size_t aux_bytes, int config)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!aux) {
        ctx->aux[0] = ctx->aux[1] = nullptr;
        ctx->k2 = nullptr;
        return FD_OK;
    }
    const Layout &L = ctx->L;
    int count = 0;
    const Fwd2Entry *tab = (L.ndim == 3 && ctx->dtype == FD_F32) ? fwd2_configs_f32(ctx->r, &count) : nullptr;
    if (!tab || count == 0) return fail(FD_E_INVAL, "fd_set_time_blocking: no two-step kernel for this dtype/r/ndim");
    if (config < 0 || config >= count) return fail(FD_E_RANGE, "fd_set_time_blocking: config %d of %d", config, count);
    if (reinterpret_cast<uintptr_t>(aux) % 256 != 0) return fail(FD_E_INVAL, "fd_set_time_blocking: aux not 256-byte aligned");
    if (aux_bytes < 2 * L.field_bytes)
        return fail(FD_E_NOMEM, "fd_set_time_blocking: aux %zu bytes < %zu needed", aux_bytes, 2 * L.field_bytes);
    // the kernel writes interiors only: ghosts and padding of the extra fields stay zero
    HIP_TRY(ctx, hipMemsetAsync(aux, 0, 2 * L.field_bytes, ctx->stream));
    ctx->aux[0] = aux;
    ctx->aux[1] = (char *)aux + L.field_bytes;
    ctx->k2 = &tab[config];
    ctx->tiles2_x = (L.knx + ctx->k2->bx - 1) / ctx->k2->bx;
    ctx->tiles2_y = (L.kny + ctx->k2->by - 1) / ctx->k2->by;
    ctx->zch2 = choose_zch(ctx->tiles2_x * ctx->tiles2_y, L.knz, ctx->r, resident_slots(ctx->k2->kernel, ctx->k2->nt));
    ctx->chunks2_z = (L.knz + ctx->zch2 - 1) / ctx->zch2;
    return FD_OK;
}

extern "C" int fd_step(fd_ctx *ctx, int64_t nsteps)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (nsteps < 0) return fail(FD_E_INVAL, "fd_step: negative nsteps");
    if (nsteps == 0) return FD_OK;
    if (ctx->nrec > 0 && ctx->step + nsteps - ctx->rec_base > ctx->rec_cap)
        return fail(FD_E_RANGE, "fd_step: trace capacity %lld exceeded (step %lld + %lld, recording from %lld)",
                    (long long)ctx->rec_cap, (long long)ctx->step, (long long)nsteps, (long long)ctx->rec_base);
    const int64_t nwg = nwg_of(ctx);
    const Geom gm = geom_of(ctx->L);
    int64_t i = 0;
    if (ctx->k2 && ctx->bc == FD_BC_ZERO && !ctx->desc.damp) {
        // pairs of two-step launches: (u^n, u^{n-1}) -> aux -> back into the two context
        // fields with their usual roles, so every other call sees the usual layout
        for (; i + 4 <= nsteps; i += 4) {
            const int64_t n = ctx->step;
            launch_two_step(ctx, ctx->buf((int)(n & 1)), ctx->buf((int)((n + 1) & 1)), ctx->aux[0], ctx->aux[1], n);
            HIP_TRY(ctx, hipGetLastError());
            launch_two_step(ctx, ctx->aux[1], ctx->aux[0], ctx->buf((int)((n + 3) & 1)), ctx->buf((int)(n & 1)), n + 2);
            HIP_TRY(ctx, hipGetLastError());
            ctx->step += 4;
        }
    }
    for (; i < nsteps; ++i) {
        if (ctx->bc == FD_BC_PERIODIC)
            HIP_TRY(ctx, launch_halo_periodic((int)ctx->dtype, gm, ctx->r, ctx->L.ndim == 3 ? ctx->r : 0, ctx->r,
                                              ctx->buf((int)(ctx->step & 1)), ctx->stream));
        LaunchArgs a = direct_args(ctx, ctx->step);
        ctx->kf->launch(a, (int)nwg, ctx->stream);
        HIP_TRY(ctx, hipGetLastError());
        ctx->step++;
    }
    return FD_OK;
}

extern "C" int fd_sync(fd_ctx *ctx)
{
    if (!ctx) return fail(FD_E_INVAL, "fd_sync: null context");
    if (ctx->poisoned) return fail(FD_E_STATE, "context is poisoned");
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipGetLastError());
    return FD_OK;
}

extern "C" int fd_check_finite(fd_ctx *ctx, int *finite)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!finite) return fail(FD_E_INVAL, "fd_check_finite: null result pointer");
    const int64_t n = (int64_t)(ctx->L.field_bytes / ctx->L.esize);
    double *out = reinterpret_cast<double *>(ctx->ws + ctx->L.o_minmax);
    HIP_TRY(ctx, launch_nonfinite((int)ctx->dtype, ctx->buf(0), ctx->buf(1), n,
                                  reinterpret_cast<double *>(ctx->ws + ctx->L.o_partial), out, ctx->stream));
    double flag[2] = {0.0, 0.0};
    HIP_TRY(ctx, hipMemcpyAsync(flag, out, sizeof(flag), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *finite = flag[1] == 0.0 ? 1 : 0;
    return FD_OK;
}

extern "C" int fd_get_step(const fd_ctx *ctx, int64_t *step)
{
    if (!ctx || !step) return fail(FD_E_INVAL, "fd_get_step: null argument");
    *step = ctx->step;
    return FD_OK;
}

extern "C" int fd_get_state(fd_ctx *ctx, void *u_cur, void *u_prev, int64_t *step, fd_layout layout)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (layout != FD_DENSE && layout != FD_PADDED) return fail(FD_E_INVAL, "fd_get_state: bad layout");
    void *dst[2] = {u_cur, u_prev};
    const int src[2] = {(int)(ctx->step & 1), (int)((ctx->step + 1) & 1)};
    for (int i = 0; i < 2; ++i) {
        if (!dst[i]) continue;
        if (layout == FD_PADDED)
            HIP_TRY(ctx, hipMemcpyAsync(dst[i], ctx->buf(src[i]), ctx->L.field_bytes, hipMemcpyDeviceToDevice, ctx->stream));
        else
            HIP_TRY(ctx, launch_pack((int)ctx->dtype, geom_of(ctx->L), ctx->buf(src[i]), dst[i], ctx->stream));
    }
    if (step) *step = ctx->step;
    return FD_OK;
}

extern "C" int fd_set_state(fd_ctx *ctx, const void *u_cur, const void *u_prev, int64_t step, fd_layout layout)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (layout != FD_DENSE && layout != FD_PADDED) return fail(FD_E_INVAL, "fd_set_state: bad layout");
    if (step < 0) return fail(FD_E_INVAL, "fd_set_state: negative step");
    const void *srcp[2] = {u_cur, u_prev};
    const int dst[2] = {(int)(step & 1), (int)((step + 1) & 1)};
    // a new step parity may move the roles of the two buffers: copy both before use
    for (int i = 0; i < 2; ++i) {
        if (!srcp[i]) continue;
        if (layout == FD_PADDED)
            HIP_TRY(ctx, hipMemcpyAsync(ctx->buf(dst[i]), srcp[i], ctx->L.field_bytes, hipMemcpyDeviceToDevice, ctx->stream));
        else
            HIP_TRY(ctx, launch_unpack((int)ctx->dtype, geom_of(ctx->L), srcp[i], ctx->buf(dst[i]), ctx->stream));
    }
    ctx->step = step;
    return FD_OK;
}

static int step_explicit(fd_ctx *ctx, const void *cur, const void *prev, void *out, int64_t step, int record,
                         const char *who)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!cur || !prev || !out || step < 0) return fail(FD_E_INVAL, "%s: bad arguments", who);
    if (out == cur) return fail(FD_E_INVAL, "%s: out must not alias cur", who);
    if (ctx->bc != FD_BC_ZERO) return fail(FD_E_STATE, "%s: zero boundary only", who);
    LaunchArgs a = direct_args(ctx, step);
    a.cur = cur;
    a.prev = prev;
    a.out = out;
    a.record = record;
    ctx->kf->launch(a, (int)nwg_of(ctx), ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return FD_OK;
}

extern "C" int fd_step_explicit(fd_ctx *ctx, const void *cur, const void *prev, void *out, int64_t step)
{
    return step_explicit(ctx, cur, prev, out, step, 0, "fd_step_explicit");
}

extern "C" int fd_step_record(fd_ctx *ctx, const void *cur, const void *prev, void *out, int64_t step)
{
    return step_explicit(ctx, cur, prev, out, step, 1, "fd_step_record");
}

// ------------------------------------------------------------------ adjoint

template <class Slot>
static int adjoint_steps(fd_ctx *ctx, const Slot &slot, int64_t k_lo, int64_t k_hi, void *mu, const void *resid,
                         double resid_amp, void *grad, void *grad_seg);

extern "C" int fd_adjoint_segment(fd_ctx *ctx, const void *u_ckpt_cur, const void *u_ckpt_prev, int64_t k_lo,
                                  int64_t k_hi, void *ring, void *mu, const void *resid, double resid_amp, void *grad,
                                  void *grad_seg)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (ctx->bc != FD_BC_ZERO) return fail(FD_E_STATE, "fd_adjoint_segment: zero boundary only");
    if (ctx->desc.damp) return fail(FD_E_STATE, "fd_adjoint_segment: the adjoint of the damped scheme is not built");
    const int64_t nk = k_hi - k_lo;
    if (k_lo < 0 || nk < 1 || !u_ckpt_cur || !u_ckpt_prev || !mu || !grad || (nk > 1 && !ring))
        return fail(FD_E_INVAL, "fd_adjoint_segment: bad arguments");
    if (ctx->nrec > 0 && !resid) return fail(FD_E_INVAL, "fd_adjoint_segment: null residual");
    const size_t fb = ctx->L.field_bytes;
    auto slot = [&](int64_t i) -> void * {  // u^{k_lo + i}
        return i == 0 ? const_cast<void *>(u_ckpt_cur) : (char *)ring + (size_t)(i - 1) * fb;
    };
    // recompute u^{k_lo+1} .. u^{k_hi-1} from the checkpoint into the ring
    for (int64_t i = 1; i < nk; ++i) {
        const void *prev = (i == 1) ? u_ckpt_prev : slot(i - 2);
        int s2 = fd_step_explicit(ctx, slot(i - 1), prev, slot(i), k_lo + i - 1);
        if (s2) return s2;
    }
    return adjoint_steps(ctx, slot, k_lo, k_hi, mu, resid, resid_amp, grad, grad_seg);
}

extern "C" int fd_adjoint_stored(fd_ctx *ctx, const void *states, int64_t k_lo, int64_t k_hi, void *mu,
                                 const void *resid, double resid_amp, void *grad, void *grad_seg)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (ctx->bc != FD_BC_ZERO) return fail(FD_E_STATE, "fd_adjoint_stored: zero boundary only");
    if (ctx->desc.damp) return fail(FD_E_STATE, "fd_adjoint_stored: the adjoint of the damped scheme is not built");
    if (k_lo < 0 || k_hi - k_lo < 1 || !states || !mu || !grad)
        return fail(FD_E_INVAL, "fd_adjoint_stored: bad arguments");
    if (ctx->nrec > 0 && !resid) return fail(FD_E_INVAL, "fd_adjoint_stored: null residual");
    const size_t fb = ctx->L.field_bytes;
    auto slot = [&](int64_t i) -> void * {  // u^{k_lo + i}
        return const_cast<char *>(static_cast<const char *>(states)) + (size_t)i * fb;
    };
    return adjoint_steps(ctx, slot, k_lo, k_hi, mu, resid, resid_amp, grad, grad_seg);
}

// Adjoint steps k = k_hi .. k_lo + 1, u^{k-1} taken from slot(k - 1 - k_lo).
template <class Slot>
static int adjoint_steps(fd_ctx *ctx, const Slot &slot, int64_t k_lo, int64_t k_hi, void *mu, const void *resid,
                         double resid_amp, void *grad, void *grad_seg)
{
    const size_t fb = ctx->L.field_bytes;
    const int64_t nk = k_hi - k_lo;
    void *m[2] = {mu, (char *)mu + fb};
    const int64_t nwg = ctx->adj_tiles_x * ctx->adj_tiles_y * ctx->adj_chunks_z;
    for (int64_t k = k_hi; k > k_lo; --k) {
        AdjArgs a;
        std::memset(&a, 0, sizeof(a));
        a.shot = ctx->d_desc();
        a.mu_cur = m[(k + 1) & 1];
        a.mu_out = m[k & 1];
        a.u_km1 = slot(k - 1 - k_lo);
        a.grad = grad;
        a.gseg = grad_seg;
        if (!grad_seg || nk == 1)
            a.gmode = GM_DIRECT;
        else
            a.gmode = (k == k_hi) ? GM_FIRST : (k == k_lo + 1 ? GM_FOLD : GM_ACC);
        a.resid = resid;
        a.k = k;
        a.resid_amp = resid_amp;
        a.xcd_remap = ctx->xcd_remap;
        a.zch = ctx->adj_zch;
        a.tiles_x = (int32_t)ctx->adj_tiles_x;
        a.tiles_y = (int32_t)ctx->adj_tiles_y;
        a.chunks_z = (int32_t)ctx->adj_chunks_z;
        ctx->ka->launch(a, (int)nwg, ctx->stream);
        HIP_TRY(ctx, hipGetLastError());
    }
    return FD_OK;
}

extern "C" int fd_clear_ghosts(fd_ctx *ctx, void *fields, int64_t count)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!fields || count < 0) return fail(FD_E_INVAL, "fd_clear_ghosts: bad arguments");
    if (count == 0) return FD_OK;
    const Layout &L = ctx->L;
    GhostBox b;
    b.count = count;
    b.field_elems = (int64_t)(L.field_bytes / (size_t)L.esize);
    b.px = L.px;
    b.py = L.py;
    b.planes = L.planes;
    b.y0 = L.ndim == 3 ? L.r : 0;
    b.z0 = L.r;
    b.x0 = L.off0 - b.z0 * L.pxy - b.y0 * L.px;
    b.nx = L.knx;
    b.ny = L.kny;
    b.nz = L.knz;
    HIP_TRY(ctx, launch_clear_ghosts((int)ctx->dtype, b, fields, ctx->stream));
    return FD_OK;
}

extern "C" int fd_gradient_finish(fd_ctx *ctx, const void *grad_padded, const void *velocity, void *out, double scale)
{
    int st = check_ctx(ctx);
    if (st) return st;
    if (!grad_padded || !velocity || !out) return fail(FD_E_INVAL, "fd_gradient_finish: null pointer");
    HIP_TRY(ctx, launch_grad_finish((int)ctx->dtype, geom_of(ctx->L), grad_padded, velocity, out, scale, ctx->stream));
    return FD_OK;
}

// ------------------------------------------------------------------ batched serving

struct fd_batch {
    int max_shots;
    char *ws;
    hipStream_t stream;
    hipStream_t cap_stream;
    hipEvent_t order_ev;  // orders member streams and the batch stream (no timing)
    std::vector<fd_ctx *> members;
    std::vector<int64_t> target;
    std::vector<ShotDesc> h_desc;
    std::vector<int32_t> h_prefix;
    int64_t nwg;
    int slot;
    const FwdEntry *kf;
    hipGraphExec_t exec;
    int64_t exec_len;
    bool has_exec;
    // no-allocation batch: the shot table is the device's fixed array, every member runs
    // on the batch stream, and steps are launched directly (no graph, no capture stream)
    bool noalloc;
    int device;

    ShotDesc *d_desc() const { return reinterpret_cast<ShotDesc *>(ws); }
    int32_t *d_prefix() const { return reinterpret_cast<int32_t *>(ws + align_up((int64_t)max_shots * sizeof(ShotDesc), 256)); }
};

static constexpr int64_t batch_table_bytes(int max_shots)
{
    return ((int64_t)max_shots * (int64_t)sizeof(ShotDesc) + 255) / 256 * 256 +
           ((int64_t)(max_shots + 1) * (int64_t)sizeof(int32_t) + 255) / 256 * 256;
}

extern "C" size_t fd_batch_workspace_bytes(int max_shots)
{
    if (max_shots < 1) return 0;
    return (size_t)batch_table_bytes(max_shots);
}

extern "C" int fd_batch_create(fd_batch **out, int max_shots, void *workspace, size_t ws_bytes, void *stream)
{
    if (!out || max_shots < 1 || !workspace) return fail(FD_E_INVAL, "fd_batch_create: bad arguments");
    if (ws_bytes < fd_batch_workspace_bytes(max_shots)) return fail(FD_E_NOMEM, "fd_batch_create: workspace too small");
    fd_batch *b = new fd_batch();
    b->max_shots = max_shots;
    b->ws = (char *)workspace;
    b->stream = (hipStream_t)stream;
    b->nwg = 0;
    b->slot = 0;
    b->kf = nullptr;
    b->has_exec = false;
    b->exec_len = 0;
    b->noalloc = false;
    b->device = -1;
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return fail(FD_E_DEVICE, "fd_batch_create: %s", hipGetErrorString(e));
    }
    e = hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(b->cap_stream);
        delete b;
        return fail(FD_E_DEVICE, "fd_batch_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return FD_OK;
}

// ------------------------------------------------------------------ batch without allocation

// The shot table (descriptors + workgroup prefix) of the no-allocation batch.  Each GPU
// holds its own copy for the life of the process.  Host code never uses this name as an
// address (on the host it is a stand-in symbol): it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device below.
static __device__ __align__(256) char scratch[batch_table_bytes(FD_BATCH_NOALLOC_MAX_SHOTS)];

namespace {
constexpr int kMaxDevices = 64;
struct NoallocSlot {
    char *ptr = nullptr;     // device address of `scratch` on this device (once resolved)
    bool in_use = false;     // held by a live no-allocation batch
    fd_batch batch;          // the handle fd_batch_create_noalloc returns on this device
};
std::mutex g_noalloc_mu;
NoallocSlot g_noalloc[kMaxDevices];
}  // namespace

extern "C" int fd_batch_create_noalloc(fd_batch **out, int max_shots, void *stream)
{
    if (!out) return fail(FD_E_INVAL, "fd_batch_create_noalloc: null out");
    if (max_shots < 1 || max_shots > FD_BATCH_NOALLOC_MAX_SHOTS)
        return fail(FD_E_RANGE, "fd_batch_create_noalloc: max_shots %d outside [1, %d] (the fixed shot table's size)",
                    max_shots, FD_BATCH_NOALLOC_MAX_SHOTS);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_create_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(FD_E_RANGE, "fd_batch_create_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoallocSlot &sl = g_noalloc[dev];
    if (sl.in_use)
        return fail(FD_E_STATE, "fd_batch_create_noalloc: device %d's fixed shot table is held by another batch "
                                "(fd_batch_destroy it first)", dev);
    if (!sl.ptr) {  // first use on this device (it is current): resolve the array's device address
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FD_E_DEVICE, "fd_batch_create_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        sl.ptr = static_cast<char *>(p);
    }
    fd_batch *b = &sl.batch;
    b->max_shots = max_shots;
    b->ws = sl.ptr;
    b->stream = (hipStream_t)stream;
    b->cap_stream = nullptr;
    b->order_ev = nullptr;
    b->members.clear();
    b->target.clear();
    b->h_desc.clear();
    b->h_prefix.clear();
    b->nwg = 0;
    b->slot = 0;
    b->kf = nullptr;
    b->has_exec = false;
    b->exec_len = 0;
    b->noalloc = true;
    b->device = dev;
    sl.in_use = true;
    *out = b;
    return FD_OK;
}

static void batch_drop_graph(fd_batch *b)
{
    if (b->has_exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->has_exec = false;
    }
}

extern "C" int fd_batch_destroy(fd_batch *b)
{
    if (!b) return fail(FD_E_INVAL, "fd_batch_destroy: null batch");
    (void)hipStreamSynchronize(b->stream);
    if (b->noalloc) {  // the device's fixed handle: release the shot table for the next batch
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        b->members.clear();
        b->target.clear();
        b->nwg = 0;
        g_noalloc[b->device].in_use = false;
        return FD_OK;
    }
    batch_drop_graph(b);
    (void)hipEventDestroy(b->order_ev);
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return FD_OK;
}

// Validate a member set and build its shot table: descriptors with both step-counter
// slots at the member's step, the member's target and the batch's z chunking, plus the
// workgroup prefix.
static int batch_table(fd_ctx *const *ctxs, const int64_t *target, int nctx, const char *who,
                       std::vector<ShotDesc> &desc, std::vector<int32_t> &prefix, const FwdEntry **kf_out)
{
    const FwdEntry *kf = nullptr;
    bool mixed = false;
    for (int i = 0; i < nctx; ++i) {
        fd_ctx *c = ctxs[i];
        int st = check_ctx(c);
        if (st) return st;
        if (c->bc != FD_BC_ZERO) return fail(FD_E_INVAL, "%s: member %d is not zero-boundary", who, i);
        if (c->r != ctxs[0]->r || c->dtype != ctxs[0]->dtype || c->g.ndim != ctxs[0]->g.ndim)
            return fail(FD_E_INVAL, "%s: member %d has another radius, dtype or dimension", who, i);
        if (!kf) kf = c->kf;
        mixed = mixed || c->kf != kf;
        if (target[i] < c->step) return fail(FD_E_INVAL, "%s: target below the member's step", who);
        if (c->nrec > 0 && target[i] - c->rec_base > c->rec_cap)
            return fail(FD_E_RANGE, "%s: member %d target exceeds its trace capacity", who, i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(FD_E_INVAL, "%s: member %d appears twice", who, i);
    }
    // One launch runs one kernel: members whose contexts chose different tile builds (the
    // library picks one per grid) are stepped with the default tile, whose tiles fit every
    // grid; the arithmetic, and so every result, is the same whatever the tile.
    int slots = nctx > 0 ? ctxs[0]->slots : 0;
    if (mixed) {
        int count = 0;
        kf = &fwd_table(ctxs[0]->dtype, ctxs[0]->r, (int)ctxs[0]->g.ndim, &count)[0];
        slots = resident_slots(kf->kernel, kf->nt);
    }
    std::vector<int64_t> btx((size_t)nctx), bty((size_t)nctx);
    for (int i = 0; i < nctx; ++i) {
        btx[(size_t)i] = (ctxs[i]->L.knx + kf->bx - 1) / kf->bx;
        bty[(size_t)i] = (ctxs[i]->L.kny + kf->by - 1) / kf->by;
    }
    desc.resize((size_t)nctx);
    prefix.assign((size_t)nctx + 1, 0);
    // Re-chunk the members for the batch as a whole: the other shots supply parallelism,
    // so each shot can march longer z chunks (fewer prologue re-reads) than it would
    // alone.  For a target length Z every member takes c = ceil(nz / Z) chunks of equal
    // length ceil(nz / c) <= Z (no short tail chunk); the launch costs about
    // ceil(workgroups / slots) x (longest chunk + 2r) plane-times, minimised over the
    // targets that are some member's exact chunk length.
    std::vector<int64_t> zchm((size_t)nctx, 1);
    if (nctx > 0) {
        const int r = ctxs[0]->r;
        std::vector<int64_t> cand;
        for (int i = 0; i < nctx; ++i) {
            const int64_t nz = ctxs[i]->L.knz;
            for (int64_t c = 1; c <= std::max<int64_t>(1, nz); ++c) cand.push_back((nz + c - 1) / c);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        double best = 1e300;
        int64_t zt = cand.empty() ? 1 : cand.back();
        for (int64_t Z : cand) {
            int64_t nwg = 0, planes = 0;
            for (int i = 0; i < nctx; ++i) {
                const int64_t nz = ctxs[i]->L.knz, cm = (nz + Z - 1) / Z, zm = (nz + cm - 1) / cm;
                nwg += btx[(size_t)i] * bty[(size_t)i] * cm;
                planes = std::max<int64_t>(planes, zm);
            }
            const double cost = (double)((nwg + slots - 1) / slots) * (double)(planes + 2 * r);
            if (cost < best - 1e-9) {
                best = cost;
                zt = Z;
            }
        }
        for (int i = 0; i < nctx; ++i) {
            const int64_t nz = ctxs[i]->L.knz, cm = (nz + zt - 1) / zt;
            zchm[(size_t)i] = (nz + cm - 1) / cm;
        }
    }
    for (int i = 0; i < nctx; ++i) {
        fd_ctx *c = ctxs[i];
        ShotDesc d = c->desc;
        d.ctr[0] = c->step;
        d.ctr[1] = c->step;
        d.target = target[i];
        d.tiles_x = (int32_t)btx[(size_t)i];
        d.tiles_y = (int32_t)bty[(size_t)i];
        d.zch = (int32_t)zchm[(size_t)i];
        d.chunks_z = (int32_t)((c->L.knz + d.zch - 1) / d.zch);
        desc[(size_t)i] = d;
        const int64_t next = (int64_t)prefix[(size_t)i] + btx[(size_t)i] * bty[(size_t)i] * d.chunks_z;
        if (next > INT32_MAX) return fail(FD_E_RANGE, "%s: too many workgroups in one launch", who);
        prefix[(size_t)i + 1] = (int32_t)next;
    }
    *kf_out = kf;
    return FD_OK;
}

extern "C" int fd_batch_set(fd_batch *b, fd_ctx *const *ctxs, const int64_t *target, int nctx)
{
    if (!b || nctx < 0 || nctx > b->max_shots || (nctx > 0 && (!ctxs || !target)))
        return fail(FD_E_INVAL, "fd_batch_set: bad arguments");
    std::vector<ShotDesc> desc;
    std::vector<int32_t> prefix;
    const FwdEntry *kf = nullptr;
    int st = batch_table(ctxs, target, nctx, "fd_batch_set", desc, prefix, &kf);
    if (st) return st;
    if (b->noalloc)
        for (int i = 0; i < nctx; ++i)
            if (ctxs[i]->stream != b->stream)
                return fail(FD_E_INVAL, "fd_batch_set: member %d runs on another stream than the no-allocation batch", i);
    // Work a member still has queued on its own stream (steps, state uploads, source or
    // receiver tables) must finish before a batched launch touches that member: the batch
    // stream waits for each member stream's current tail (one event, re-recorded per
    // stream; a wait binds to the record made before it).
    hipError_t e = hipSuccess;
    for (int i = 0; i < nctx && e == hipSuccess; ++i) {
        if (ctxs[i]->stream == b->stream) continue;
        e = hipEventRecord(b->order_ev, ctxs[i]->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->order_ev, 0);
    }
    // wait for earlier batched work before rewriting the shot table it reads
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_set: %s", hipGetErrorString(e));
    batch_drop_graph(b);
    b->members.assign(ctxs, ctxs + nctx);
    b->target.assign(target, target + nctx);
    b->h_desc.swap(desc);
    b->h_prefix.swap(prefix);
    b->nwg = b->h_prefix[(size_t)nctx];
    b->kf = kf;
    b->slot = 0;
    if (nctx > 0) {
        e = hipMemcpyAsync(b->d_desc(), b->h_desc.data(), (size_t)nctx * sizeof(ShotDesc), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_prefix(), b->h_prefix.data(), b->h_prefix.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_set: %s", hipGetErrorString(e));
    }
    return FD_OK;
}

static LaunchArgs batch_args(const fd_batch *b, int slot)
{
    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.shots = b->d_desc();
    a.wg_prefix = b->members.size() > 1 ? b->d_prefix() : nullptr;
    a.nshots = (int32_t)b->members.size();
    a.slot = slot;
    a.step = -1;
    a.record = 1;
    a.xcd_remap = 1;
    return a;
}

extern "C" int fd_batch_step(fd_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return fail(FD_E_INVAL, "fd_batch_step: bad arguments");
    if (b->members.empty() || nsteps == 0) return FD_OK;
    int64_t done = 0;
    // align to slot 0 with a direct launch, then replay the captured even-length chunk
    while (done < nsteps && (b->slot != 0 || nsteps - done < 2)) {
        b->kf->launch(batch_args(b, b->slot), (int)b->nwg, b->stream);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: %s", hipGetErrorString(e));
        b->slot ^= 1;
        ++done;
    }
    const int64_t rest = nsteps - done;
    const int64_t chunk = b->noalloc ? 0 : rest - (rest & 1);  // a no-allocation batch launches directly
    if (chunk > 0) {
        if (!b->has_exec || b->exec_len != chunk) {
            batch_drop_graph(b);
            hipGraph_t graph;
            hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: capture: %s", hipGetErrorString(e));
            for (int64_t i = 0; i < chunk; ++i) b->kf->launch(batch_args(b, (int)(i & 1)), (int)b->nwg, b->cap_stream);
            e = hipStreamEndCapture(b->cap_stream, &graph);
            if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: end capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: instantiate: %s", hipGetErrorString(e));
            b->has_exec = true;
            b->exec_len = chunk;
        }
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: graph launch: %s", hipGetErrorString(e));
        done += chunk;
    }
    // an odd tail
    while (done < nsteps) {
        b->kf->launch(batch_args(b, b->slot), (int)b->nwg, b->stream);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: %s", hipGetErrorString(e));
        b->slot ^= 1;
        ++done;
    }
    // Later work on a member's own stream (fd_sync, fd_get_state, fd_step, ...) is ordered
    // after these batched steps: each member stream waits for the batch stream's tail.
    bool other = false;
    for (const fd_ctx *c : b->members) other = other || c->stream != b->stream;
    if (other) {
        hipError_t e = hipEventRecord(b->order_ev, b->stream);
        for (size_t i = 0; i < b->members.size() && e == hipSuccess; ++i)
            if (b->members[i]->stream != b->stream) e = hipStreamWaitEvent(b->members[i]->stream, b->order_ev, 0);
        if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_batch_step: %s", hipGetErrorString(e));
    }
    for (size_t i = 0; i < b->members.size(); ++i) {
        fd_ctx *c = b->members[i];
        c->step = std::min(c->step + nsteps, b->target[i]);
    }
    return FD_OK;
}

// ------------------------------------------------------------------ measurement helpers

extern "C" int fd_copy_probe(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return fail(FD_E_INVAL, "fd_copy_probe: bad arguments");
    hipError_t e = launch_copy_probe(dst, src, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_copy_probe: %s", hipGetErrorString(e));
    return FD_OK;
}

extern "C" int fd_stream_probe(const void *a, const void *b, void *c, size_t bytes, int blocks, void *stream)
{
    if (!a || !b || !c || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(a) % 16 ||
        reinterpret_cast<uintptr_t>(b) % 16 || reinterpret_cast<uintptr_t>(c) % 16)
        return fail(FD_E_INVAL, "fd_stream_probe: bad arguments");
    if (blocks < 0 || blocks > 65536) return fail(FD_E_INVAL, "fd_stream_probe: blocks must be in [0, 65536]");
    hipError_t e = launch_stream_probe(a, b, c, bytes, blocks == 0 ? 512 : blocks, (hipStream_t)stream);
    if (e != hipSuccess) return fail(FD_E_DEVICE, "fd_stream_probe: %s", hipGetErrorString(e));
    return FD_OK;
}
