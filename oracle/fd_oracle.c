/*
 * fd_oracle.c -- plain FP64 CPU reference for explicit leapfrog time stepping
 * of the acoustic wave equation  u_tt = v(x)^2 lap(u) + s(t) delta(x - x_s).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the GPU library.
 *
 * What it follows (Medina, St-Cyr, Warburton, "High-Order Finite-differences
 * on multi-threaded architectures using OCCA"):
 *   - Sec. 1, the centred second-order time scheme
 *         u^{n+1} - 2 u^n + u^{n-1} = dt^2 F(u^n),   t^n = n dt;
 *   - Sec. 1, the symmetric star stencil
 *         h^2 (d_xx + d_yy) p ~ w0 p + sum_{l=1..R} w_l (p_{i+l} + p_{i-l} + p_{j+l} + p_{j-l}),
 *     used here with one radius r and one spacing h on every axis;
 *   - Sec. 1, the solution taken as zero for R points outside the domain
 *     (zero Dirichlet ghost cells); a periodic mode exists for closed-form tests;
 *   - Sec. 1, eq. (p): the point source s(t) delta(x - x_i), not multiplied by
 *     the squared velocity.  A discrete delta is 1/h^ndim at the grid point, so
 *     the source adds dt^2 s[n] / h^ndim to u^{n+1}.
 *   - Isotropic reduction (end of Sec. 1): one field u, F = v^2 lap(u) + source.
 *
 * Layout: dense row-major [nz][ny][nx], x fastest.  ndim = 1 uses nx only,
 * ndim = 2 uses [ny][nx].  All arithmetic is IEEE double, no reassociation.
 * The only parallelism is an OpenMP loop over the slowest index of each
 * point loop; every point is computed exactly as written.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FDO_OK 0
#define FDO_EINVAL -1
#define FDO_ENOMEM -6

typedef struct {
    int ndim;
    int64_t n[3]; /* nx, ny, nz; unused axes are 1 */
    int r;
    const double *w; /* w[0..r]: w0 (centre, per axis) and w_1..w_r */
    double h;
    int periodic;
} grid_t;

static int64_t npoints(const grid_t *g) { return g->n[0] * g->n[1] * g->n[2]; }

/* Value of u at integer coordinates (i, j, k), which may lie outside the
 * domain: zero ghost cells for the Dirichlet reading, wrap-around when periodic. */
static double value_at(const grid_t *g, const double *u, int64_t i, int64_t j, int64_t k)
{
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (g->periodic) {
            c[a] = ((c[a] % g->n[a]) + g->n[a]) % g->n[a];
        } else if (c[a] < 0 || c[a] >= g->n[a]) {
            return 0.0;
        }
    }
    return u[(c[2] * g->n[1] + c[1]) * g->n[0] + c[0]];
}

/* A copy of u with g->r ghost cells on each side of every active axis, filled by
 * value_at (zeros, or wrapped values when periodic).  The stencil then reads
 * neighbours by plain indexing; the values it sees are exactly value_at's. */
typedef struct {
    int64_t pn[3]; /* padded extents */
    int64_t pad[3];
    double *data;
} padded_t;

static int pad_field(const grid_t *g, const double *u, padded_t *pf)
{
    for (int a = 0; a < 3; ++a) {
        pf->pad[a] = a < g->ndim ? g->r : 0;
        pf->pn[a] = g->n[a] + 2 * pf->pad[a];
    }
    if (!pf->data) {
        pf->data = (double *)malloc((size_t)(pf->pn[0] * pf->pn[1] * pf->pn[2]) * sizeof(double));
        if (!pf->data) return FDO_ENOMEM;
    }
    double *d = pf->data;
    const int64_t px = pf->pn[0], py = pf->pn[1];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < pf->pn[2]; ++k)
        for (int64_t j = 0; j < py; ++j)
            for (int64_t i = 0; i < px; ++i)
                d[(k * py + j) * px + i] = value_at(g, u, i - pf->pad[0], j - pf->pad[1], k - pf->pad[2]);
    return FDO_OK;
}

/* (L u) at one point: h^-2 [ ndim w0 u + sum_axes sum_l w_l (u_{+l} + u_{-l}) ],
 * the stencil form of Sec. 1 applied on each active axis. */
static double laplacian_at(const grid_t *g, const padded_t *pf, int64_t i, int64_t j, int64_t k)
{
    const int64_t stride[3] = {1, pf->pn[0], pf->pn[0] * pf->pn[1]};
    const double *c = pf->data + ((k + pf->pad[2]) * pf->pn[1] + (j + pf->pad[1])) * pf->pn[0] + (i + pf->pad[0]);
    double acc = (double)g->ndim * g->w[0] * c[0];
    for (int a = 0; a < g->ndim; ++a) {
        for (int l = 1; l <= g->r; ++l) {
            double plus = c[l * stride[a]];
            double minus = c[-l * stride[a]];
            acc += g->w[l] * (plus + minus);
        }
    }
    return acc / (g->h * g->h);
}

static int check_grid(int ndim, const int64_t *n, int r, const double *w, double h)
{
    if (ndim < 1 || ndim > 3 || r < 1 || r > 16 || !w || !(h > 0.0))
        return FDO_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return FDO_EINVAL;
        if (a >= ndim && n[a] != 1) return FDO_EINVAL;
    }
    return FDO_OK;
}

static grid_t make_grid(int ndim, const int64_t *n, int r, const double *w, double h, int periodic)
{
    grid_t g;
    g.ndim = ndim;
    g.n[0] = n[0];
    g.n[1] = n[1];
    g.n[2] = n[2];
    g.r = r;
    g.w = w;
    g.h = h;
    g.periodic = periodic;
    return g;
}

/* out = L u over the whole grid. */
int fdo_laplacian(int ndim, const int64_t *n, int r, const double *w, double h, int periodic,
                  const double *u, double *out)
{
    int st = check_grid(ndim, n, r, w, h);
    if (st) return st;
    grid_t g = make_grid(ndim, n, r, w, h, periodic);
    padded_t pf = {{0, 0, 0}, {0, 0, 0}, NULL};
    st = pad_field(&g, u, &pf);
    if (st) return st;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g.n[2]; ++k)
        for (int64_t j = 0; j < g.n[1]; ++j)
            for (int64_t i = 0; i < g.n[0]; ++i)
                out[(k * g.n[1] + j) * g.n[0] + i] = laplacian_at(&g, &pf, i, j, k);
    free(pf.data);
    return FDO_OK;
}

/*
 * Forward solve.  For n = 0 .. nsteps-1:
 *     u^{n+1} = 2 u^n - u^{n-1} + dt^2 m (L u^n) + (dt^2 / h^ndim) sum_s src[n][s] e_{p_s}
 *     traces[n][j] = u^{n+1}(x_j)
 * with m = v^2 per point.
 *   u_cur  in: u^0,      out: u^T
 *   u_prev in: u^{-1},   out: u^{T-1}
 *   src_idx[s]  linear index of source s; src[n * nsrc + s] its sample at step n
 *   rec_idx[j]  linear index of receiver j; traces[n * nrec + j]
 *   states      optional [nsteps + 1][N]: u^0 .. u^T
 *   damp        optional [N]: the absorbing-sponge factor G of each point (1 outside the
 *               sponge).  The sponge of Sec. 1 (after Cerjan et al.) scales both time
 *               levels by G at every step; fused into the update this is
 *                   u^{n+1} = G (2 u^n - G u^{n-1} + dt^2 m L u^n),
 *               unchanged where G = 1.  Sources are added after it.
 */
int fdo_forward(int ndim, const int64_t *n, int r, const double *w, double h, double dt,
                const double *m, int periodic, int64_t nsteps, int64_t nsrc, const int64_t *src_idx,
                const double *src, int64_t nrec, const int64_t *rec_idx, double *traces,
                double *u_cur, double *u_prev, double *states, const double *damp)
{
    int st = check_grid(ndim, n, r, w, h);
    if (st) return st;
    if (nsteps < 0 || nsrc < 0 || nrec < 0 || !(dt > 0.0)) return FDO_EINVAL;
    grid_t g = make_grid(ndim, n, r, w, h, periodic);
    const int64_t N = npoints(&g);
    for (int64_t s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || src_idx[s] >= N) return FDO_EINVAL;
    for (int64_t j = 0; j < nrec; ++j)
        if (rec_idx[j] < 0 || rec_idx[j] >= N) return FDO_EINVAL;

    /* Three buffers whose roles rotate every step (u^{n+1} is written into the buffer that
     * held u^{n-2}); the results are copied back into the caller's arrays at the end. */
    double *spare = (double *)malloc((size_t)N * sizeof(double));
    if (!spare) return FDO_ENOMEM;
    double *cur = u_cur, *prev = u_prev, *next = spare;
    padded_t pf = {{0, 0, 0}, {0, 0, 0}, NULL};
    const double dt2 = dt * dt;
    const double src_scale = dt2 / pow(h, (double)ndim);

    if (states) memcpy(states, u_cur, (size_t)N * sizeof(double));
    for (int64_t step = 0; step < nsteps; ++step) {
        if (pad_field(&g, cur, &pf)) {
            free(spare);
            return FDO_ENOMEM;
        }
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < g.n[2]; ++k)
            for (int64_t j = 0; j < g.n[1]; ++j)
                for (int64_t i = 0; i < g.n[0]; ++i) {
                    int64_t p = (k * g.n[1] + j) * g.n[0] + i;
                    if (damp) {
                        const double G = damp[p];
                        next[p] = G * (2.0 * cur[p] - G * prev[p] + dt2 * m[p] * laplacian_at(&g, &pf, i, j, k));
                    } else {
                        next[p] = 2.0 * cur[p] - prev[p] + dt2 * m[p] * laplacian_at(&g, &pf, i, j, k);
                    }
                }
        for (int64_t s = 0; s < nsrc; ++s)
            next[src_idx[s]] += src_scale * src[step * nsrc + s];
        for (int64_t jr = 0; jr < nrec; ++jr)
            traces[step * nrec + jr] = next[rec_idx[jr]];
        /* rotate: u^{n-1} <- u^n, u^n <- u^{n+1} */
        double *t = prev;
        prev = cur;
        cur = next;
        next = t;
        if (states) memcpy(states + (step + 1) * N, cur, (size_t)N * sizeof(double));
    }
    /* u^T and u^{T-1} back into the caller's arrays.  The buffers hold them in some
     * rotation; `next` holds nothing needed, so the caller array it is gets filled first. */
    if (next == u_prev) {
        memcpy(u_prev, prev, (size_t)N * sizeof(double));
        memcpy(u_cur, cur, (size_t)N * sizeof(double));
    } else if (next == u_cur) {
        memcpy(u_cur, cur, (size_t)N * sizeof(double));
        memcpy(u_prev, prev, (size_t)N * sizeof(double));
    }
    free(spare);
    free(pf.data);
    return FDO_OK;
}

/*
 * Discrete adjoint of fdo_forward for the misfit J = 1/2 sum_n sum_j resid[n][j]^2,
 * resid = traces - observed.  Written as the Lagrange multiplier recursion of the
 * forward scheme (discretise, then differentiate):
 *     lambda^{T+1} = lambda^{T+2} = 0,  for k = T .. 1:
 *     lambda^k = 2 lambda^{k+1} - lambda^{k+2} + dt^2 L( m lambda^{k+1} ) + sum_j resid[k-1][j] e_{x_j}
 *     dJ/dm   += dt^2 lambda^k (L u^{k-1})
 * L is symmetric for the zero and periodic boundaries, so L^T (m .) = L (m .).
 *
 * fdo_adjoint_range runs the recursion for k = k_hi down to k_lo + 1 only, so that the
 * forward states can be recomputed segment by segment from checkpoints:
 *   states_seg  [k_hi - k_lo][N]: u^{k_lo} .. u^{k_hi - 1}
 *   lam1, lam2  in: lambda^{k_hi+1}, lambda^{k_hi+2};  out: lambda^{k_lo+1}, lambda^{k_lo+2}
 *   grad_m      dJ/dm, accumulated (the caller zeroes it before the first range)
 * fdo_adjoint is the whole range k = T .. 1 from zero multipliers:
 *   states   [nsteps][N]: u^0 .. u^{T-1} (as stored by fdo_forward)
 *   grad_m   out: dJ/dm per point (m = v^2)
 */
int fdo_adjoint_range(int ndim, const int64_t *n, int r, const double *w, double h, double dt,
                      const double *m, int periodic, int64_t k_hi, int64_t k_lo, int64_t nrec,
                      const int64_t *rec_idx, const double *resid, const double *states_seg,
                      double *lam1_io, double *lam2_io, double *grad_m)
{
    int st = check_grid(ndim, n, r, w, h);
    if (st) return st;
    if (k_lo < 0 || k_hi < k_lo || nrec < 0 || !(dt > 0.0)) return FDO_EINVAL;
    grid_t g = make_grid(ndim, n, r, w, h, periodic);
    const int64_t N = npoints(&g);
    for (int64_t j = 0; j < nrec; ++j)
        if (rec_idx[j] < 0 || rec_idx[j] >= N) return FDO_EINVAL;

    double *spare = (double *)malloc((size_t)N * sizeof(double)); /* holds lambda^k */
    double *mlam = (double *)malloc((size_t)N * sizeof(double));  /* m lambda^{k+1} */
    if (!spare || !mlam) {
        free(spare);
        free(mlam);
        return FDO_ENOMEM;
    }
    double *lam1 = lam1_io, *lam2 = lam2_io, *lam0 = spare; /* lambda^{k+1}, lambda^{k+2}, lambda^k */
    const double dt2 = dt * dt;
    padded_t pf = {{0, 0, 0}, {0, 0, 0}, NULL};
    int status = FDO_OK;

    for (int64_t k = k_hi; k >= k_lo + 1; --k) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < N; ++p) mlam[p] = m[p] * lam1[p];
        if (pad_field(&g, mlam, &pf)) {
            status = FDO_ENOMEM;
            break;
        }
#pragma omp parallel for schedule(static)
        for (int64_t kk = 0; kk < g.n[2]; ++kk)
            for (int64_t j = 0; j < g.n[1]; ++j)
                for (int64_t i = 0; i < g.n[0]; ++i) {
                    int64_t p = (kk * g.n[1] + j) * g.n[0] + i;
                    lam0[p] = 2.0 * lam1[p] - lam2[p] + dt2 * laplacian_at(&g, &pf, i, j, kk);
                }
        for (int64_t jr = 0; jr < nrec; ++jr)
            lam0[rec_idx[jr]] += resid[(k - 1) * nrec + jr];
        const double *u_km1 = states_seg + (k - 1 - k_lo) * N;
        if (pad_field(&g, u_km1, &pf)) {
            status = FDO_ENOMEM;
            break;
        }
#pragma omp parallel for schedule(static)
        for (int64_t kk = 0; kk < g.n[2]; ++kk)
            for (int64_t j = 0; j < g.n[1]; ++j)
                for (int64_t i = 0; i < g.n[0]; ++i) {
                    int64_t p = (kk * g.n[1] + j) * g.n[0] + i;
                    grad_m[p] += dt2 * lam0[p] * laplacian_at(&g, &pf, i, j, kk);
                }
        /* rotate: lambda^{k+2} <- lambda^{k+1}, lambda^{k+1} <- lambda^k */
        double *t = lam2;
        lam2 = lam1;
        lam1 = lam0;
        lam0 = t;
    }
    /* the two newest multipliers back into the caller's arrays; lam0 holds nothing needed,
     * so the caller array it is gets filled first */
    if (lam0 == lam2_io) {
        memcpy(lam2_io, lam2, (size_t)N * sizeof(double));
        memcpy(lam1_io, lam1, (size_t)N * sizeof(double));
    } else if (lam0 == lam1_io) {
        memcpy(lam1_io, lam1, (size_t)N * sizeof(double));
        memcpy(lam2_io, lam2, (size_t)N * sizeof(double));
    }
    free(spare);
    free(mlam);
    free(pf.data);
    return status;
}

int fdo_adjoint(int ndim, const int64_t *n, int r, const double *w, double h, double dt,
                const double *m, int periodic, int64_t nsteps, int64_t nrec, const int64_t *rec_idx,
                const double *resid, const double *states, double *grad_m)
{
    int st = check_grid(ndim, n, r, w, h);
    if (st) return st;
    if (nsteps < 0) return FDO_EINVAL;
    grid_t g = make_grid(ndim, n, r, w, h, periodic);
    const int64_t N = npoints(&g);
    double *lam1 = (double *)calloc((size_t)N, sizeof(double)); /* lambda^{T+1} = 0 */
    double *lam2 = (double *)calloc((size_t)N, sizeof(double)); /* lambda^{T+2} = 0 */
    if (!lam1 || !lam2) {
        free(lam1);
        free(lam2);
        return FDO_ENOMEM;
    }
    memset(grad_m, 0, (size_t)N * sizeof(double));
    st = fdo_adjoint_range(ndim, n, r, w, h, dt, m, periodic, nsteps, 0, nrec, rec_idx, resid, states, lam1,
                           lam2, grad_m);
    free(lam1);
    free(lam2);
    return st;
}
