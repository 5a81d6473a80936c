/*
 * vti_oracle.c -- plain FP64 CPU reference for the two-field VTI propagator of
 * Sec. 1 (the pseudo-acoustic vertical transversely isotropic equations for p
 * and the auxiliary field q), stepped with the centred second-order time scheme
 * of Sec. 1.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite uses it.  It shares no code with the GPU
 * library.
 *
 * What it computes, per time step n (Sec. 1, eqs. (p) and (q), and the centred
 * time difference that follows them):
 *
 *   p^{n+1} = 2 p^n - p^{n-1} + dt^2 [ nux2 (Dxx + Dyy) p^n + nuz2 Dzz q^n ] + dt^2 sp[n] / (h^2 dz_k)
 *   q^{n+1} = 2 q^n - q^{n-1} + dt^2 [ nun2 (Dxx + Dyy) p^n + nuz2 Dzz q^n ] + dt^2 sq[n] / (h^2 dz_k)
 *
 * with nuz2 = vz^2, nux2 = vz^2 (1 + 2 eps), nun2 = vz^2 (1 + 2 delta) (the
 * velocities of Sec. 1), and
 *
 *   h^2 (Dxx + Dyy) p_{ijk} = 2 w_0 p_{ijk} + sum_{l=1..Rxy} w_l (p_{i+l,j,k} + p_{i-l,j,k} + p_{i,j+l,k} + p_{i,j-l,k})
 *       -- the symmetric xy stencil of Sec. 1, its centre weight 2 w_0 being the
 *          sum of the two 1-D centre weights;
 *   Dzz q_{ijk} = sum_{l=-Rz..Rz} wz_{k,l} q_{i,j,k+l}
 *       -- the per-plane z stencil of Sec. 1 with 2 Rz + 1 weights per plane; the
 *          caller supplies the table wz (variable spacing is absorbed in it).
 *
 * The sources are point sources: sample n of each source's wavelet, times its
 * amplitudes (amp_p, amp_q), divided by the cell volume h^2 dz_k of the source
 * point (dz_k supplied per plane), enters the step that produces level n+1.
 * Values outside the domain are zero for Rxy points in x and y and Rz planes in
 * z (Sec. 1, last paragraph), or wrap around per axis group when periodic.
 *
 * Layout: dense row-major [nz][ny][nx], x fastest.  All arithmetic is IEEE
 * double, no reassociation; the only parallelism is an OpenMP loop over z.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FDO_OK 0
#define FDO_EINVAL -1
#define FDO_ENOMEM -6

typedef struct {
    int64_t nx, ny, nz;
    int rxy, rz;
    const double *wxy; /* wxy[0..rxy]: 1-D centre weight and w_1..w_rxy */
    const double *wz;  /* [nz][2 rz + 1]: weight of plane k + l at index l + rz */
    double h;
    int per_xy, per_z;
} vgrid_t;

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* Value of field f at (i, j, k): zero outside the domain, or wrapped. */
static double at(const vgrid_t *g, const double *f, int64_t i, int64_t j, int64_t k)
{
    if (g->per_xy) {
        i = wrap(i, g->nx);
        j = wrap(j, g->ny);
    } else if (i < 0 || i >= g->nx || j < 0 || j >= g->ny) {
        return 0.0;
    }
    if (g->per_z)
        k = wrap(k, g->nz);
    else if (k < 0 || k >= g->nz)
        return 0.0;
    return f[(k * g->ny + j) * g->nx + i];
}

static double lxy_at(const vgrid_t *g, const double *p, int64_t i, int64_t j, int64_t k)
{
    double s = 2.0 * g->wxy[0] * at(g, p, i, j, k);
    for (int l = 1; l <= g->rxy; ++l)
        s += g->wxy[l] * (at(g, p, i + l, j, k) + at(g, p, i - l, j, k) + at(g, p, i, j + l, k) +
                          at(g, p, i, j - l, k));
    return s / (g->h * g->h);
}

static double dzz_at(const vgrid_t *g, const double *q, int64_t i, int64_t j, int64_t k)
{
    const double *w = g->wz + k * (2 * g->rz + 1);
    double s = 0.0;
    for (int l = -g->rz; l <= g->rz; ++l) s += w[l + g->rz] * at(g, q, i, j, k + l);
    return s;
}

/*
 * nsteps steps of the VTI scheme.  p, pm, q, qm hold p^0, p^{-1}, q^0, q^{-1} on
 * entry and p^T, p^{T-1}, q^T, q^{T-1} on return.  src is [nsteps][nsrc]
 * (sample n of source s), amp is [nsrc][2] (p and q amplitudes), dzc is [nz]
 * (the z extent of a cell at plane k).  trp / trq are [nsteps][nrec] (either may
 * be NULL): trp[n][j] = p^{n+1} at receiver j.
 */
int fdo_vti_forward(const int64_t *n, int rxy, int rz, const double *wxy, const double *wz, const double *dzc,
                    double h, double dt, const double *vz, const double *eps, const double *delta, int per_xy,
                    int per_z, int64_t nsteps, int64_t nsrc, const int64_t *src_idx, const double *src,
                    const double *amp, int64_t nrec, const int64_t *rec_idx, double *trp, double *trq, double *p,
                    double *pm, double *q, double *qm)
{
    if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1 || rxy < 1 || rz < 1 || !wxy || !wz || !dzc || !(h > 0) ||
        !vz || !eps || !delta || !p || !pm || !q || !qm || nsteps < 0 || nsrc < 0 || nrec < 0)
        return FDO_EINVAL;
    vgrid_t g = {n[0], n[1], n[2], rxy, rz, wxy, wz, h, per_xy, per_z};
    const int64_t np = n[0] * n[1] * n[2];
    const int64_t plane = n[0] * n[1];
    double *pn = (double *)malloc((size_t)np * sizeof(double));
    double *qn = (double *)malloc((size_t)np * sizeof(double));
    if (!pn || !qn) {
        free(pn);
        free(qn);
        return FDO_ENOMEM;
    }
    const double dt2 = dt * dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t k;
#pragma omp parallel for schedule(static)
        for (k = 0; k < n[2]; ++k)
            for (int64_t j = 0; j < n[1]; ++j)
                for (int64_t i = 0; i < n[0]; ++i) {
                    const int64_t x = (k * n[1] + j) * n[0] + i;
                    const double nuz2 = vz[x] * vz[x];
                    const double nux2 = nuz2 * (1.0 + 2.0 * eps[x]);
                    const double nun2 = nuz2 * (1.0 + 2.0 * delta[x]);
                    const double lp = lxy_at(&g, p, i, j, k);
                    const double dq = dzz_at(&g, q, i, j, k);
                    pn[x] = 2.0 * p[x] - pm[x] + dt2 * (nux2 * lp + nuz2 * dq);
                    qn[x] = 2.0 * q[x] - qm[x] + dt2 * (nun2 * lp + nuz2 * dq);
                }
        for (int64_t e = 0; e < nsrc; ++e) {
            const int64_t x = src_idx[e];
            const double vol = h * h * dzc[x / plane];
            pn[x] += dt2 * amp[2 * e] * src[s * nsrc + e] / vol;
            qn[x] += dt2 * amp[2 * e + 1] * src[s * nsrc + e] / vol;
        }
        for (int64_t j = 0; j < nrec; ++j) {
            if (trp) trp[s * nrec + j] = pn[rec_idx[j]];
            if (trq) trq[s * nrec + j] = qn[rec_idx[j]];
        }
        memcpy(pm, p, (size_t)np * sizeof(double));
        memcpy(p, pn, (size_t)np * sizeof(double));
        memcpy(qm, q, (size_t)np * sizeof(double));
        memcpy(q, qn, (size_t)np * sizeof(double));
    }
    free(pn);
    free(qn);
    return FDO_OK;
}
