// fd_util.h -- launchers of the element-wise kernels in fd_util.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

// Interior extent and padded addressing of one field (kernel axes: 2-D grids use
// nx = grid nx, ny = 1, nz = grid ny).
struct Geom {
    int64_t nx, ny, nz;
    int64_t px, pxy, off0;
};

constexpr int kPrepBlocks = 1024;  // partial min/max slots the prep kernel writes

hipError_t launch_prep(int dtype, const Geom &g, const void *v, void *c, double k, double *partial,
                       double *minmax, hipStream_t st);
hipError_t launch_pack(int dtype, const Geom &g, const void *padded, void *dense, hipStream_t st);

// count consecutive padded fields of field_elems elements each: rows of px elements,
// py rows per plane, `planes` planes; the interior is x in [x0, x0 + nx), y in
// [y0, y0 + ny), plane in [z0, z0 + nz)
struct GhostBox {
    int64_t count, field_elems, px, py, planes;
    int64_t x0, y0, z0, nx, ny, nz;
};
hipError_t launch_clear_ghosts(int dtype, const GhostBox &b, void *fields, hipStream_t st);
hipError_t launch_unpack(int dtype, const Geom &g, const void *dense, void *padded, hipStream_t st);
hipError_t launch_halo_periodic(int dtype, const Geom &g, int hx, int hy, int hz, void *u, hipStream_t st);
hipError_t launch_ricker(int dtype, void *out, int64_t nsamp, double dt, double f0, double t0, hipStream_t st);
hipError_t launch_grad_finish(int dtype, const Geom &g, const void *gpad, const void *v, void *out, double scale,
                              hipStream_t st);
hipError_t launch_copy_probe(void *dst, const void *src, size_t bytes, hipStream_t st);
// out[1] = 1 if a or b (n elements each) holds a non-finite value, else 0; partial holds
// 2 * kPrepBlocks doubles.
hipError_t launch_nonfinite(int dtype, const void *a, const void *b, int64_t n, double *partial, double *out,
                           hipStream_t st);
hipError_t launch_stream_probe(const void *a, const void *b, void *c, size_t bytes, int blocks, hipStream_t st);

// VTI model preparation: from dense vz, eps, delta write ax, an, az = k nu^2 (k = dt^2/h^2)
// into the padded layout and reduce, over all points, the largest eigenvalue of the
// mode matrix [[nu_x^2 a, nu_z^2 b], [nu_n^2 a, nu_z^2 b]] and two flags (invalid model
// value; delta > eps) into out[0..2].  partial holds 3 * kPrepBlocks doubles.
hipError_t launch_vti_prep(int dtype, const Geom &g, const void *vz, const void *eps, const void *delta, void *ax,
                           void *an, void *az, double k, double a, double b, double *partial, double *out,
                           hipStream_t st);

}  // namespace fdw
