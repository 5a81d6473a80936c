// fd_util.hip -- element-wise device kernels around the stencil: model preparation
// (v -> c = (v dt / h)^2 in the padded layout, with min/max of v), dense <-> padded
// copies, the periodic ghost fill, clearing of ghost cells, Ricker samples, the gradient
// finish and the bandwidth probe.  All are HBM-bound streaming kernels with grid-stride
// loops.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "fd_util.h"

namespace fdw {

namespace {

constexpr int kThreads = 256;

inline int blocks_for(int64_t n, int cap = 8192)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__device__ __forceinline__ int64_t padded_offset(const Geom &g, int64_t i)
{
    const int64_t x = i % g.nx;
    const int64_t t = i / g.nx;
    const int64_t y = t % g.ny;
    const int64_t z = t / g.ny;
    return g.off0 + z * g.pxy + y * g.px + x;
}

// Any non-finite value in two arrays of n elements: per block partial[2b] = 0,
// partial[2b+1] = 1 if the block saw one (reduced by minmax_final).
template <typename T>
__global__ void nonfinite_kernel(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                 double *__restrict__ partial)
{
    __shared__ int sbad[kThreads];
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i]) || !isfinite(b[i])) bad = 1;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sbad[threadIdx.x] = max(sbad[threadIdx.x], sbad[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = 0.0;
        partial[2 * blockIdx.x + 1] = sbad[0] ? 1.0 : 0.0;
    }
}

template <typename T>
__global__ void prep_kernel(Geom g, const T *__restrict__ v, T *__restrict__ c, double k,
                            double *__restrict__ partial)
{
    __shared__ double smin[kThreads], smax[kThreads];
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    double lo = INFINITY, hi = -INFINITY;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double vi = (double)v[i];
        if (!(vi > 0.0) || !isfinite(vi)) bad = true;
        lo = fmin(lo, vi);
        hi = fmax(hi, vi);
        c[padded_offset(g, i)] = (T)(k * vi * vi);
    }
    if (bad) lo = -1.0;  // reported as an invalid velocity
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = smin[0];
        partial[2 * blockIdx.x + 1] = smax[0];
    }
}

__global__ void minmax_final(const double *__restrict__ partial, int nb, double *__restrict__ out)
{
    __shared__ double smin[kThreads], smax[kThreads];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        lo = fmin(lo, partial[2 * i]);
        hi = fmax(hi, partial[2 * i + 1]);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smin[0];
        out[1] = smax[0];
    }
}

template <typename T>
__global__ void pack_kernel(Geom g, const T *__restrict__ padded, T *__restrict__ dense)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dense[i] = padded[padded_offset(g, i)];
}

template <typename T>
__global__ void unpack_kernel(Geom g, const T *__restrict__ dense, T *__restrict__ padded)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        padded[padded_offset(g, i)] = dense[i];
}

// Periodic ghost fill: every cell of the box [-hx, nx+hx) x [-hy, ny+hy) x [-hz, nz+hz)
// that lies outside the interior takes the value of its wrapped interior image.
template <typename T>
__global__ void halo_periodic_kernel(Geom g, int hx, int hy, int hz, T *__restrict__ u)
{
    const int64_t ex = g.nx + 2 * hx, ey = g.ny + 2 * hy, ez = g.nz + 2 * hz;
    const int64_t n = ex * ey * ez;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i % ex - hx;
        const int64_t t = i / ex;
        const int64_t y = t % ey - hy;
        const int64_t z = t / ey - hz;
        const bool inside = x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        if (inside) continue;
        const int64_t wx = (x % g.nx + g.nx) % g.nx;
        const int64_t wy = (y % g.ny + g.ny) % g.ny;
        const int64_t wz = (z % g.nz + g.nz) % g.nz;
        u[g.off0 + z * g.pxy + y * g.px + x] = u[g.off0 + wz * g.pxy + wy * g.px + wx];
    }
}

template <typename T>
__global__ void ricker_kernel(T *__restrict__ out, int64_t nsamp, double dt, double f0, double t0)
{
    const double pf = 3.14159265358979323846 * f0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nsamp; n += (int64_t)gridDim.x * blockDim.x) {
        const double tau = (double)n * dt - t0;
        const double a = pf * pf * tau * tau;
        out[n] = (T)((1.0 - 2.0 * a) * exp(-a));
    }
}

template <typename T>
__global__ void grad_finish_kernel(Geom g, const T *__restrict__ gpad, const T *__restrict__ v,
                                   T *__restrict__ out, double scale)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (T)(scale * 2.0 * (double)gpad[padded_offset(g, i)] / (double)v[i]);
}

// VTI model preparation (see launch_vti_prep).  lam is the larger root of
// x^2 - (A + B) x + B (A - C) with A = nu_x^2 a, B = nu_z^2 b, C = nu_n^2 a.
template <typename T>
__global__ void vti_prep_kernel(Geom g, const T *__restrict__ vz, const T *__restrict__ eps,
                                const T *__restrict__ delta, T *__restrict__ ax, T *__restrict__ an,
                                T *__restrict__ az, double k, double a, double b, double *__restrict__ partial)
{
    __shared__ double s0[kThreads], s1[kThreads], s2[kThreads];
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    double lam = 0.0, bad = 0.0, anis = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)vz[i], e = (double)eps[i], d = (double)delta[i];
        const double fx = 1.0 + 2.0 * e, fn = 1.0 + 2.0 * d;
        if (!(v > 0.0) || !isfinite(v) || !(fx > 0.0) || !isfinite(fx) || !(fn >= 0.0) || !isfinite(fn)) bad = 1.0;
        if (d > e) anis = 1.0;
        const double z2 = v * v, x2 = z2 * fx, n2 = z2 * fn;
        const double A = x2 * a, B = z2 * b, C = n2 * a;
        const double l = 0.5 * ((A + B) + sqrt((A - B) * (A - B) + 4.0 * B * C));
        lam = fmax(lam, l);
        const int64_t o = padded_offset(g, i);
        ax[o] = (T)(k * x2);
        an[o] = (T)(k * n2);
        az[o] = (T)(k * z2);
    }
    s0[threadIdx.x] = lam;
    s1[threadIdx.x] = bad;
    s2[threadIdx.x] = anis;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + s]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = s0[0];
        partial[3 * blockIdx.x + 1] = s1[0];
        partial[3 * blockIdx.x + 2] = s2[0];
    }
}

__global__ void max3_final(const double *__restrict__ partial, int nb, double *__restrict__ out)
{
    __shared__ double s0[kThreads], s1[kThreads], s2[kThreads];
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        m0 = fmax(m0, partial[3 * i]);
        m1 = fmax(m1, partial[3 * i + 1]);
        m2 = fmax(m2, partial[3 * i + 2]);
    }
    s0[threadIdx.x] = m0;
    s1[threadIdx.x] = m1;
    s2[threadIdx.x] = m2;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + s]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
        out[2] = s2[0];
    }
}

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void copy_probe_kernel(f4 *__restrict__ dst, const f4 *__restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// The forward stencil's stream mix without halo or stencil arithmetic: read a, b and c,
// write c in place (as the update writes u^{n+1} over u^{n-1}); b and c nontemporal.
// Grid-stride over 16-byte vectors, two vectors in flight per thread.
__global__ __launch_bounds__(256) void stream_probe_kernel(const f4 *__restrict__ a, const f4 *__restrict__ b, f4 *c,
                                                           int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 2 * stride) {
        f4 x[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < n) x[u] = (a[i] + __builtin_nontemporal_load(&b[i])) * __builtin_nontemporal_load(&c[i]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < n) __builtin_nontemporal_store(x[u], &c[i]);
        }
    }
}

}  // namespace

template <typename T>
static hipError_t prep_t(const Geom &g, const void *v, void *c, double k, double *partial, double *minmax,
                         hipStream_t st)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int nb = blocks_for(n, kPrepBlocks);
    hipLaunchKernelGGL(prep_kernel<T>, dim3(nb), dim3(kThreads), 0, st, g, (const T *)v, (T *)c, k, partial);
    hipLaunchKernelGGL(minmax_final, dim3(1), dim3(kThreads), 0, st, (const double *)partial, nb, minmax);
    return hipGetLastError();
}

hipError_t launch_prep(int dtype, const Geom &g, const void *v, void *c, double k, double *partial,
                       double *minmax, hipStream_t st)
{
    return dtype == 0 ? prep_t<float>(g, v, c, k, partial, minmax, st)
                      : prep_t<double>(g, v, c, k, partial, minmax, st);
}

hipError_t launch_pack(int dtype, const Geom &g, const void *padded, void *dense, hipStream_t st)
{
    const int nb = blocks_for((int64_t)g.nx * g.ny * g.nz);
    if (dtype == 0)
        hipLaunchKernelGGL(pack_kernel<float>, dim3(nb), dim3(kThreads), 0, st, g, (const float *)padded, (float *)dense);
    else
        hipLaunchKernelGGL(pack_kernel<double>, dim3(nb), dim3(kThreads), 0, st, g, (const double *)padded, (double *)dense);
    return hipGetLastError();
}

// Zero what lies outside the interior of each field, one plane per workgroup at a time
// (grid-stride over planes): planes outside the interior's z range are cleared whole,
// and so are the rows above and below the interior's y range (contiguous runs);
// each interior row is cleared left and right of [x0, x0 + nx) by one wave, its lanes
// taking the row's pad elements in turn.
template <typename T>
__global__ void clear_ghosts_kernel(GhostBox b, T *__restrict__ f)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
    const int64_t plane_elems = b.py * b.px;
    const int x0 = (int)b.x0, nx = (int)b.nx, y0 = (int)b.y0, ny = (int)b.ny;
    const int padw = (int)(b.px - b.nx);  // pad elements per interior row
    for (int64_t pl = blockIdx.x; pl < b.count * b.planes; pl += gridDim.x) {
        const int64_t fi = pl / b.planes;
        const int64_t z = pl - fi * b.planes;
        T *P = f + fi * b.field_elems + z * plane_elems;
        if (z < b.z0 || z >= b.z0 + b.nz) {
            for (int64_t e = tid; e < plane_elems; e += nt) P[e] = T(0);
            continue;
        }
        for (int64_t e = tid; e < (int64_t)y0 * b.px; e += nt) P[e] = T(0);
        for (int64_t e = (int64_t)(y0 + ny) * b.px + tid; e < plane_elems; e += nt) P[e] = T(0);
        for (int y = y0 + wave; y < y0 + ny; y += nw) {
            T *row = P + (int64_t)y * b.px;
            for (int k = lane; k < padw; k += 64) row[k < x0 ? k : k + nx] = T(0);
        }
    }
}

hipError_t launch_clear_ghosts(int dtype, const GhostBox &b, void *fields, hipStream_t st)
{
    const int64_t planes = b.count * b.planes;
    const int nb = (int)std::min<int64_t>(planes, 16384);
    if (dtype == 0)
        hipLaunchKernelGGL(clear_ghosts_kernel<float>, dim3(nb), dim3(kThreads), 0, st, b, (float *)fields);
    else
        hipLaunchKernelGGL(clear_ghosts_kernel<double>, dim3(nb), dim3(kThreads), 0, st, b, (double *)fields);
    return hipGetLastError();
}

hipError_t launch_unpack(int dtype, const Geom &g, const void *dense, void *padded, hipStream_t st)
{
    const int nb = blocks_for((int64_t)g.nx * g.ny * g.nz);
    if (dtype == 0)
        hipLaunchKernelGGL(unpack_kernel<float>, dim3(nb), dim3(kThreads), 0, st, g, (const float *)dense, (float *)padded);
    else
        hipLaunchKernelGGL(unpack_kernel<double>, dim3(nb), dim3(kThreads), 0, st, g, (const double *)dense, (double *)padded);
    return hipGetLastError();
}

hipError_t launch_halo_periodic(int dtype, const Geom &g, int hx, int hy, int hz, void *u, hipStream_t st)
{
    const int64_t n = (int64_t)(g.nx + 2 * hx) * (g.ny + 2 * hy) * (g.nz + 2 * hz);
    const int nb = blocks_for(n);
    if (dtype == 0)
        hipLaunchKernelGGL(halo_periodic_kernel<float>, dim3(nb), dim3(kThreads), 0, st, g, hx, hy, hz, (float *)u);
    else
        hipLaunchKernelGGL(halo_periodic_kernel<double>, dim3(nb), dim3(kThreads), 0, st, g, hx, hy, hz, (double *)u);
    return hipGetLastError();
}

hipError_t launch_ricker(int dtype, void *out, int64_t nsamp, double dt, double f0, double t0, hipStream_t st)
{
    if (nsamp <= 0) return hipSuccess;
    const int nb = blocks_for(nsamp);
    if (dtype == 0)
        hipLaunchKernelGGL(ricker_kernel<float>, dim3(nb), dim3(kThreads), 0, st, (float *)out, nsamp, dt, f0, t0);
    else
        hipLaunchKernelGGL(ricker_kernel<double>, dim3(nb), dim3(kThreads), 0, st, (double *)out, nsamp, dt, f0, t0);
    return hipGetLastError();
}

hipError_t launch_grad_finish(int dtype, const Geom &g, const void *gpad, const void *v, void *out, double scale,
                              hipStream_t st)
{
    const int nb = blocks_for((int64_t)g.nx * g.ny * g.nz);
    if (dtype == 0)
        hipLaunchKernelGGL(grad_finish_kernel<float>, dim3(nb), dim3(kThreads), 0, st, g, (const float *)gpad,
                           (const float *)v, (float *)out, scale);
    else
        hipLaunchKernelGGL(grad_finish_kernel<double>, dim3(nb), dim3(kThreads), 0, st, g, (const double *)gpad,
                           (const double *)v, (double *)out, scale);
    return hipGetLastError();
}

hipError_t launch_vti_prep(int dtype, const Geom &g, const void *vz, const void *eps, const void *delta, void *ax,
                           void *an, void *az, double k, double a, double b, double *partial, double *out,
                           hipStream_t st)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int nb = blocks_for(n, kPrepBlocks);
    if (dtype == 0)
        hipLaunchKernelGGL(vti_prep_kernel<float>, dim3(nb), dim3(kThreads), 0, st, g, (const float *)vz,
                           (const float *)eps, (const float *)delta, (float *)ax, (float *)an, (float *)az, k, a, b,
                           partial);
    else
        hipLaunchKernelGGL(vti_prep_kernel<double>, dim3(nb), dim3(kThreads), 0, st, g, (const double *)vz,
                           (const double *)eps, (const double *)delta, (double *)ax, (double *)an, (double *)az, k,
                           a, b, partial);
    hipLaunchKernelGGL(max3_final, dim3(1), dim3(kThreads), 0, st, (const double *)partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_nonfinite(int dtype, const void *a, const void *b, int64_t n, double *partial, double *out,
                           hipStream_t st)
{
    const int nb = blocks_for(n, kPrepBlocks);
    if (dtype == 0)
        hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(nb), dim3(kThreads), 0, st, (const float *)a,
                           (const float *)b, n, partial);
    else
        hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(nb), dim3(kThreads), 0, st, (const double *)a,
                           (const double *)b, n, partial);
    hipLaunchKernelGGL(minmax_final, dim3(1), dim3(kThreads), 0, st, (const double *)partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_stream_probe(const void *a, const void *b, void *c, size_t bytes, int blocks, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(stream_probe_kernel, dim3(blocks), dim3(kThreads), 0, st, (const f4 *)a, (const f4 *)b, (f4 *)c,
                       n);
    return hipGetLastError();
}

hipError_t launch_copy_probe(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int nb = blocks_for(n, 4 * 256 * 8);
    hipLaunchKernelGGL(copy_probe_kernel, dim3(nb), dim3(kThreads), 0, st, (f4 *)dst, (const f4 *)src, n);
    return hipGetLastError();
}

}  // namespace fdw
