// fd_stencil.h -- gfx950 stencil kernels for the leapfrog acoustic update.
//
// One launch performs one time step of
//     u^{n+1} = 2 u^n - u^{n-1} + c * Lh u^n + sources,   c = (v dt / h)^2,
// where Lh = h^2 L is the radius-R star stencil applied on every axis (the xy
// stencil form of Sec. 1 of Medina, St-Cyr and Warburton, extended to z with
// the same radius and spacing).  For R <= 4 the forward evaluates it in
// difference form,
//     Lh u = sum_axes sum_l w_l [ (u_{+l} - u) + (u_{-l} - u) ],
// algebraically the centre-weight form, which keeps FP32 rounding of smooth
// fields small and costs nothing there (the kernel is bandwidth-bound).  For
// R > 4 the vector work of that form limits the kernel, so it uses the
// centre-weight form of the paper, ndim w_0 u + sum_axes sum_l w_l (u_{+l} + u_{-l}),
// two operations per neighbour pair instead of four.
//
// Design (a star stencil is not a dense contraction, so no MFMA):
//  - A workgroup owns a BX x BY tile of the xy plane and marches a chunk of z
//    planes.  Each thread owns VEC consecutive x points (one 16-byte vector) in
//    EY rows and keeps u^n of its column at planes z-R..z+R in registers (the
//    z "register queue"); the plane z with an R-wide x/y halo is staged in LDS
//    (double buffered, one barrier per plane) for the x and y neighbours.
//  - Global traffic is x-contiguous 16-byte vectors: u^n once per point (plus
//    the halo), u^{n-1} and c streamed with nontemporal loads, u^{n+1} written
//    with nontemporal stores.  Every load of the next plane is issued one plane
//    ahead of its use.
//  - Sources and receivers are fused: a CSR event list over (x, y) columns,
//    sorted by z, gives each thread the next plane where one of its columns has
//    an event; only that plane takes the slow path.
//  - Workgroup ids are remapped so that a contiguous run of tiles lands on one
//    XCD (workgroups are dealt round-robin to the 8 XCDs), which keeps halo
//    re-reads inside that XCD's L2.
//
// Field layout (padded): element (x, y, z) of the interior sits at
// off0 + z * pxy + y * px + x; at least R zero ghost cells surround the
// interior on every face (the zero solution outside the domain, Sec. 1) and
// rows/planes carry alignment padding so that every tile load is in bounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "fd_types.h"

#pragma clang fp contract(off)

namespace fdw {

// ------------------------------------------------------------------ weights

constexpr unsigned __int128 gcd_u128(unsigned __int128 a, unsigned __int128 b)
{
    while (b != 0) {
        const unsigned __int128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Exact central weight of the radius-r second-derivative stencil:
// w_l = 2 (-1)^{l+1} (r!)^2 / (l^2 (r-l)! (r+l)!) = 2 (-1)^{l+1} [r!/(r-l)!] / (l^2 [(r+l)!/r!]).
// The fraction is reduced in 128-bit integers; for r <= 12 its reduced numerator and
// denominator are below 2^53, so the one division is correctly rounded.
constexpr double stencil_weight(int r, int l)
{
    unsigned __int128 num = 2, den = (unsigned __int128)(l * l);
    for (int i = r - l + 1; i <= r; ++i) num *= (unsigned)i;
    for (int i = r + 1; i <= r + l; ++i) den *= (unsigned)i;
    const unsigned __int128 g = gcd_u128(num, den);
    num /= g;
    den /= g;
    const double w = (double)(uint64_t)num / (double)(uint64_t)den;
    return (l % 2 == 1) ? w : -w;
}

template <int R>
struct StencilWeights {
    double w[R + 1];
    constexpr StencilWeights() : w()
    {
        double s = 0.0;
        for (int l = 1; l <= R; ++l) {
            w[l] = stencil_weight(R, l);
            s += w[l];
        }
        w[0] = -2.0 * s;
    }
};

// ------------------------------------------------------------------ x vectors

// N consecutive x points of one row, moved with one load or store instruction.  The
// kernels use 16-byte vectors (4 floats, 2 doubles) unless a tile asks for 8-byte ones.
template <typename T, int N>
struct VecT {
    typedef T t __attribute__((ext_vector_type(N)));
};
template <typename T>
struct V16 {
    static constexpr int N = 16 / (int)sizeof(T);
};

template <typename T, int N>
__device__ __forceinline__ void vld(T (&d)[N], const T *p)
{
    typename VecT<T, N>::t v = *reinterpret_cast<const typename VecT<T, N>::t *>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = v[i];
}

template <typename T, int N>
__device__ __forceinline__ void vld_nt(T (&d)[N], const T *p)
{
    typename VecT<T, N>::t v = __builtin_nontemporal_load(reinterpret_cast<const typename VecT<T, N>::t *>(p));
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = v[i];
}

template <typename T, int N>
__device__ __forceinline__ void vst(T *p, const T (&s)[N])
{
    typename VecT<T, N>::t v;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = s[i];
    *reinterpret_cast<typename VecT<T, N>::t *>(p) = v;
}

template <typename T, int N>
__device__ __forceinline__ void vst_nt(T *p, const T (&s)[N])
{
    typename VecT<T, N>::t v;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = s[i];
    __builtin_nontemporal_store(v, reinterpret_cast<typename VecT<T, N>::t *>(p));
}

template <typename T, int N>
__device__ __forceinline__ void vzero(T (&d)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = T(0);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of
// logical tile ids so that neighbouring tiles share an L2.  Bijective for any G.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    constexpr int NX = 8;
    const int q = G / NX, rem = G % NX;
    const int xcd = b % NX, idx = b / NX;
    return (xcd < rem) ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

// Calls f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>): the index is a
// compile-time constant inside f whatever the loop unroller decides.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int lower_bound_z(const Event *ev, int lo, int hi, int z)
{
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (ev[mid].z < z)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ tile configuration

template <typename T, int R_, int NDIM_, int TXN_, int TYN_, int EY_, int VEC_ = V16<T>::N, int OCC_ = 0>
struct TileCfg {
    typedef T type;
    // OCC > 0: the forward kernel is built for OCC waves per SIMD (the compiler keeps to
    // the matching register budget), keeps one set of prefetch registers instead of two
    // and, for OCC >= 4, fetches the early halo one plane later (a smaller LDS ring)
    static constexpr int OCC = OCC_;
    static constexpr int R = R_;
    static constexpr int NDIM = NDIM_;
    static constexpr int TXN = TXN_;                       // threads along x
    static constexpr int TYN = (NDIM_ == 3) ? TYN_ : 1;    // threads along y
    static constexpr int EY = (NDIM_ == 3) ? EY_ : 1;      // rows per thread
    static constexpr int VEC = VEC_;                       // x points per thread (one vector)
    static constexpr int NT = TXN * TYN;
    static constexpr int BX = TXN * VEC;
    static constexpr int BY = TYN * EY;
    static constexpr int LPAD = (R + VEC - 1) / VEC * VEC; // x halo rounded to vectors
    static constexpr int LW = BX + 2 * LPAD;               // LDS row length
    static constexpr int HY = (NDIM == 3) ? R : 0;         // y halo rows
    static constexpr int LH = BY + 2 * HY;
    static constexpr int LDS = LW * LH;                    // elements per LDS plane
    static constexpr int NXV = 2 * LPAD / VEC + 1;         // vectors read per row for x neighbours
    static constexpr int NHY = 2 * HY * TXN;               // y-halo vectors per plane
    static constexpr int NHS = LPAD / VEC;                 // x-halo vectors per side per row
    static constexpr int NHX = 2 * BY * NHS;
    static constexpr int NH = NHY + NHX;
    static constexpr int HPT = (NH + NT - 1) / NT;         // halo vectors per thread
    static constexpr int YR = EY + 2 * HY;                 // rows a thread touches along y
    // forward kernel: halo fetched HOFF planes ahead into a ring of NB LDS plane buffers
    // (early halo for R <= 4; larger radii would need too much LDS)
    static constexpr int HOFF = (R <= 4) ? (OCC_ >= 4 ? R - 1 : R) : 0;
    static constexpr int NB = HOFF + 2;
    static_assert(256 % BX == 0 && 64 % BY == 0, "tile must divide the layout alignment");
};

// Per-thread geometry of one tile, shared by the forward and adjoint kernels.
template <class C>
struct TileGeom {
    int lx, ly, gx, gy, x0, y0, z0, z1;
    int64_t col;             // element offset of (gx, gy, 0)
    bool rin[C::EY];         // row e of this thread lies inside the grid (computed and stored)
    bool lin[C::EY];         // row e lies inside the grid or its R-wide ghost ring (loaded)
    int64_t hoff[C::HPT];    // halo vector k: element offset at z = 0
    int hl[C::HPT];          // halo vector k: LDS offset
    bool hval[C::HPT];

    __device__ __forceinline__ void init(const ShotDesc &s, int tx, int ty, int cz, int zch)
    {
        const int tid = threadIdx.x;
        lx = (tid % C::TXN) * C::VEC;
        ly = (tid / C::TXN) * C::EY;
        x0 = tx * C::BX;
        y0 = ty * C::BY;
        gx = x0 + lx;
        gy = y0 + ly;
        z0 = cz * zch;
        z1 = min(z0 + zch, s.nz);
        col = s.off0 + (int64_t)gy * s.px + gx;
#pragma unroll
        for (int e = 0; e < C::EY; ++e) {
            rin[e] = (gx < s.nx) && (gy + e < s.ny);
            lin[e] = (gx < s.nx + C::R) && (gy + e < s.ny + C::HY);
        }
#pragma unroll
        for (int k = 0; k < C::HPT; ++k) {
            const int hv = tid + k * C::NT;
            hval[k] = hv < C::NH;
            int ry = 0, cx = 0;
            if (hv < C::NHY) {
                const int ri = hv / C::TXN;
                cx = (hv % C::TXN) * C::VEC;
                ry = (ri < C::HY) ? ri - C::HY : C::BY + (ri - C::HY);
            } else if (hv < C::NH) {
                const int hx = hv - C::NHY;
                ry = hx / (2 * C::NHS);
                const int si = hx % (2 * C::NHS);
                cx = (si < C::NHS) ? -C::LPAD + si * C::VEC : C::BX + (si - C::NHS) * C::VEC;
            }
            hoff[k] = s.off0 + (int64_t)(y0 + ry) * s.px + (x0 + cx);
            hl[k] = (ry + C::HY) * C::LW + (cx + C::LPAD);
        }
    }
};

// Next plane >= z at which one of this thread's columns has an event (INT_MAX if none).
template <class C>
__device__ __forceinline__ int next_event(const ShotDesc &s, const TileGeom<C> &g, int z)
{
    int nxt = 0x7fffffff;
    if (!s.ev_ptr) return nxt;
#pragma unroll
    for (int e = 0; e < C::EY; ++e) {
#pragma unroll
        for (int v = 0; v < C::VEC; ++v) {
            if (g.rin[e] && g.gx + v < s.nx) {
                const int cidx = (g.gy + e) * s.nx + g.gx + v;
                const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
                if (lo < hi) {
                    const int p = lower_bound_z(s.ev, lo, hi, z);
                    if (p < hi) nxt = min(nxt, s.ev[p].z);
                }
            }
        }
    }
    return nxt;
}

// ------------------------------------------------------------------ forward step

// Byte address of element byte-offset `ob` inside plane z of a padded field whose
// first ghost plane starts at `base` (plane pitch pxy elements).  The plane base is
// uniform across the workgroup, the in-plane offset is a 32-bit per-lane value.
template <typename T>
__device__ __forceinline__ const T *plane_at(const T *base, int64_t pxy, int zp, uint32_t ob)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base + (int64_t)zp * pxy) + ob);
}
template <typename T>
__device__ __forceinline__ T *plane_at(T *base, int64_t pxy, int zp, uint32_t ob)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base + (int64_t)zp * pxy) + ob);
}

// One leapfrog step over this workgroup's tile and z chunk.
//
// The z register queue has P = 2R+2 slots: planes z-R .. z+R of the current plane
// z plus one slot receiving plane z+R+1 while z is computed; it shifts by one slot
// per plane.  (Unrolling the plane loop by P to rotate the queue instead removes the
// register moves but multiplies the code size, and measured slower on gfx950.)
//
// Halo timing: the x/y halo of a plane is interior data of the neighbouring tiles.
// With HOFF = R the halo of plane z+R+1 is fetched in the same iteration in which
// the neighbours fetch that plane as their queue tail, so the requests meet in L2,
// and it waits in a ring of NB = R+2 LDS plane buffers until the plane becomes the
// centre.  (Fetching it only when it is needed comes R planes later, by which time
// the XCD has streamed several MB and the lines have left its 4 MB L2.)  Plane p
// lives in buffer p mod NB: when iteration z writes the halo of plane z+R its buffer
// was last read by iteration z-2, and every thread passed the barrier of z-1.
//
// The plane loop is unrolled by 2 (static_for) so that the u^{n-1}, c and halo
// prefetch registers alternate between two sets by parity.
template <class C>
__device__ __forceinline__ void fwd_tile(const ShotDesc &s, const typename C::type *__restrict__ cur,
                                         const typename C::type *prev, typename C::type *out,
                                         int64_t step, bool record, int tx, int ty, int cz,
                                         typename C::type *lds)
{
    typedef typename C::type T;
    constexpr int R = C::R, VEC = C::VEC, EY = C::EY, HPT = C::HPT, HY = C::HY;
    constexpr int P = 2 * R + 2;
    constexpr int HOFF = C::HOFF, NB = C::NB;
    constexpr StencilWeights<R> W{};
    const T *__restrict__ cc = static_cast<const T *>(s.c);
    const int64_t pxy = s.pxy;

    TileGeom<C> g;
    g.init(s, tx, ty, cz, s.zch);
    if (g.z0 >= g.z1) return;

    // in-plane byte offsets (plane index zp = z + R counts the R ghost planes)
    const int64_t colp = g.col - (int64_t)R * pxy;
    uint32_t ob[EY];
#pragma unroll
    for (int e = 0; e < EY; ++e) ob[e] = (uint32_t)((colp + (int64_t)e * s.px) * (int64_t)sizeof(T));
    uint32_t hob[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) hob[k] = (uint32_t)((g.hoff[k] - (int64_t)R * pxy) * (int64_t)sizeof(T));

    // LEAN: one register set for the u^{n-1}, c and halo prefetches (the next plane's
    // values are loaded into it once the current plane is done with it) instead of two
    constexpr bool LEAN = C::OCC > 0;
    constexpr int NSET = LEAN ? 1 : 2;
    T q[P][EY][VEC];
    T pv[NSET][EY][VEC], cv[NSET][EY][VEC], hv[NSET][HPT][VEC];

    // prologue: planes z0-R .. z0+R into slots 0 .. 2R; u^{n-1} and c of plane z0 into
    // set 0; halos of planes z0 .. z0+HOFF-1 straight into their LDS buffers and the
    // halo of plane z0+HOFF into set 0
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k)
#pragma unroll
        for (int e = 0; e < EY; ++e) {
            if (g.lin[e])
                vld(q[k][e], plane_at(cur, pxy, g.z0 + k, ob[e]));
            else
                vzero(q[k][e]);
        }
#pragma unroll
    for (int e = 0; e < EY; ++e) {
        if (g.rin[e]) {
            vld_nt(pv[0][e], plane_at(prev, pxy, g.z0 + R, ob[e]));
            vld_nt(cv[0][e], plane_at(cc, pxy, g.z0 + R, ob[e]));
        } else {
            vzero(pv[0][e]);
            vzero(cv[0][e]);
        }
    }
#pragma unroll
    for (int j = 0; j < HOFF; ++j) {
        if (g.z0 + j < g.z1) {
            T *L = lds + ((g.z0 + j) % NB) * C::LDS;
#pragma unroll
            for (int k = 0; k < HPT; ++k)
                if (g.hval[k]) {
                    T t[VEC];
                    vld(t, plane_at(cur, pxy, g.z0 + j + R, hob[k]));
                    vst(L + g.hl[k], t);
                }
        }
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        if (g.hval[k] && g.z0 + HOFF < g.z1)
            vld(hv[0][k], plane_at(cur, pxy, g.z0 + HOFF + R, hob[k]));
        else
            vzero(hv[0][k]);
    }
    int nev = next_event<C>(s, g, g.z0);
    int bz = g.z0 % NB;              // LDS buffer of plane z
    int bh = (g.z0 + HOFF) % NB;     // LDS buffer of plane z + HOFF

    // absorbing sponge: G = gx gy gz scales both time levels (1 outside the sponge)
    const T *__restrict__ damp = static_cast<const T *>(s.damp);
    T gxy[EY][VEC];
    if (damp) {
#pragma unroll
        for (int e = 0; e < EY; ++e)
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                gxy[e][v] = (g.rin[e] && g.gx + v < s.nx) ? damp[g.gx + v] * damp[s.nx + g.gy + e] : T(1);
    }

    for (int zb = g.z0; zb < g.z1; zb += 2) {
        static_for<2>([&](auto st_) __attribute__((always_inline)) {
            constexpr int st = decltype(st_)::value;
            constexpr int cs = LEAN ? 0 : (st & 1), ns = LEAN ? 0 : (cs ^ 1);
            constexpr int tail = 2 * R + 1;  // slot receiving plane z+R+1
            constexpr int ctr = R;           // slot of plane z
            const int z = zb + st;
            if (z >= g.z1) return;
            if (z + 1 < g.z1) {
#pragma unroll
                for (int e = 0; e < EY; ++e) {
                    if (g.lin[e]) vld(q[tail][e], plane_at(cur, pxy, z + 1 + 2 * R, ob[e]));
                    if (!LEAN && g.rin[e]) {
                        vld_nt(pv[ns][e], plane_at(prev, pxy, z + 1 + R, ob[e]));
                        vld_nt(cv[ns][e], plane_at(cc, pxy, z + 1 + R, ob[e]));
                    }
                }
            }
            if (!LEAN && z + 1 + HOFF < g.z1) {
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    if (g.hval[k]) vld(hv[ns][k], plane_at(cur, pxy, z + 1 + HOFF + R, hob[k]));
            }

            // stage plane z's interior (from the queue) and plane z+HOFF's halo in LDS
            T *L = lds + bz * C::LDS;
#pragma unroll
            for (int e = 0; e < EY; ++e) vst(L + (g.ly + e + HY) * C::LW + C::LPAD + g.lx, q[ctr][e]);
            if (z + HOFF < g.z1) {
                T *LH = lds + bh * C::LDS;
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    if (g.hval[k]) vst(LH + g.hl[k], hv[cs][k]);
            }
            if (LEAN && z + 1 + HOFF < g.z1) {  // the next halo, into the registers just staged
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    if (g.hval[k]) vld(hv[0][k], plane_at(cur, pxy, z + 1 + HOFF + R, hob[k]));
            }
            __syncthreads();

            // y neighbour rows: yr[k] is row ly - HY + k at this thread's x vector
            T yr[C::YR][VEC];
#pragma unroll
            for (int k = 0; k < C::YR; ++k) {
                if (k >= HY && k < HY + EY) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) yr[k][v] = q[ctr][k - HY][v];
                } else {
                    vld(yr[k], L + (g.ly + k) * C::LW + C::LPAD + g.lx);
                }
            }

            T un[EY][VEC];
#pragma unroll
            for (int e = 0; e < EY; ++e) {
                T xs[C::NXV * VEC];
#pragma unroll
                for (int j = 0; j < C::NXV; ++j) {
                    T tmp[VEC];
                    vld(tmp, L + (g.ly + e + HY) * C::LW + g.lx + j * VEC);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) xs[j * VEC + v] = tmp[v];
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T u0 = q[ctr][e][v];
                    T acc;
                    if constexpr (R > 4) {
                        acc = T(C::NDIM * W.w[0]) * u0;
#pragma unroll
                        for (int l = 1; l <= R; ++l) acc = fma_t(T(W.w[l]), xs[C::LPAD + v + l] + xs[C::LPAD + v - l], acc);
                        if (C::NDIM == 3) {
#pragma unroll
                            for (int l = 1; l <= R; ++l) acc = fma_t(T(W.w[l]), yr[HY + e + l][v] + yr[HY + e - l][v], acc);
                        }
#pragma unroll
                        for (int l = 1; l <= R; ++l) acc = fma_t(T(W.w[l]), q[R + l][e][v] + q[R - l][e][v], acc);
                    } else {
                        acc = T(0);
#pragma unroll
                        for (int l = 1; l <= R; ++l)
                            acc = fma_t(T(W.w[l]), (xs[C::LPAD + v + l] - u0) + (xs[C::LPAD + v - l] - u0), acc);
                        if (C::NDIM == 3) {
#pragma unroll
                            for (int l = 1; l <= R; ++l)
                                acc = fma_t(T(W.w[l]), (yr[HY + e + l][v] - u0) + (yr[HY + e - l][v] - u0), acc);
                        }
#pragma unroll
                        for (int l = 1; l <= R; ++l)
                            acc = fma_t(T(W.w[l]), (q[R + l][e][v] - u0) + (q[R - l][e][v] - u0), acc);
                    }
                    if (damp) {
                        const T G = gxy[e][v] * damp[s.nx + s.ny + z];
                        un[e][v] = G * fma_t(cv[cs][e][v], acc, T(2) * u0 - G * pv[cs][e][v]);
                    } else {
                        un[e][v] = fma_t(cv[cs][e][v], acc, T(2) * u0 - pv[cs][e][v]);
                    }
                }
            }

            if (LEAN && z + 1 < g.z1) {  // u^{n-1} and c of the next plane, into the registers just used
#pragma unroll
                for (int e = 0; e < EY; ++e)
                    if (g.rin[e]) {
                        vld_nt(pv[0][e], plane_at(prev, pxy, z + 1 + R, ob[e]));
                        vld_nt(cv[0][e], plane_at(cc, pxy, z + 1 + R, ob[e]));
                    }
            }

            // fused sources (added before the store) and receivers (recorded after them)
            if (z == nev) {
                int nxt = 0x7fffffff;
#pragma unroll
                for (int e = 0; e < EY; ++e) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        if (g.rin[e] && g.gx + v < s.nx) {
                            const int cidx = (g.gy + e) * s.nx + g.gx + v;
                            const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
                            if (lo < hi) {
                                int p = lower_bound_z(s.ev, lo, hi, z);
                                for (; p < hi && s.ev[p].z == z; ++p) {
                                    const int code = s.ev[p].code;
                                    if (code < 0) {
                                        const SourceInfo si = s.src[~code];
                                        if (step < si.nsamp)
                                            un[e][v] += T(si.scale) * static_cast<const T *>(si.wav)[step];
                                    } else if (record) {
                                        const int64_t row = step - s.rec_base;
                                        if (row >= 0 && row < s.rec_cap)
                                            static_cast<T *>(s.traces)[row * s.nrec + code] = un[e][v];
                                    }
                                }
                                if (p < hi) nxt = min(nxt, s.ev[p].z);
                            }
                        }
                    }
                }
                nev = nxt;
            }

#pragma unroll
            for (int e = 0; e < EY; ++e) {
                if (g.rin[e]) {
                    T *p = plane_at(out, pxy, z + R, ob[e]);
                    if (g.gx + VEC <= s.nx) {
                        vst_nt(p, un[e]);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v)
                            if (g.gx + v < s.nx) p[v] = un[e][v];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < P - 1; ++k)
#pragma unroll
                for (int e = 0; e < EY; ++e)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) q[k][e][v] = q[k + 1][e][v];
            bz = (bz + 1 == NB) ? 0 : bz + 1;
            bh = (bh + 1 == NB) ? 0 : bh + 1;
        });
    }
}

template <class C>
__device__ __forceinline__ void fwd_body(LaunchArgs a);

template <class C>
__global__ __launch_bounds__(C::NT) void fwd_kernel(LaunchArgs a)
{
    fwd_body<C>(a);
}

// the same step built for C::OCC waves per SIMD
template <class C>
__global__ __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(C::OCC > 0 ? C::OCC : 1)))
void fwd_kernel_occ(LaunchArgs a)
{
    fwd_body<C>(a);
}

template <class C>
__device__ __forceinline__ void fwd_body(LaunchArgs a)
{
    typedef typename C::type T;
    __shared__ __attribute__((aligned(16))) T lds[C::NB * C::LDS];
    int wg = blockIdx.x;
    if (a.xcd_remap) wg = xcd_remap(wg, (int)gridDim.x);
    int shot = 0, local = wg;
    if (a.nshots > 1) {
        int lo = 0, hi = a.nshots;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.wg_prefix[mid] <= wg)
                lo = mid;
            else
                hi = mid;
        }
        shot = lo;
        local = wg - a.wg_prefix[lo];
    }
    ShotDesc *sp = a.shots + shot;
    int64_t step;
    if (a.step >= 0) {
        step = a.step;
    } else {
        step = sp->ctr[a.slot];
        const bool active = step < sp->target;
        if (local == 0 && threadIdx.x == 0) sp->ctr[a.slot ^ 1] = active ? step + 1 : step;
        if (!active) return;
    }
    const ShotDesc &s = *sp;
    const T *cur;
    const T *prev;
    T *out;
    if (a.cur) {
        cur = static_cast<const T *>(a.cur);
        prev = static_cast<const T *>(a.prev);
        out = static_cast<T *>(a.out);
    } else {
        cur = static_cast<const T *>(s.buf[step & 1]);
        prev = static_cast<const T *>(s.buf[(step + 1) & 1]);
        out = static_cast<T *>(s.buf[(step + 1) & 1]);
    }
    const int tx = local % s.tiles_x;
    const int t2 = local / s.tiles_x;
    const int ty = t2 % s.tiles_y;
    const int cz = t2 / s.tiles_y;
    if (cz >= s.chunks_z) return;
    fwd_tile<C>(s, cur, prev, out, step, a.record != 0, tx, ty, cz, lds);
}

// ------------------------------------------------------------------ adjoint step

// One step of the discrete adjoint in the variable mu = c * lambda, fused with the
// imaging condition:
//     mu^k = 2 mu^{k+1} - mu^{k+2} + c Lh mu^{k+1} + resid_amp c_j resid[k-1][j] e_j
//     t    = mu^k * Lh u^{k-1}
// Two register queues (mu^{k+1}, u^{k-1}) march in z together; both planes are
// staged in LDS.  The imaging term t is summed in the working precision, blocked by
// checkpoint segment so that the rounding error grows with the segment length plus
// the number of segments instead of with the number of steps:
//     gmode 0: gseg += t         (inside a segment)
//     gmode 1: gseg  = t         (first step of a segment)
//     gmode 2: g    += gseg + t  (last step of a segment)
//     gmode 3: g    += t         (unblocked)
enum { GM_ACC = 0, GM_FIRST = 1, GM_FOLD = 2, GM_DIRECT = 3 };
template <class C>
__device__ __forceinline__ void adj_tile(const ShotDesc &s, const typename C::type *__restrict__ mcur,
                                         typename C::type *mout, const typename C::type *__restrict__ ucur,
                                         typename C::type *grad, typename C::type *gseg, int gmode,
                                         const typename C::type *__restrict__ resid,
                                         int64_t k, typename C::type ramp, int tx, int ty, int cz, int zch,
                                         typename C::type *lds)
{
    typedef typename C::type T;
    constexpr int R = C::R, VEC = C::VEC, EY = C::EY, HPT = C::HPT, HY = C::HY;
    constexpr StencilWeights<R> W{};
    const T *__restrict__ cc = static_cast<const T *>(s.c);
    const int64_t px = s.px, pxy = s.pxy;

    TileGeom<C> g;
    g.init(s, tx, ty, cz, zch);
    if (g.z0 >= g.z1) return;

    // imaging accumulator: g1 (added through the FMA), g2 (added after it), gout (stored)
    const T *g1 = gmode == GM_ACC ? gseg : (gmode == GM_FOLD ? gseg : (gmode == GM_DIRECT ? grad : nullptr));
    const T *g2 = gmode == GM_FOLD ? grad : nullptr;
    T *gout = (gmode == GM_ACC || gmode == GM_FIRST) ? gseg : grad;

    T qm[2 * R + 1][EY][VEC], qu[2 * R + 1][EY][VEC];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j)
#pragma unroll
        for (int e = 0; e < EY; ++e) {
            if (g.lin[e]) {
                vld(qm[j][e], mcur + g.col + e * px + (int64_t)(g.z0 - R + j) * pxy);
                vld(qu[j][e], ucur + g.col + e * px + (int64_t)(g.z0 - R + j) * pxy);
            } else {
                vzero(qm[j][e]);
                vzero(qu[j][e]);
            }
        }
    T nm[EY][VEC], nuu[EY][VEC], npv[EY][VEC], ncc[EY][VEC], ngr[EY][VEC], ng2[EY][VEC], nhm[HPT][VEC],
        nhu[HPT][VEC];
    {
        const int64_t zo = (int64_t)g.z0 * pxy;
#pragma unroll
        for (int e = 0; e < EY; ++e) {
            if (g.lin[e]) {
                vld(nm[e], mcur + g.col + e * px + zo + R * pxy);
                vld(nuu[e], ucur + g.col + e * px + zo + R * pxy);
            } else {
                vzero(nm[e]);
                vzero(nuu[e]);
            }
            vzero(ngr[e]);
            vzero(ng2[e]);
            if (g.rin[e]) {
                vld_nt(npv[e], mout + g.col + e * px + zo);
                vld_nt(ncc[e], cc + g.col + e * px + zo);
                if (g1) vld_nt(ngr[e], g1 + g.col + e * px + zo);
                if (g2) vld_nt(ng2[e], g2 + g.col + e * px + zo);
            } else {
                vzero(npv[e]);
                vzero(ncc[e]);
            }
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (g.hval[j]) {
                vld(nhm[j], mcur + g.hoff[j] + zo);
                vld(nhu[j], ucur + g.hoff[j] + zo);
            } else {
                vzero(nhm[j]);
                vzero(nhu[j]);
            }
        }
    }
    int nev = next_event<C>(s, g, g.z0);

    int buf = 0;
    for (int z = g.z0; z < g.z1; ++z) {
        T pv[EY][VEC], cv[EY][VEC], gv[EY][VEC], gv2[EY][VEC], hm[HPT][VEC], hu[HPT][VEC];
#pragma unroll
        for (int e = 0; e < EY; ++e)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                qm[2 * R][e][v] = nm[e][v];
                qu[2 * R][e][v] = nuu[e][v];
                pv[e][v] = npv[e][v];
                cv[e][v] = ncc[e][v];
                gv[e][v] = ngr[e][v];
                gv2[e][v] = ng2[e][v];
            }
#pragma unroll
        for (int j = 0; j < HPT; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                hm[j][v] = nhm[j][v];
                hu[j][v] = nhu[j][v];
            }
        if (z + 1 < g.z1) {
            const int64_t zo = (int64_t)(z + 1) * pxy;
#pragma unroll
            for (int e = 0; e < EY; ++e) {
                if (g.lin[e]) {
                    vld(nm[e], mcur + g.col + e * px + zo + R * pxy);
                    vld(nuu[e], ucur + g.col + e * px + zo + R * pxy);
                }
                if (g.rin[e]) {
                    vld_nt(npv[e], mout + g.col + e * px + zo);
                    vld_nt(ncc[e], cc + g.col + e * px + zo);
                    if (g1) vld_nt(ngr[e], g1 + g.col + e * px + zo);
                    if (g2) vld_nt(ng2[e], g2 + g.col + e * px + zo);
                }
            }
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                if (g.hval[j]) {
                    vld(nhm[j], mcur + g.hoff[j] + zo);
                    vld(nhu[j], ucur + g.hoff[j] + zo);
                }
        }

        T *Lm = lds + buf * (2 * C::LDS);
        T *Lu = Lm + C::LDS;
#pragma unroll
        for (int e = 0; e < EY; ++e) {
            vst(Lm + (g.ly + e + HY) * C::LW + C::LPAD + g.lx, qm[R][e]);
            vst(Lu + (g.ly + e + HY) * C::LW + C::LPAD + g.lx, qu[R][e]);
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (g.hval[j]) {
                vst(Lm + g.hl[j], hm[j]);
                vst(Lu + g.hl[j], hu[j]);
            }
        __syncthreads();

        T mnew[EY][VEC], lapu[EY][VEC];
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const T *Lp = pass == 0 ? Lm : Lu;
            T yr[C::YR][VEC];
#pragma unroll
            for (int j = 0; j < C::YR; ++j) {
                if (j >= HY && j < HY + EY) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) yr[j][v] = pass == 0 ? qm[R][j - HY][v] : qu[R][j - HY][v];
                } else {
                    vld(yr[j], Lp + (g.ly + j) * C::LW + C::LPAD + g.lx);
                }
            }
#pragma unroll
            for (int e = 0; e < EY; ++e) {
                T xs[C::NXV * VEC];
#pragma unroll
                for (int j = 0; j < C::NXV; ++j) {
                    T tmp[VEC];
                    vld(tmp, Lp + (g.ly + e + HY) * C::LW + g.lx + j * VEC);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) xs[j * VEC + v] = tmp[v];
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T u0 = pass == 0 ? qm[R][e][v] : qu[R][e][v];
                    T acc = T(0);
#pragma unroll
                    for (int l = 1; l <= R; ++l)
                        acc = fma_t(T(W.w[l]), (xs[C::LPAD + v + l] - u0) + (xs[C::LPAD + v - l] - u0), acc);
                    if (C::NDIM == 3) {
#pragma unroll
                        for (int l = 1; l <= R; ++l)
                            acc = fma_t(T(W.w[l]), (yr[HY + e + l][v] - u0) + (yr[HY + e - l][v] - u0), acc);
                    }
#pragma unroll
                    for (int l = 1; l <= R; ++l) {
                        const T zp = pass == 0 ? qm[R + l][e][v] : qu[R + l][e][v];
                        const T zm = pass == 0 ? qm[R - l][e][v] : qu[R - l][e][v];
                        acc = fma_t(T(W.w[l]), (zp - u0) + (zm - u0), acc);
                    }
                    if (pass == 0)
                        mnew[e][v] = fma_t(cv[e][v], acc, T(2) * u0 - pv[e][v]);
                    else
                        lapu[e][v] = acc;
                }
            }
        }

        // adjoint sources: the residual enters at the receivers, scaled by c there
        if (z == nev) {
            int nxt = 0x7fffffff;
#pragma unroll
            for (int e = 0; e < EY; ++e) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    if (g.rin[e] && g.gx + v < s.nx) {
                        const int cidx = (g.gy + e) * s.nx + g.gx + v;
                        const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
                        if (lo < hi) {
                            int p = lower_bound_z(s.ev, lo, hi, z);
                            for (; p < hi && s.ev[p].z == z; ++p) {
                                const int code = s.ev[p].code;
                                if (code >= 0)
                                    mnew[e][v] = fma_t(ramp * cv[e][v], resid[(k - 1) * s.nrec + code], mnew[e][v]);
                            }
                            if (p < hi) nxt = min(nxt, s.ev[p].z);
                        }
                    }
                }
            }
            nev = nxt;
        }

#pragma unroll
        for (int e = 0; e < EY; ++e) {
            T gn[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                gn[v] = fma_t(mnew[e][v], lapu[e][v], gv[e][v]);
                if (g2) gn[v] = gn[v] + gv2[e][v];
            }
            if (g.rin[e]) {
                T *pm = mout + g.col + e * px + (int64_t)z * pxy;
                T *pg = gout + g.col + e * px + (int64_t)z * pxy;
                if (g.gx + VEC <= s.nx) {
                    vst_nt(pm, mnew[e]);
                    vst_nt(pg, gn);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        if (g.gx + v < s.nx) {
                            pm[v] = mnew[e][v];
                            pg[v] = gn[v];
                        }
                }
            }
        }

#pragma unroll
        for (int j = 0; j < 2 * R; ++j)
#pragma unroll
            for (int e = 0; e < EY; ++e)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    qm[j][e][v] = qm[j + 1][e][v];
                    qu[j][e][v] = qu[j + 1][e][v];
                }
        buf ^= 1;
    }
}

template <class C>
__global__ __launch_bounds__(C::NT) void adj_kernel(AdjArgs a)
{
    typedef typename C::type T;
    __shared__ __attribute__((aligned(16))) T lds[4 * C::LDS];
    int wg = blockIdx.x;
    if (a.xcd_remap) wg = xcd_remap(wg, (int)gridDim.x);
    const ShotDesc &s = *a.shot;
    const int tx = wg % a.tiles_x;
    const int t2 = wg / a.tiles_x;
    const int ty = t2 % a.tiles_y;
    const int cz = t2 / a.tiles_y;
    if (cz >= a.chunks_z) return;
    adj_tile<C>(s, static_cast<const T *>(a.mu_cur), static_cast<T *>(a.mu_out),
                static_cast<const T *>(a.u_km1), static_cast<T *>(a.grad), static_cast<T *>(a.gseg), a.gmode,
                static_cast<const T *>(a.resid), a.k, T(a.resid_amp), tx, ty, cz, a.zch, lds);
}

// ------------------------------------------------------------------ registry

// Roles of a forward tile entry: an option for fd_set_tuning, or the one the library
// takes by itself for grids whose default z chunk is short (many short chunks: more
// resident waves pay off there).
enum { FWD_OPTION = 0, FWD_SMALL_GRID = 1 };

struct FwdEntry {
    const char *name;
    int bx, by, nt;
    void (*launch)(const LaunchArgs &, int nwg, hipStream_t);
    const void *kernel;  // the __global__ function (for occupancy queries)
    int role;
};

// role of an adjoint table entry: an option for fd_set_adj_tuning, or the build that
// fd_create takes by itself for grids whose rows the default tile fits badly
enum { ADJ_OPTION = 0, ADJ_RAGGED_X = 1 };

struct AdjEntry {
    const char *name;
    int bx, by, nt;
    void (*launch)(const AdjArgs &, int nwg, hipStream_t);
    const void *kernel;
    int role;
};

template <class C>
void launch_fwd(const LaunchArgs &a, int nwg, hipStream_t st)
{
    if constexpr (C::OCC > 0)
        hipLaunchKernelGGL(fwd_kernel_occ<C>, dim3(nwg), dim3(C::NT), 0, st, a);
    else
        hipLaunchKernelGGL(fwd_kernel<C>, dim3(nwg), dim3(C::NT), 0, st, a);
}

template <class C>
void launch_adj(const AdjArgs &a, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(adj_kernel<C>, dim3(nwg), dim3(C::NT), 0, st, a);
}

template <class C>
FwdEntry fwd_entry(const char *name, int role = FWD_OPTION)
{
    const void *k;
    if constexpr (C::OCC > 0)
        k = reinterpret_cast<const void *>(&fwd_kernel_occ<C>);
    else
        k = reinterpret_cast<const void *>(&fwd_kernel<C>);
    return FwdEntry{name, C::BX, C::BY, C::NT, &launch_fwd<C>, k, role};
}

template <class C>
AdjEntry adj_entry(const char *name, int role = ADJ_OPTION)
{
    return AdjEntry{name, C::BX, C::BY, C::NT, &launch_adj<C>, reinterpret_cast<const void *>(&adj_kernel<C>), role};
}

// Implemented in the per-dtype translation units.
const FwdEntry *fwd_configs_f32(int r, int ndim, int *count);
const FwdEntry *fwd_configs_f64(int r, int ndim, int *count);
const AdjEntry *adj_configs_f32(int r, int ndim, int *count);
const AdjEntry *adj_configs_f64(int r, int ndim, int *count);

}  // namespace fdw
