// fd_fwd2.h -- two leapfrog steps per launch (temporal blocking) for the 3-D forward.
//
// One launch takes (u^n, u^{n-1}) to (u^{n+1}, u^{n+2}) and writes both into two
// buffers other than its inputs: u^{n+1} is needed at the next launch as the previous
// level, and neither input may be overwritten while neighbouring workgroups still read
// its halo.  Per grid point and two time steps it moves 20 bytes (read u^n, u^{n-1},
// c; write u^{n+1}, u^{n+2}) instead of the 32 of two single steps.
//
// Per workgroup, for a BX x BY output tile and a z chunk [z0, z1):
//  - level 1 (u^{n+1}) is computed on the tile widened by R on each side (E), for
//    planes z0-R .. z1+R-1, so that level 2 has all its neighbours: the tile's own
//    columns ("A", one vector per thread) and the R-wide ring ("B", at most one vector
//    per thread);
//  - level 0 (u^n) is staged per plane in LDS over the tile widened by 2R (the ring of
//    E, plus an outer ring "O" loaded for the x/y neighbours of E); the z neighbours of
//    the A columns come from a register queue of 2R+2 planes, those of the B columns
//    from a per-thread ring of 2R+2 planes in LDS (registers would spill);
//  - level 1 of each plane is staged in LDS over E; its x/y part of the level-2 sum is
//    formed at once and kept in a ring of R+1 planes, its z part comes from a register
//    queue of 2R+1 level-1 planes, and level 2 of plane z-R is finished R planes later.
// Every point value is computed by the same operations in the same order as the
// single-step kernel (x, then y, then z neighbour pairs in one FMA chain; the same
// update and source/receiver handling), so the result is bitwise that of two single
// steps.  Zero values outside the grid hold for both levels: ring columns outside the
// grid and planes outside [0, nz) are set to zero, never computed.
#pragma once

#include "fd_stencil.h"

namespace fdw {

template <typename T, int R_, int TXN_, int TYN_>
struct Tile2Cfg {
    typedef T type;
    static constexpr int R = R_;
    static constexpr int TXN = TXN_;
    static constexpr int TYN = TYN_;
    static constexpr int VEC = V16<T>::N;
    static constexpr int NT = TXN * TYN;
    static constexpr int BX = TXN * VEC;
    static constexpr int BY = TYN;
    static_assert(R % VEC == 0, "ring columns must be whole vectors");
    static constexpr int RV = R / VEC;
    static constexpr int EW = BX + 2 * R, EH = BY + 2 * R;        // level-1 region E
    static constexpr int EWV = EW / VEC;
    static constexpr int NBV = (EW * EH - BX * BY) / VEC;          // ring (B) vectors
    static constexpr int W0 = BX + 4 * R, H0 = BY + 4 * R;        // level-0 region
    static constexpr int W0V = W0 / VEC;
    static constexpr int NOV = (W0 * H0 - EW * EH) / VEC;          // outer ring (O) vectors
    static constexpr int NXV = 2 * RV + 1;                         // vectors for x neighbours
    static_assert(NBV <= NT && NOV <= NT, "at most one ring and one outer vector per thread");
    static constexpr int QSL = 2 * R + 2;                          // planes in the B ring
    static_assert(256 % BX == 0 && 64 % BY == 0, "tile must divide the layout alignment");
};

struct Fwd2Args {
    const ShotDesc *shot;
    const void *cur;   // u^n
    const void *prev;  // u^{n-1}
    void *out1;        // u^{n+1}
    void *out2;        // u^{n+2}
    int64_t step;      // n
    int32_t zch, tiles_x, tiles_y, chunks_z, xcd_remap, pad0;
};

// Sum of the x and y neighbour pairs (difference form) of the value u0 at LDS row
// `row`, column `col` of a plane of width W: the first two parts of the FMA chain of
// the single-step kernel.
template <class C, int W>
__device__ __forceinline__ void xy_pairs(const typename C::type *L, int row, int col,
                                         const typename C::type (&u0)[C::VEC], typename C::type (&acc)[C::VEC])
{
    typedef typename C::type T;
    constexpr int R = C::R, VEC = C::VEC;
    constexpr StencilWeights<R> Wt{};
    T xs[C::NXV * VEC];
#pragma unroll
    for (int j = 0; j < C::NXV; ++j) {
        T tmp[VEC];
        vld(tmp, L + row * W + col - R + j * VEC);
#pragma unroll
        for (int v = 0; v < VEC; ++v) xs[j * VEC + v] = tmp[v];
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        T a = T(0);
#pragma unroll
        for (int l = 1; l <= R; ++l) a = fma_t(T(Wt.w[l]), (xs[R + v + l] - u0[v]) + (xs[R + v - l] - u0[v]), a);
        acc[v] = a;
    }
#pragma unroll
    for (int l = 1; l <= R; ++l) {
        T up[VEC], dn[VEC];
        vld(up, L + (row - l) * W + col);
        vld(dn, L + (row + l) * W + col);
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = fma_t(T(Wt.w[l]), (dn[v] - u0[v]) + (up[v] - u0[v]), acc[v]);
    }
}

// Events (sources, receivers) of one vector of columns at plane z: sources add
// scale * wav[sample] to val, receivers (if rec_row >= 0) record val after them.
template <class C>
__device__ __forceinline__ int vec_events(const ShotDesc &s, int gx, int gy, bool inside, int z, int64_t sample,
                                          int64_t rec_row, typename C::type (&val)[C::VEC])
{
    typedef typename C::type T;
    int nxt = 0x7fffffff;
    if (!inside) return nxt;
#pragma unroll
    for (int v = 0; v < C::VEC; ++v) {
        if (gx + v < s.nx) {
            const int cidx = gy * s.nx + gx + v;
            const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
            if (lo < hi) {
                int p = lower_bound_z(s.ev, lo, hi, z);
                for (; p < hi && s.ev[p].z == z; ++p) {
                    const int code = s.ev[p].code;
                    if (code < 0) {
                        const SourceInfo si = s.src[~code];
                        if (sample < si.nsamp) val[v] += T(si.scale) * static_cast<const T *>(si.wav)[sample];
                    } else if (rec_row >= 0 && rec_row < s.rec_cap) {
                        static_cast<T *>(s.traces)[rec_row * s.nrec + code] = val[v];
                    }
                }
                if (p < hi) nxt = min(nxt, s.ev[p].z);
            }
        }
    }
    return nxt;
}

template <class C>
__device__ __forceinline__ int vec_next_event(const ShotDesc &s, int gx, int gy, bool inside, int z)
{
    int nxt = 0x7fffffff;
    if (!inside || !s.ev_ptr) return nxt;
#pragma unroll
    for (int v = 0; v < C::VEC; ++v) {
        if (gx + v < s.nx) {
            const int cidx = gy * s.nx + gx + v;
            const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
            if (lo < hi) {
                const int p = lower_bound_z(s.ev, lo, hi, z);
                if (p < hi) nxt = min(nxt, s.ev[p].z);
            }
        }
    }
    return nxt;
}

template <class C>
__device__ __forceinline__ void fwd2_tile(const ShotDesc &s, const Fwd2Args &a, int tx, int ty, int cz,
                                          typename C::type *L0, typename C::type *L1, typename C::type *LQ)
{
    typedef typename C::type T;
    constexpr int R = C::R, VEC = C::VEC, P = 2 * R + 2, Q = 2 * R + 1;
    constexpr StencilWeights<R> Wt{};
    const T *__restrict__ cur = static_cast<const T *>(a.cur);
    const T *__restrict__ prev = static_cast<const T *>(a.prev);
    const T *__restrict__ cc = static_cast<const T *>(s.c);
    T *out1 = static_cast<T *>(a.out1);
    T *out2 = static_cast<T *>(a.out2);
    const int64_t pxy = s.pxy, px = s.px;
    const int rows = (int)(pxy / px);  // padded rows per plane: y in [-R, rows - R)
    const int64_t n = a.step;

    const int tid = threadIdx.x;
    const int x0 = tx * C::BX, y0 = ty * C::BY;
    const int z0 = cz * a.zch;
    const int z1 = min(z0 + a.zch, s.nz);
    if (z0 >= z1) return;  // uniform

    // A: this thread's vector of the tile
    const int ax = (tid % C::TXN) * VEC, ay = tid / C::TXN;
    const int agx = x0 + ax, agy = y0 + ay;
    const bool ain = agx < s.nx && agy < s.ny;
    // B: ring vector of E (top/bottom full rows of E, then R rows' left and right blocks)
    const bool hasb = tid < C::NBV;
    int bex = 0, bey = 0;
    {
        constexpr int NTB = 2 * R * C::EWV;
        if (tid < NTB) {
            const int row = tid / C::EWV;
            bey = row < R ? row : row + C::BY;
            bex = (tid % C::EWV) * VEC;
        } else {
            const int bs = tid - NTB;
            bey = R + bs / (2 * C::RV);
            const int side = bs % (2 * C::RV);
            bex = (side < C::RV ? side : C::EWV - 2 * C::RV + side) * VEC;
        }
    }
    const int bgx = x0 - R + bex, bgy = y0 - R + bey;  // grid coordinates of the B vector
    // B vector lanes inside the grid (both coordinates); the vector never straddles x = 0
    const bool bin = hasb && bgx >= 0 && bgx < s.nx && bgy >= 0 && bgy < s.ny;
    // O: outer-ring vector of the level-0 region
    const bool haso = tid < C::NOV;
    int oex = 0, oey = 0;
    {
        constexpr int NTO = 2 * R * C::W0V;
        if (tid < NTO) {
            const int row = tid / C::W0V;
            oey = row < R ? row : row + C::EH;
            oex = (tid % C::W0V) * VEC;
        } else {
            const int os = tid - NTO;
            oey = R + os / (2 * C::RV);
            const int side = os % (2 * C::RV);
            oex = (side < C::RV ? side : C::W0V - 2 * C::RV + side) * VEC;
        }
    }
    const int ogx = x0 - 2 * R + oex, ogy = y0 - 2 * R + oey;
    // rows outside [-R, rows - R) are not stored: their values are zero
    const bool oload = haso && ogy >= -R && ogy < rows - R;

    // in-plane byte offsets (plane index zp = z + R counts the R ghost planes)
    const int64_t base = s.off0 - (int64_t)R * pxy;
    const uint32_t oba = (uint32_t)((base + (int64_t)agy * px + agx) * (int64_t)sizeof(T));
    const uint32_t obb = hasb ? (uint32_t)((base + (int64_t)bgy * px + bgx) * (int64_t)sizeof(T)) : oba;
    const uint32_t obo = oload ? (uint32_t)((base + (int64_t)ogy * px + ogx) * (int64_t)sizeof(T)) : oba;

    // lane masks of computed level-1 values (outside the grid level 1 is zero)
    bool amask[VEC], bmask[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        amask[v] = ain && agx + v < s.nx;
        bmask[v] = bin && bgx + v < s.nx;
    }

    T qa[P][VEC];                   // level 0 at planes z-R .. z+R (+ the tail z+R+1), A column
    T qbt[2][VEC];                  // B column: the plane in flight to the LDS ring
    // B column's level-0 plane p lives in slot p mod QSL of this thread's LDS ring
    T *const qring = LQ + tid * VEC;
    auto qslot = [&](int p) __attribute__((always_inline)) -> T * {
        const int m = p % C::QSL;
        return qring + (m < 0 ? m + C::QSL : m) * (C::NBV * VEC);
    };
    T wa[Q][VEC];                   // level 1 at planes z-2R .. z (A column)
    T xyp[R + 1][VEC];              // x/y part of level 2 at planes z-R .. z (A column)
    T cring[R + 1][VEC];            // c at planes z-R .. z (A column)
    T pa[2][VEC], ca[2][VEC], pb[2][VEC], cb[2][VEC], ho[2][VEC];

    // level-0 plane pz (grid plane index) for the queues: zero outside [-R, nz + R)
    auto load_q = [&](T(&qa_)[VEC], T(&qb_)[VEC], int pz) __attribute__((always_inline)) {
        if (pz >= -R && pz < s.nz + R) {
            vld(qa_, plane_at(cur, pxy, pz + R, oba));
            if (hasb)
                vld(qb_, plane_at(cur, pxy, pz + R, obb));
            else
                vzero(qb_);
        } else {
            vzero(qa_);
            vzero(qb_);
        }
    };
    // plane z in [z0 - R, z1 + R): always a stored plane; st_ is the register set (a
    // compile-time index, so the arrays stay in registers)
    auto load_streams = [&](auto st_, int z) __attribute__((always_inline)) {
        constexpr int st = decltype(st_)::value;
        vld_nt(pa[st], plane_at(prev, pxy, z + R, oba));
        vld_nt(ca[st], plane_at(cc, pxy, z + R, oba));
        if (hasb) {
            vld_nt(pb[st], plane_at(prev, pxy, z + R, obb));
            vld_nt(cb[st], plane_at(cc, pxy, z + R, obb));
        } else {
            vzero(pb[st]);
            vzero(cb[st]);
        }
        if (oload)
            vld(ho[st], plane_at(cur, pxy, z + R, obo));
        else
            vzero(ho[st]);
    };

    const int zs = z0 - R;  // first level-1 plane
    const int ze = z1 + R;  // one past the last level-1 plane
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        load_q(qa[k], qbt[0], zs - R + k);
        if (hasb) vst(qslot(zs - R + k), qbt[0]);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) vzero(wa[k]);
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        vzero(xyp[k]);
        vzero(cring[k]);
    }
    load_streams(std::integral_constant<int, 0>{}, zs);

    const bool events = s.ev_ptr != nullptr;
    int nev_a1 = events ? vec_next_event<C>(s, agx, agy, ain, max(zs, 0)) : 0x7fffffff;
    int nev_b1 = events ? vec_next_event<C>(s, bgx, bgy, bin, max(zs, 0)) : 0x7fffffff;
    int nev_a2 = events ? vec_next_event<C>(s, agx, agy, ain, z0) : 0x7fffffff;

    const int la0 = (ay + 2 * R) * C::W0 + ax + 2 * R;   // A in the level-0 region
    const int lb0 = (bey + R) * C::W0 + bex + R;         // B in the level-0 region
    const int lo0 = oey * C::W0 + oex;                   // O in the level-0 region
    const int la1 = (ay + R) * C::EW + ax + R;           // A in E
    const int lb1 = bey * C::EW + bex;                   // B in E

    for (int zb = zs; zb < ze; zb += 2) {
        static_for<2>([&](auto st_) __attribute__((always_inline)) {
            constexpr int cs = decltype(st_)::value, ns = cs ^ 1;
            constexpr int tail = 2 * R + 1;
            const int z = zb + cs;
            if (z >= ze) return;
            // the B plane z+R loaded one iteration ago enters the ring (in the prologue
            // for the first iteration)
            if (hasb && z > zs) vst(qslot(z + R), qbt[cs]);
            if (z + 1 < ze) {
                load_q(qa[tail], qbt[ns], z + 1 + R);
                load_streams(std::integral_constant<int, ns>{}, z + 1);
            }

            // level 0 of plane z into LDS
            vst(L0 + la0, qa[R]);
            if (hasb) {
                T t[VEC];
                vld(t, qslot(z));
                vst(L0 + lb0, t);
            }
            if (haso) vst(L0 + lo0, ho[cs]);
            __syncthreads();

            // level 1 of plane z on the A and B columns (zero outside the grid)
            const bool zin = z >= 0 && z < s.nz;
            T w1a[VEC], w1b[VEC];
            {
                T acc[VEC];
                xy_pairs<C, C::W0>(L0, ay + 2 * R, ax + 2 * R, qa[R], acc);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T u0 = qa[R][v];
#pragma unroll
                    for (int l = 1; l <= R; ++l)
                        acc[v] = fma_t(T(Wt.w[l]), (qa[R + l][v] - u0) + (qa[R - l][v] - u0), acc[v]);
                    w1a[v] = fma_t(ca[cs][v], acc[v], T(2) * u0 - pa[cs][v]);
                }
            }
            if (hasb) {
                T acc[VEC], u0[VEC];
                vld(u0, qslot(z));
                xy_pairs<C, C::W0>(L0, bey + R, bex + R, u0, acc);
#pragma unroll
                for (int l = 1; l <= R; ++l) {
                    T zp[VEC], zm[VEC];
                    vld(zp, qslot(z + l));
                    vld(zm, qslot(z - l));
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        acc[v] = fma_t(T(Wt.w[l]), (zp[v] - u0[v]) + (zm[v] - u0[v]), acc[v]);
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) w1b[v] = fma_t(cb[cs][v], acc[v], T(2) * u0[v] - pb[cs][v]);
            } else {
                vzero(w1b);
            }
            if (zin) {
                if (z == nev_a1)  // sources of step n; receivers only on the owned planes
                    nev_a1 = vec_events<C>(s, agx, agy, ain, z, n, (z >= z0 && z < z1) ? n - s.rec_base : -1, w1a);
                if (z == nev_b1) nev_b1 = vec_events<C>(s, bgx, bgy, bin, z, n, -1, w1b);
            }
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                if (!zin || !amask[v]) w1a[v] = T(0);
                if (!zin || !bmask[v]) w1b[v] = T(0);
            }
            if (ain && z >= z0 && z < z1) {
                T *p1 = plane_at(out1, pxy, z + R, oba);
                if (agx + VEC <= s.nx) {
                    vst_nt(p1, w1a);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        if (agx + v < s.nx) p1[v] = w1a[v];
                }
            }

            // level 1 of plane z into LDS; its x/y part of the level-2 sum
            vst(L1 + la1, w1a);
            if (hasb) vst(L1 + lb1, w1b);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < Q - 1; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) wa[k][v] = wa[k + 1][v];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                wa[Q - 1][v] = w1a[v];
                cring[R][v] = ca[cs][v];
            }
            xy_pairs<C, C::EW>(L1, ay + R, ax + R, w1a, xyp[R]);

            // level 2 of plane z - R on the A column
            const int zz = z - R;
            if (zz >= z0) {
                T u2[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T u1 = wa[R][v];
                    T acc = xyp[0][v];
#pragma unroll
                    for (int l = 1; l <= R; ++l) acc = fma_t(T(Wt.w[l]), (wa[R + l][v] - u1) + (wa[R - l][v] - u1), acc);
                    u2[v] = fma_t(cring[0][v], acc, T(2) * u1 - qa[0][v]);
                }
                if (zz == nev_a2) nev_a2 = vec_events<C>(s, agx, agy, ain, zz, n + 1, n + 1 - s.rec_base, u2);
                if (ain) {
                    T *p2 = plane_at(out2, pxy, zz + R, oba);
                    if (agx + VEC <= s.nx) {
                        vst_nt(p2, u2);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v)
                            if (agx + v < s.nx) p2[v] = u2[v];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    xyp[k][v] = xyp[k + 1][v];
                    cring[k][v] = cring[k + 1][v];
                }
#pragma unroll
            for (int k = 0; k < P - 1; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) qa[k][v] = qa[k + 1][v];
        });
    }
}

template <class C>
__global__ __launch_bounds__(C::NT) void fwd2_kernel(Fwd2Args a)
{
    typedef typename C::type T;
    __shared__ __attribute__((aligned(16))) T l0[C::W0 * C::H0];
    __shared__ __attribute__((aligned(16))) T l1[C::EW * C::EH];
    __shared__ __attribute__((aligned(16))) T lq[C::QSL * C::NBV * C::VEC];
    int wg = blockIdx.x;
    if (a.xcd_remap) wg = xcd_remap(wg, (int)gridDim.x);
    const ShotDesc &s = *a.shot;
    const int tx = wg % a.tiles_x;
    const int t2 = wg / a.tiles_x;
    const int ty = t2 % a.tiles_y;
    const int cz = t2 / a.tiles_y;
    if (cz >= a.chunks_z) return;
    fwd2_tile<C>(s, a, tx, ty, cz, l0, l1, lq);
}

struct Fwd2Entry {
    const char *name;
    int r, bx, by, nt;
    void (*launch)(const Fwd2Args &, int nwg, hipStream_t);
    const void *kernel;
};

template <class C>
void launch_fwd2(const Fwd2Args &a, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(fwd2_kernel<C>, dim3(nwg), dim3(C::NT), 0, st, a);
}

template <class C>
Fwd2Entry fwd2_entry(const char *name)
{
    return Fwd2Entry{name, C::R, C::BX, C::BY, C::NT, &launch_fwd2<C>, reinterpret_cast<const void *>(&fwd2_kernel<C>)};
}

// Implemented in fd_fwd2_f32.hip: the two-step kernels for FP32 (radius r, 3-D).
const Fwd2Entry *fwd2_configs_f32(int r, int *count);

}  // namespace fdw
