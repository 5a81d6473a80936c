// fd_vti.h -- gfx950 kernel for the two-field VTI propagator.
//
// One launch performs one step of the centred time scheme of Sec. 1 of Medina,
// St-Cyr and Warburton applied to the pseudo-acoustic VTI equations (p) and (q):
//     p^{n+1} = 2 p^n - p^{n-1} + ax * Sxy + az * Sz + sources
//     q^{n+1} = 2 q^n - q^{n-1} + an * Sxy + az * Sz + sources
// with ax, an, az = dt^2 (nu_x^2, nu_n^2, nu_z^2) / h^2 and
//     Sxy = 2 w_0 p + sum_{l=1..RXY} w_l (p_{x+l} + p_{x-l} + p_{y+l} + p_{y-l})
//           (the symmetric xy stencil of Sec. 1, acting on p only),
//     Sz  = sum_{l=-RZ..RZ} Wz[z][l] q_{z+l}
//           (the per-plane z stencil of Sec. 1 with 2 RZ + 1 weights per plane,
//            variable spacing absorbed in the weights, acting on q only).
// Both sums are evaluated in the centre-weight form of the paper (two operations
// per neighbour pair): with RXY = 12 the difference form would double the vector
// work of the xy part, and this kernel is meant to stay memory-bound.
//
// Design (no MFMA: a star stencil is not a dense contraction):
//  - A workgroup owns a BX x BY tile of the xy plane and marches a chunk of z
//    planes.  Each thread owns one 16-byte vector of x points in one row.
//  - p is needed with its xy neighbours only, q with its z neighbours only.  So the
//    plane z of p^n, with its RXY-wide x/y halo, is staged in LDS (two buffers, one
//    barrier per plane), and q^n of the thread's column is kept for planes
//    z-RZ .. z+RZ in a register queue that shifts by one plane per step.
//  - Global traffic is x-contiguous 16-byte vectors: p^n and q^n once per point
//    (plus the p halo and the q chunk prologue), p^{n-1}, q^{n-1} and the three
//    coefficient fields streamed with nontemporal loads, p^{n+1} and q^{n+1}
//    written with nontemporal stores over p^{n-1} and q^{n-1}.  Every load of the
//    next plane is issued one plane ahead of its use.
//  - The z weights of plane z are uniform across the workgroup (scalar loads).
//  - Sources and receivers use the column-sorted event list of the acoustic kernel.
#pragma once

#include "fd_stencil.h"

namespace fdw {

template <typename T, int RXY_, int RZ_, int TXN_, int TYN_>
struct VtiCfg {
    typedef T type;
    static constexpr int RXY = RXY_;
    static constexpr int RZ = RZ_;
    static constexpr int TXN = TXN_;                          // threads along x
    static constexpr int TYN = TYN_;                          // threads (= rows) along y
    static constexpr int VEC = V16<T>::N;
    static constexpr int NT = TXN * TYN;
    static constexpr int BX = TXN * VEC;
    static constexpr int BY = TYN;
    static constexpr int LPAD = (RXY + VEC - 1) / VEC * VEC;  // x halo rounded to vectors
    static constexpr int LW = BX + 2 * LPAD;
    static constexpr int LH = BY + 2 * RXY;
    static constexpr int LDS = LW * LH;                       // elements per LDS plane
    static constexpr int NXV = 2 * LPAD / VEC + 1;            // vectors per row for x neighbours
    static constexpr int NHY = 2 * RXY * TXN;                 // y-halo vectors per plane
    static constexpr int NHS = LPAD / VEC;                    // x-halo vectors per side per row
    static constexpr int NHX = 2 * BY * NHS;
    static constexpr int NH = NHY + NHX;
    static constexpr int HPT = (NH + NT - 1) / NT;            // halo vectors per thread
    static constexpr int NWZ = 2 * RZ + 1;
    static_assert(256 % BX == 0 && 64 % BY == 0, "tile must divide the layout alignment");
};

template <class C>
__device__ __forceinline__ void vti_tile(const VtiDesc &s, int64_t step, int tx, int ty, int cz,
                                         typename C::type *lds)
{
    typedef typename C::type T;
    constexpr int RXY = C::RXY, RZ = C::RZ, VEC = C::VEC, HPT = C::HPT, NWZ = C::NWZ;
    constexpr int P = 2 * RZ + 2;  // q planes z-RZ .. z+RZ and the slot receiving z+RZ+1
    constexpr StencilWeights<RXY> W{};
    const int cb = (int)(step & 1), nb = cb ^ 1;
    const T *__restrict__ pcur = static_cast<const T *>(s.pbuf[cb]);
    const T *__restrict__ qcur = static_cast<const T *>(s.qbuf[cb]);
    const T *pprev = static_cast<const T *>(s.pbuf[nb]);  // read point-wise, then overwritten
    const T *qprev = static_cast<const T *>(s.qbuf[nb]);
    T *pout = static_cast<T *>(s.pbuf[nb]);
    T *qout = static_cast<T *>(s.qbuf[nb]);
    const T *__restrict__ fax = static_cast<const T *>(s.ax);
    const T *__restrict__ fan = static_cast<const T *>(s.an);
    const T *__restrict__ faz = static_cast<const T *>(s.az);
    const T *__restrict__ wz = static_cast<const T *>(s.wz);
    const int64_t pxy = s.pxy;

    const int tid = threadIdx.x;
    const int lx = (tid % C::TXN) * VEC, ly = tid / C::TXN;
    const int x0 = tx * C::BX, y0 = ty * C::BY;
    const int gx = x0 + lx, gy = y0 + ly;
    const int z0 = cz * s.zch;
    const int z1 = min(z0 + s.zch, s.nz);
    if (z0 >= z1) return;  // uniform over the workgroup
    const bool rin = gx < s.nx && gy < s.ny;

    // byte offsets inside a plane; the plane index zp = z + RZ counts the ghost planes.
    // Every tile point lies inside the aligned row/plane extents, whose padding is zero,
    // so the loads of the thread's own column need no mask.
    const int64_t colp = s.off0 + (int64_t)gy * s.px + gx - (int64_t)RZ * pxy;
    const uint32_t ob = (uint32_t)(colp * (int64_t)sizeof(T));
    uint32_t hob[HPT];
    int hl[HPT];
    bool hval[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int hv = tid + k * C::NT;
        hval[k] = hv < C::NH;
        int ry = 0, cx = 0;
        if (hv < C::NHY) {
            const int ri = hv / C::TXN;
            cx = (hv % C::TXN) * VEC;
            ry = (ri < RXY) ? ri - RXY : C::BY + (ri - RXY);
        } else if (hv < C::NH) {
            const int hx = hv - C::NHY;
            ry = hx / (2 * C::NHS);
            const int si = hx % (2 * C::NHS);
            cx = (si < C::NHS) ? -C::LPAD + si * VEC : C::BX + (si - C::NHS) * VEC;
        }
        const int64_t ho = s.off0 + (int64_t)(y0 + ry) * s.px + (x0 + cx) - (int64_t)RZ * pxy;
        hob[k] = (uint32_t)(ho * (int64_t)sizeof(T));
        hl[k] = (ry + RXY) * C::LW + (cx + C::LPAD);
    }

    T q[P][VEC];
    T pc[2][VEC], pm[2][VEC], qm[2][VEC], a1[2][VEC], a2[2][VEC], a3[2][VEC];
    T hv[2][HPT][VEC];

    // prologue: q planes z0-RZ .. z0+RZ into slots 0 .. 2RZ; everything of plane z0 into set 0
#pragma unroll
    for (int k = 0; k <= 2 * RZ; ++k) vld(q[k], plane_at(qcur, pxy, z0 + k, ob));
    vld(pc[0], plane_at(pcur, pxy, z0 + RZ, ob));
    vld_nt(pm[0], plane_at(pprev, pxy, z0 + RZ, ob));
    vld_nt(qm[0], plane_at(qprev, pxy, z0 + RZ, ob));
    vld_nt(a1[0], plane_at(fax, pxy, z0 + RZ, ob));
    vld_nt(a2[0], plane_at(fan, pxy, z0 + RZ, ob));
    vld_nt(a3[0], plane_at(faz, pxy, z0 + RZ, ob));
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        if (hval[k])
            vld(hv[0][k], plane_at(pcur, pxy, z0 + RZ, hob[k]));
        else
            vzero(hv[0][k]);
    }

    // next plane >= z with an event in this thread's column (INT_MAX if none)
    auto next_ev = [&](int z) {
        int nxt = 0x7fffffff;
        if (!s.ev_ptr || !rin) return nxt;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
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
    };
    int nev = next_ev(z0);

    for (int zb = z0; zb < z1; zb += 2) {
        static_for<2>([&](auto st_) __attribute__((always_inline)) {
            constexpr int cs = decltype(st_)::value, ns = cs ^ 1;
            constexpr int tail = 2 * RZ + 1;
            const int z = zb + cs;
            if (z >= z1) return;
            if (z + 1 < z1) {
                const int zn = z + 1 + RZ;
                vld(q[tail], plane_at(qcur, pxy, zn + RZ, ob));
                vld(pc[ns], plane_at(pcur, pxy, zn, ob));
                vld_nt(pm[ns], plane_at(pprev, pxy, zn, ob));
                vld_nt(qm[ns], plane_at(qprev, pxy, zn, ob));
                vld_nt(a1[ns], plane_at(fax, pxy, zn, ob));
                vld_nt(a2[ns], plane_at(fan, pxy, zn, ob));
                vld_nt(a3[ns], plane_at(faz, pxy, zn, ob));
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    if (hval[k]) vld(hv[ns][k], plane_at(pcur, pxy, zn, hob[k]));
            }

            // stage plane z of p^n (interior from registers, halo) in LDS buffer cs;
            // buffer cs was last read two planes ago, before the previous barrier
            T *L = lds + cs * C::LDS;
            vst(L + (ly + RXY) * C::LW + C::LPAD + lx, pc[cs]);
#pragma unroll
            for (int k = 0; k < HPT; ++k)
                if (hval[k]) vst(L + hl[k], hv[cs][k]);
            __syncthreads();

            // Sxy from LDS
            T sxy[VEC];
            {
                T xs[C::NXV * VEC];
#pragma unroll
                for (int j = 0; j < C::NXV; ++j) {
                    T tmp[VEC];
                    vld(tmp, L + (ly + RXY) * C::LW + lx + j * VEC);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) xs[j * VEC + v] = tmp[v];
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T acc = T(2.0 * W.w[0]) * pc[cs][v];
#pragma unroll
                    for (int l = 1; l <= RXY; ++l)
                        acc = fma_t(T(W.w[l]), xs[C::LPAD + v + l] + xs[C::LPAD + v - l], acc);
                    sxy[v] = acc;
                }
#pragma unroll
                for (int l = 1; l <= RXY; ++l) {
                    T up[VEC], dn[VEC];
                    vld(up, L + (ly + RXY - l) * C::LW + C::LPAD + lx);
                    vld(dn, L + (ly + RXY + l) * C::LW + C::LPAD + lx);
#pragma unroll
                    for (int v = 0; v < VEC; ++v) sxy[v] = fma_t(T(W.w[l]), up[v] + dn[v], sxy[v]);
                }
            }

            // Sz from the queue with this plane's weights (uniform: scalar loads)
            T sz[VEC];
            {
                const T *__restrict__ wrow = wz + (int64_t)z * NWZ;
                T wk[NWZ];
#pragma unroll
                for (int j = 0; j < NWZ; ++j) wk[j] = wrow[j];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    T acc = wk[0] * q[0][v];
#pragma unroll
                    for (int j = 1; j < NWZ; ++j) acc = fma_t(wk[j], q[j][v], acc);
                    sz[v] = acc;
                }
            }

            T pn[VEC], qn[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const T p0 = pc[cs][v], q0 = q[RZ][v];
                const T zt = a3[cs][v] * sz[v];
                pn[v] = fma_t(a1[cs][v], sxy[v], (T(2) * p0 - pm[cs][v]) + zt);
                qn[v] = fma_t(a2[cs][v], sxy[v], (T(2) * q0 - qm[cs][v]) + zt);
            }

            // fused sources (before the store) and receivers (after them)
            if (z == nev) {
                int nxt = 0x7fffffff;
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    if (rin && gx + v < s.nx) {
                        const int cidx = gy * s.nx + gx + v;
                        const int lo = s.ev_ptr[cidx], hi = s.ev_ptr[cidx + 1];
                        if (lo < hi) {
                            int p = lower_bound_z(s.ev, lo, hi, z);
                            for (; p < hi && s.ev[p].z == z; ++p) {
                                const int code = s.ev[p].code;
                                if (code < 0) {
                                    const VtiSource si = s.src[~code];
                                    if (step < si.nsamp) {
                                        const T sv = static_cast<const T *>(si.wav)[step];
                                        pn[v] += T(si.scale_p) * sv;
                                        qn[v] += T(si.scale_q) * sv;
                                    }
                                } else {
                                    const int64_t row = step - s.rec_base;
                                    if (row >= 0 && row < s.rec_cap) {
                                        if (s.traces_p) static_cast<T *>(s.traces_p)[row * s.nrec + code] = pn[v];
                                        if (s.traces_q) static_cast<T *>(s.traces_q)[row * s.nrec + code] = qn[v];
                                    }
                                }
                            }
                            if (p < hi) nxt = min(nxt, s.ev[p].z);
                        }
                    }
                }
                nev = nxt;
            }

            if (rin) {
                T *pp = plane_at(pout, pxy, z + RZ, ob);
                T *qp = plane_at(qout, pxy, z + RZ, ob);
                if (gx + VEC <= s.nx) {
                    vst_nt(pp, pn);
                    vst_nt(qp, qn);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        if (gx + v < s.nx) {
                            pp[v] = pn[v];
                            qp[v] = qn[v];
                        }
                }
            }
#pragma unroll
            for (int k = 0; k < P - 1; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) q[k][v] = q[k + 1][v];
        });
    }
}

template <class C>
__global__ __launch_bounds__(C::NT) void vti_kernel(VtiDesc s, int64_t step)
{
    typedef typename C::type T;
    __shared__ __attribute__((aligned(16))) T lds[2 * C::LDS];
    int wg = blockIdx.x;
    if (s.xcd_remap) wg = xcd_remap(wg, (int)gridDim.x);
    const int tx = wg % s.tiles_x;
    const int t2 = wg / s.tiles_x;
    const int ty = t2 % s.tiles_y;
    const int cz = t2 / s.tiles_y;
    if (cz >= s.chunks_z) return;
    vti_tile<C>(s, step, tx, ty, cz, lds);
}

struct VtiEntry {
    const char *name;
    int rxy, rz, bx, by, nt;
    void (*launch)(const VtiDesc &, int64_t step, int nwg, hipStream_t);
    const void *kernel;
};

template <class C>
void launch_vti(const VtiDesc &d, int64_t step, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(vti_kernel<C>, dim3(nwg), dim3(C::NT), 0, st, d, step);
}

template <class C>
VtiEntry vti_entry(const char *name)
{
    return VtiEntry{name, C::RXY, C::RZ, C::BX, C::BY, C::NT, &launch_vti<C>,
                    reinterpret_cast<const void *>(&vti_kernel<C>)};
}

// Implemented in the per-dtype translation units.
const VtiEntry *vti_configs_f32(int rxy, int rz, int *count);
const VtiEntry *vti_configs_f64(int rxy, int rz, int *count);

}  // namespace fdw
