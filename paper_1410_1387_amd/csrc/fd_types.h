// fd_types.h -- data structures shared by the host side of the library and its
// device kernels: the padded field geometry, the per-shot descriptor that the
// stencil kernels read from device memory, and the per-launch arguments.
#pragma once

#include <stdint.h>

namespace fdw {

// Event of the fused source/receiver list, sorted by (column, z, kind).
// A "column" is one (x, y) position of the kernel's xy plane (3-D) or one x (2-D).
struct Event {
    int32_t z;     // kernel z index (grid z in 3-D, grid y in 2-D)
    int32_t code;  // >= 0: receiver column in the trace; < 0: source ~code
};

// One registered point source: sample n of `wav` (dtype of the shot) times `scale`
// = amp * dt^2 / h^ndim is added to u^{n+1} at the source point.
struct SourceInfo {
    const void *wav;
    int64_t nsamp;
    double scale;
};

// Everything a stencil launch needs to know about one shot.  Lives in device memory
// (inside the context workspace); `ctr` is written by the kernels.
struct ShotDesc {
    void *buf[2];          // padded wavefields; u^n is buf[n & 1], u^{n+1} overwrites buf[(n+1) & 1]
    const void *c;         // padded coefficient field c = (v dt / h)^2
    int32_t nx, ny, nz;    // interior extent along the kernel's x, y, z (2-D: ny = 1, nz = grid ny)
    int32_t tiles_x, tiles_y, chunks_z, zch, pad0;
    int64_t px, pxy, off0; // row pitch, plane pitch, element offset of interior (0, 0, 0)
    int64_t ctr[2];        // step counter slots (graph / batched mode)
    int64_t target;        // batched mode: stop at this step
    const int32_t *ev_ptr; // CSR over columns: events of column col are ev[ev_ptr[col] .. ev_ptr[col+1])
    const Event *ev;
    const SourceInfo *src;
    void *traces;          // [cap][nrec] of dtype
    int64_t nrec, rec_base, rec_cap;
    const void *damp;      // absorbing sponge: per-axis factors [nx | ny | nz] of dtype, or null
};

// Per-launch arguments (passed by value).
struct LaunchArgs {
    ShotDesc *shots;           // device array of shot descriptors
    const int32_t *wg_prefix;  // device, nshots + 1 workgroup offsets (NULL when nshots == 1)
    int32_t nshots;
    int32_t slot;              // counter mode: this launch reads ctr[slot], writes ctr[slot ^ 1]
    int64_t step;              // >= 0: step index for the single shot; < 0: counter mode
    const void *cur;           // explicit-pointer mode (single shot): u^n, u^{n-1}, u^{n+1}
    const void *prev;
    void *out;
    int32_t record;            // write receiver traces
    int32_t xcd_remap;         // map consecutive tiles onto one XCD
};

// Adjoint launch arguments (single shot, explicit pointers).
struct AdjArgs {
    const ShotDesc *shot;
    const void *mu_cur;    // mu^{k+1}
    void *mu_out;          // in: mu^{k+2}, out: mu^k
    const void *u_km1;     // u^{k-1}
    void *grad;            // accumulator g (padded)
    void *gseg;            // segment partial sum of the imaging term (padded), or null
    int32_t gmode;         // imaging accumulation, see adj_tile
    int32_t pad1;
    const void *resid;     // [T][nrec]
    int64_t k;             // adjoint step index (residual row k - 1)
    double resid_amp;
    int32_t xcd_remap;
    int32_t zch;           // the adjoint kernel's own tiling (its tile differs from the forward one)
    int32_t tiles_x, tiles_y, chunks_z, pad0;
};

// ------------------------------------------------------------------ VTI propagator

// One point source of the two-field VTI propagator: sample n of `wav` times scale_p
// (scale_q) = amp_p (amp_q) * dt^2 / (h^2 dz_k) is added to p^{n+1} (q^{n+1}).
struct VtiSource {
    const void *wav;
    int64_t nsamp;
    double scale_p, scale_q;
};

// Everything one VTI launch reads (passed by value as the kernel argument).
struct VtiDesc {
    void *pbuf[2];         // padded p fields: p^n is pbuf[n & 1], p^{n+1} overwrites pbuf[(n+1) & 1]
    void *qbuf[2];         // the same for q
    const void *ax;        // dt^2 nu_x^2 / h^2   (padded)
    const void *an;        // dt^2 nu_n^2 / h^2
    const void *az;        // dt^2 nu_z^2 / h^2
    const void *wz;        // [nz][2 RZ + 1] z weights times h^2
    int32_t nx, ny, nz;
    int32_t tiles_x, tiles_y, chunks_z, zch, xcd_remap;
    int64_t px, pxy, off0;
    const int32_t *ev_ptr; // CSR over (x, y) columns, as for the acoustic kernel
    const Event *ev;
    const VtiSource *src;
    void *traces_p;        // [cap][nrec] or null
    void *traces_q;
    int64_t nrec, rec_base, rec_cap;
};

}  // namespace fdw
