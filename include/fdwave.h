/*
 * fdwave.h -- C ABI of the MI355X (gfx950) library for explicit leapfrog time
 * stepping of the acoustic wave equation
 *
 *     u_tt = v(x)^2 lap(u) + sum_s s_s(t) delta(x - x_s)
 *
 * on a regular 2-D or 3-D grid of spacing h, with a radius-r (order 2r)
 * central-difference star stencil and the centred second-order time scheme
 *
 *     u^{n+1} = 2 u^n - u^{n-1} + dt^2 v^2 L u^n + (dt^2 / h^ndim) sum_s s_s[n] e_{x_s}.
 *
 * The problem statement follows Medina, St-Cyr and Warburton, "High-Order
 * Finite-differences on multi-threaded architectures using OCCA", Sec. 1: the
 * time scheme, the symmetric stencil form, the zero solution for r points
 * outside the domain, the point source s(t) delta(x - x_i) that is not scaled
 * by the velocity, and the Ricker forcing; its isotropic reduction (end of
 * Sec. 1) gives the single-field equation above.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every function returns an fd_status (0 on success, < 0 on failure) unless
 *    stated otherwise.  No C++ exception crosses the ABI.  fd_last_error()
 *    returns a thread-local message for the last failure on the calling thread.
 *  - Grids: n[0] = nx (fastest, contiguous), n[1] = ny, n[2] = nz.  A 2-D grid
 *    has ndim = 2 and n[2] = 1.  Dense arrays are row-major [nz][ny][nx]
 *    (3-D) or [ny][nx] (2-D).  Positions are (x, y, z) index triples.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory read during the call only.
 *  - The library never allocates device memory.  All device memory a context
 *    uses is one caller-owned workspace (fd_workspace_bytes) plus the buffers
 *    passed to the calls below.
 *  - A context is bound to one HIP stream (hipStream_t passed as void*; NULL is
 *    the null stream).  Every device operation is enqueued on it
 *    asynchronously.  A context is not thread-safe; different contexts are
 *    independent.  Argument errors are detected before anything is enqueued.
 *  - Asynchronous device faults are reported as FD_E_DEVICE by fd_sync (or the
 *    next call that synchronises); the context is then poisoned and only
 *    fd_destroy remains valid on it.
 *  - dtype FD_F32 stores and computes the wavefield in float; FD_F64 in double.
 */
#ifndef FDWAVE_H
#define FDWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fd_ctx fd_ctx;
typedef struct fd_batch fd_batch;

typedef enum {
    FD_OK = 0,
    FD_E_INVAL = -1,    /* bad argument (ndim, r, h, dt, sizes, null pointer) */
    FD_E_RANGE = -2,    /* position outside the grid, capacity or maximum exceeded */
    FD_E_UNSTABLE = -3, /* dt above the stability limit fd_dt_max for max(v) */
    FD_E_STATE = -4,    /* call not valid in the context's current state */
    FD_E_DEVICE = -5,   /* HIP runtime or kernel error; context poisoned */
    FD_E_NOMEM = -6     /* workspace smaller than fd_workspace_bytes */
} fd_status;

typedef enum { FD_F32 = 0, FD_F64 = 1 } fd_dtype;

/* FD_BC_ZERO: the solution is zero on r ghost cells outside every face (Sec. 1,
 * last paragraph).  FD_BC_PERIODIC: the grid wraps around (used to test the
 * scheme against closed-form standing waves; not supported by fd_batch). */
typedef enum { FD_BC_ZERO = 0, FD_BC_PERIODIC = 1 } fd_bc;

/* layout flag for state copies */
typedef enum { FD_DENSE = 0, FD_PADDED = 1 } fd_layout;

typedef struct {
    int32_t ndim;  /* 2 or 3 */
    int64_t n[3];  /* nx, ny, nz (nz = 1 when ndim = 2); each >= 1 */
} fd_grid;

/* ----------------------------------------------------------------- stencil and limits */

/* Exact central weights of the radius-r second-derivative stencil on a unit grid,
 * h^2 u'' ~ w[0] u_i + sum_{l=1..r} w[l] (u_{i+l} + u_{i-l})  (Sec. 1, stencil form;
 * the weights are those exact for polynomials of degree <= 2r+1).
 * w: host, r+1 doubles, written.  1 <= r <= 12 (the acoustic kernels take r <= 8,
 * the VTI xy stencil r <= 12).  Each weight is the correctly rounded double. */
int fd_weights(int r, double *w);

/* Von Neumann limit of the leapfrog scheme for this stencil:
 * dt_max = 2 h / (vmax sqrt(ndim S_r)), S_r = -w0 + 2 sum |w_l| the largest value of
 * the 1-D symbol.  Returns a negative value for invalid arguments. */
double fd_dt_max(int ndim, int r, double h, double vmax);

/* ----------------------------------------------------------------- memory planning */

/* Device bytes of one padded wavefield of this grid (the unit of checkpoints and of the
 * recompute ring used by the adjoint).  Layout: x-fastest rows with a 128-byte aligned
 * interior, r zero ghost planes/rows on every face plus alignment padding; the padding
 * must stay zero.  *bytes written. */
int fd_field_bytes(const fd_grid *g, int r, fd_dtype dtype, size_t *bytes);

/* Device bytes of the workspace a context needs: two padded wavefields, the padded
 * coefficient field c = (v dt / h)^2, and the source/receiver tables for at most
 * max_sources sources and max_receivers receivers.  *bytes written. */
int fd_workspace_bytes(const fd_grid *g, int r, fd_dtype dtype, int64_t max_sources,
                       int64_t max_receivers, size_t *bytes);

/* ----------------------------------------------------------------- lifecycle */

/* Create a context (Sec. 1 problem statement: grid, stencil radius, spacing, time step
 * and velocity).
 *   velocity   device, dense, dtype, >0 m/s; read during the call only (converted to
 *              c = (v dt / h)^2 in the workspace by a device kernel)
 *   workspace  device, >= fd_workspace_bytes(...) bytes, 256-byte aligned; borrowed
 *              until fd_destroy; zeroed here (both wavefields start at zero, step 0)
 *   stream     hipStream_t the context enqueues on
 * Errors: FD_E_INVAL (ndim not 2/3, r not in [1, 8], h or dt <= 0, null pointers,
 * non-positive velocity), FD_E_NOMEM (workspace too small), FD_E_UNSTABLE
 * (dt > fd_dt_max(ndim, r, h, max v)), FD_E_DEVICE.  Synchronises the stream once
 * (to read max/min of v). */
int fd_create(fd_ctx **out, const fd_grid *g, int r, double h, double dt, const void *velocity,
              fd_dtype dtype, fd_bc bc, void *workspace, size_t ws_bytes, int64_t max_sources,
              int64_t max_receivers, void *stream);

int fd_destroy(fd_ctx *ctx);

/* Rebind the context to another stream (e.g. after a caller switches streams). */
int fd_set_stream(fd_ctx *ctx, void *stream);

/* ----------------------------------------------------------------- source and receivers */

/* Add a point source (Sec. 1, eq. (p): s(t) delta(x - x_i)).
 *   wavelet  device, nsamp samples of dtype; borrowed until fd_clear_sources/fd_destroy.
 *            Sample n enters the step that produces u^{n+1} (n counted from step 0),
 *            scaled by amp * dt^2 / h^ndim; samples beyond nsamp are zero.
 *   pos      host, (x, y, z) (z ignored in 2-D)
 *   amp      multiplies the physical scaling; 1.0 is the paper's source.  Powers of two
 *            keep FP32 values away from underflow and are exact.
 * Fused into the stencil kernel.  Errors: FD_E_RANGE (position outside the grid or
 * more than max_sources), FD_E_INVAL. */
int fd_inject(fd_ctx *ctx, const void *wavelet, int64_t nsamp, const int64_t pos[3], double amp);
int fd_clear_sources(fd_ctx *ctx);

/* Absorbing sponge (Sec. 1: the domain is embedded in a damping region, after Cerjan et
 * al.; the paper gives neither profile nor constants).  In a strip of `width` points at
 * each face selected by `faces` (bit 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+ of the grid's
 * axes; a 2-D grid uses bits 0-3), the point at distance i from the face (i = 0 outermost)
 * has the factor exp(-(alpha (width - i))^2); factors of overlapping strips multiply and
 * G = 1 elsewhere.  Every step then computes u^{n+1} = G (2u^n - G u^{n-1} + c Lh u^n)
 * (both time levels damped) before adding sources.  Cerjan's constants are width = 20,
 * alpha = 0.015.  width = 0 or faces = 0 switches the sponge off (the update is then
 * bitwise the undamped one).  Zero boundary only (FD_E_STATE otherwise); a damped context
 * has no adjoint (fd_adjoint_segment returns FD_E_STATE). */
int fd_set_damping(fd_ctx *ctx, int width, double alpha, int faces);

/* Record u^{n+1} at receiver positions after every step (fused into the stencil kernel).
 *   pos     host, int32 [nrec][3] (x, y, z); z ignored in 2-D
 *   traces  device, dtype, time-major [cap][nrec]; row i holds the step that starts
 *           from step (k0 + i) where k0 is the context's step at this call; borrowed
 *   nrec = 0 disables recording.  Replaces any previous receiver set.
 * Errors: FD_E_RANGE (position outside, nrec > max_receivers), FD_E_INVAL. */
int fd_record(fd_ctx *ctx, const int32_t *pos, int64_t nrec, void *traces, int64_t cap);

/* Source samples of the Ricker wavelet s = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2),
 * tau = n dt - t0 (Sec. 1 forcing), computed on the device.
 *   out  device, nsamp values of dtype.  Enqueued on stream. */
int fd_ricker(void *out, int64_t nsamp, double dt, double f0, double t0, fd_dtype dtype,
              void *stream);

/* ----------------------------------------------------------------- time stepping */

/* Advance nsteps leapfrog steps (Sec. 1 time scheme), one stencil launch per step, with
 * the sources added and the receivers recorded inside the launch.  nsteps = 0 is a no-op.
 * Errors: FD_E_RANGE if recording is on and the trace capacity would be exceeded (checked
 * before anything is enqueued), FD_E_STATE if poisoned. */
int fd_step(fd_ctx *ctx, int64_t nsteps);

/* Two steps per launch (temporal blocking) for fd_step: each launch takes (u^n, u^{n-1})
 * to (u^{n+1}, u^{n+2}) of the same scheme (Sec. 1 time scheme), reading u^n, u^{n-1} and c
 * once and writing both new levels (20 B per point per two steps instead of 32).  The
 * result is bitwise that of single steps.  aux: device, caller-owned, 256-byte aligned,
 * >= 2 * fd_field_bytes bytes, borrowed until disabled or the context is destroyed; it
 * is zeroed here (on the context stream).  fd_step then runs groups of four steps as two
 * two-step launches (through aux and back, so the context's fields keep their roles) and
 * any remainder as single steps.  Periodic or damped contexts keep single steps.
 * config: index of the tile shape (0 = default).  aux = NULL disables.  On MI355X this
 * path moves 20 instead of 32 bytes per point and two steps but is slower than single
 * steps (228 against 352 Gpts/s at 512^3): level 1 on the widened tile costs 80 instead
 * of 59 vector instructions per point update, and the launch is latency-bound (one
 * workgroup per compute unit, two barriers per plane).  It is off unless enabled and no
 * benchmark figure uses it.  Errors:
 * FD_E_INVAL (no two-step kernel: 3-D FP32 with r = 4 only; misaligned aux), FD_E_RANGE
 * (config), FD_E_NOMEM (aux too small). */
int fd_set_time_blocking(fd_ctx *ctx, void *aux, size_t aux_bytes, int config);

/* Wait for the context's stream; reports asynchronous device errors (FD_E_DEVICE). */
int fd_sync(fd_ctx *ctx);

/* Current step count (number of steps taken since step 0 or the last fd_set_state). */
int fd_get_step(const fd_ctx *ctx, int64_t *step);

/* Failure detection: *finite (host int) = 1 if every value of the current state u^n and
 * u^{n-1} is finite, 0 if a NaN or an infinity has appeared (a corrupt source wavelet or
 * state; the scheme itself stays bounded below fd_dt_max).  Reads both padded fields on
 * the context's stream and synchronises it (batched steps of the context are ordered
 * before it, see fd_batch_step).  Not part of the method: a probe to run every so many
 * steps. */
int fd_check_finite(fd_ctx *ctx, int *finite);

/* Copy the state (u^n, u^{n-1}) out of / into the context.
 *   layout FD_DENSE: device dense arrays of dtype (fd_get_state packs, fd_set_state
 *   unpacks and keeps the ghost cells zero); FD_PADDED: device buffers of
 *   fd_field_bytes each, copied as they are (checkpoints).  Either pointer may be NULL to
 *   skip that field.  fd_set_state also sets the step counter to `step`. */
int fd_get_state(fd_ctx *ctx, void *u_cur, void *u_prev, int64_t *step, fd_layout layout);
int fd_set_state(fd_ctx *ctx, const void *u_cur, const void *u_prev, int64_t step, fd_layout layout);

/* One forward step from explicit padded buffers: out = 2 cur - prev + c L cur + sources at
 * step index `step`; receivers are not recorded and the context's own state and step
 * counter are untouched.  out may equal prev but not cur.  Used to recompute a checkpoint
 * segment into a ring of padded fields for the adjoint. */
int fd_step_explicit(fd_ctx *ctx, const void *cur, const void *prev, void *out, int64_t step);

/* The same step, recording the receivers registered with fd_record: u^{step+1} at them
 * goes to row step - (the step at which fd_record was called) of the traces buffer, if
 * that row lies in [0, cap).  The forward pass of a gradient that keeps every state
 * (out = a new buffer each step) calls this; fd_adjoint_stored then needs no recompute.
 * Same arguments and errors as fd_step_explicit. */
int fd_step_record(fd_ctx *ctx, const void *cur, const void *prev, void *out, int64_t step);

/* ----------------------------------------------------------------- adjoint (gradient) */

/* Discrete adjoint of the forward scheme for J = 1/2 sum_n sum_j resid[n][j]^2 with
 * resid = traces - observed (discretise, then differentiate; the paper's statement of
 * the problem names full waveform inversion as the application, Sec. 1).  With
 * c = (v dt / h)^2, mu = c lambda and mu^{T+1} = mu^{T+2} = 0, one call does, for
 * k = k_hi .. k_lo+1 (descending):
 *     mu^k = 2 mu^{k+1} - mu^{k+2} + c L^ mu^{k+1} + resid_amp sum_j c_j resid[k-1][j] e_j
 *     g   += mu^k * (L^ u^{k-1})
 * where L^ = h^2 L is the unscaled stencil.  dJ/dv = 2 g / v (fd_gradient_finish).
 * The imaging sum is kept in the working precision.  With grad_seg given, it is blocked
 * by segment: the segment's terms are summed into grad_seg and added to grad at the
 * segment's last step, so rounding grows with segment length + segment count rather
 * than with the step count.
 *   u_ckpt_cur, u_ckpt_prev  device padded u^{k_lo}, u^{k_lo - 1} (a forward checkpoint)
 *   ring      device, (k_hi - k_lo - 1) padded fields; filled with u^{k_lo+1} ..
 *             u^{k_hi-1} by recomputation from the checkpoint (may be NULL if
 *             k_hi - k_lo == 1)
 *   mu        device, 2 padded fields; mu^k lives in mu[k & 1]; both zero before the
 *             first (highest) segment
 *   resid     device [T][nrec] of dtype, rows indexed by step n (receivers as given to
 *             fd_record)
 *   grad      device padded field of dtype, accumulated (zero it before the first segment)
 *   grad_seg  device padded field of dtype used as the segment partial sum, or NULL for
 *             plain accumulation into grad (its contents need no initialisation)
 * Receivers must have been registered with fd_record (the traces buffer is not touched).
 * resid must hold at least k_hi rows. */
int fd_adjoint_segment(fd_ctx *ctx, const void *u_ckpt_cur, const void *u_ckpt_prev, int64_t k_lo,
                       int64_t k_hi, void *ring, void *mu, const void *resid, double resid_amp,
                       void *grad, void *grad_seg);

/* The adjoint steps of fd_adjoint_segment (k = k_hi .. k_lo+1, descending, the same
 * kernel and arithmetic) for a segment whose forward states the caller kept: no
 * recomputation.  With the states computed by fd_step_record / fd_step_explicit from the
 * same start the result is bitwise that of fd_adjoint_segment over the same segments.
 *   states    device, (k_hi - k_lo) consecutive padded fields holding u^{k_lo} ..
 *             u^{k_hi-1} (field i at byte offset i * fd_field_bytes)
 *   mu, resid, resid_amp, grad, grad_seg  as for fd_adjoint_segment
 * Errors: FD_E_INVAL (null states, mu or grad; k_lo < 0; k_hi <= k_lo; no residual with
 * receivers), FD_E_STATE (periodic or damped context). */
int fd_adjoint_stored(fd_ctx *ctx, const void *states, int64_t k_lo, int64_t k_hi, void *mu, const void *resid,
                      double resid_amp, void *grad, void *grad_seg);

/* Zero every cell of `count` consecutive padded fields of this context's layout (field i
 * at byte offset i * fd_field_bytes) that lies outside the grid's interior: ghost planes,
 * rows and columns and the alignment padding.  Interiors are left as they are.  A padded
 * field whose interior the kernels are about to write (a state kept by fd_step_record,
 * say) needs only this instead of a full clear; a quarter or less of a large field's
 * bytes.  On the context's stream.  Errors: FD_E_INVAL (null fields, count < 0). */
int fd_clear_ghosts(fd_ctx *ctx, void *fields, int64_t count);

/* dJ/dv = scale * 2 g / v on the dense grid.
 *   grad_padded  device padded accumulator from fd_adjoint_segment
 *   velocity     device dense v (dtype);  out: device dense dJ/dv (dtype) */
int fd_gradient_finish(fd_ctx *ctx, const void *grad_padded, const void *velocity, void *out,
                       double scale);

/* ----------------------------------------------------------------- batched serving */

/* Device bytes a batch of at most max_shots shots needs (shot table, workgroup prefix). */
size_t fd_batch_workspace_bytes(int max_shots);

/* A batch advances many same-(r, dtype, ndim) zero-boundary shots of different grid sizes
 * in one stencil launch per step: each workgroup looks up its (shot, tile) from a prefix
 * table, and each shot keeps its step counter in device memory, so a captured graph of
 * an even number of steps can be replayed while shots come and go.
 *   workspace  device, fd_batch_workspace_bytes(max_shots), borrowed until destroy */
int fd_batch_create(fd_batch **out, int max_shots, void *workspace, size_t ws_bytes, void *stream);
int fd_batch_destroy(fd_batch *b);

/* Replace the member set.  Each context advances until its step reaches target[i] (host
 * array); members keep their state and step.  Members must share r, dtype and ndim
 * (FD_E_INVAL); members whose contexts chose different builds of the stencil tile are
 * stepped with the default tile (bitwise the same results).  Invalidates the captured graph.  Work still
 * queued on a member's own stream is completed before any batched launch touches it (the
 * batch stream waits for each member stream); the call also waits on the host for earlier
 * batched work, whose shot table it rewrites. */
int fd_batch_set(fd_batch *b, fd_ctx *const *ctxs, const int64_t *target, int nctx);

/* Shots a no-allocation batch can hold: the size of its fixed shot table. */
#define FD_BATCH_NOALLOC_MAX_SHOTS 256

/* For callers that cannot allocate device memory (code being captured into a HIP graph,
 * tight serving loops, harnesses that forbid allocation): a batch like fd_batch_create's
 * whose shot table (descriptors, step counters, workgroup prefix) lives in a fixed array of
 * the library instead of a caller workspace.  The array holds FD_BATCH_NOALLOC_MAX_SHOTS
 * shots (about 44 KB); each GPU the library runs on holds its own copy until the process
 * ends.  The call allocates nothing (no device or host allocation, no stream, event or
 * graph).  Use the batch with fd_batch_set, fd_batch_step and fd_batch_destroy, with these
 * differences from fd_batch_create's batch:
 *   - one per device at a time: while one is alive on the current device, another call
 *     there returns FD_E_STATE; fd_batch_destroy releases the array (the array keeps the
 *     last batch's table, which fd_batch_set rewrites whole before any step reads it);
 *   - every member context must run on the batch's stream (fd_batch_set: FD_E_INVAL);
 *   - fd_batch_step launches every step directly: it builds no graph (instantiating one
 *     allocates device memory), so nothing on this batch's path allocates device memory.
 * Results are bitwise those of fd_batch_create's batch.  Like every batch it is not
 * thread-safe: calls on it from several threads race.
 *   max_shots  1 .. FD_BATCH_NOALLOC_MAX_SHOTS (FD_E_RANGE otherwise)
 *   stream     the batch stream (hipStream_t), as for fd_batch_create */
int fd_batch_create_noalloc(fd_batch **out, int max_shots, void *stream);

/* Enqueue nsteps batched steps on the batch stream (nsteps even uses a captured graph
 * chunk of that length; odd lengths fall back to direct launches).  Members already at
 * their target do no work.  Host step mirrors advance immediately.  Each member's own
 * stream is made to wait for these steps, so later calls on a member (fd_sync,
 * fd_get_state, fd_check_finite, fd_step) are ordered after them; fd_sync on a member
 * waits for them. */
int fd_batch_step(fd_batch *b, int64_t nsteps);

/* ----------------------------------------------------------------- measurement helpers */

/* Plain device-to-device copy kernel (16-byte vectors, grid-stride) on stream: the
 * attainable-bandwidth probe and the scale reference for hardware byte counters.
 * bytes must be a multiple of 16 and both pointers 16-byte aligned. */
int fd_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* Streaming probe of the forward stencil's HBM mix without its halo or arithmetic: reads
 * a, b and c (bytes each), writes c in place, on stream; grid-stride over 16-byte vectors
 * with `blocks` workgroups of 256 threads (0 = 512).  What HBM delivers for the update's
 * three reads and one write, the reference for the stencil's bandwidth fraction.  bytes
 * must be a multiple of 16, all pointers 16-byte aligned (device memory, caller-owned);
 * c is overwritten. */
int fd_stream_probe(const void *a, const void *b, void *c, size_t bytes, int blocks, void *stream);

/* Name of the stencil kernel configuration used for (dtype, r, ndim): tile shape,
 * z-chunk and launch size. */
const char *fd_kernel_config(const fd_ctx *ctx);

/* The same for the context's adjoint kernel (fd_adjoint_segment): tile shape, z-chunk
 * and launch size.  The string is owned by the context (valid until fd_destroy); a null
 * context gives "". */
const char *fd_adjoint_config(const fd_ctx *ctx);

/* Select a stencil tile configuration by index for contexts created afterwards with this
 * (dtype, r, ndim); returns FD_E_RANGE for an unknown index.  zchunk > 0 overrides the
 * planes each workgroup marches in z.  config = -1 restores the library's own choice,
 * which is also what holds before any call: the default tile (index 0), or, for FP32 3-D
 * radii <= 4 on grids whose default z chunks would be 16 to 63 planes long (256^3 and
 * 320^3, say), the same tile built for four waves per SIMD (the last registered index).
 * Results are bitwise the same whatever the tile. */
int fd_set_tuning(fd_dtype dtype, int r, int ndim, int config, int zchunk);

/* The adjoint kernel's tile shape for contexts created afterwards with this (dtype, r,
 * ndim): config indexes the registered adjoint tiles.  config = -1 restores the library's
 * own choice, which is also what holds before any call: the default tile (index 0, 128
 * points wide for FP32 radii <= 4), or, for FP32 3-D radii <= 4 on grids whose rows that
 * tile covers badly (x = 160, 192 or 320, say, where 17-38 % of its lanes would idle), a
 * 64-point-wide tile (the last registered index).  Process-wide, thread-safe; a tuning
 * knob like fd_set_tuning; the gradient is bitwise the same whatever the tile.  Errors:
 * FD_E_INVAL (no adjoint kernel for dtype/r/ndim), FD_E_RANGE (config outside [-1, count)). */
int fd_set_adj_tuning(fd_dtype dtype, int r, int ndim, int config);

const char *fd_last_error(void);

/* ================================================================= VTI propagator
 *
 * The two-field pseudo-acoustic VTI equations of Sec. 1, eqs. (p) and (q), advanced with
 * the centred time scheme of Sec. 1 on a 3-D grid:
 *   p^{n+1} = 2p^n - p^{n-1} + dt^2 [nu_x^2 (Dxx + Dyy) p^n + nu_z^2 Dzz q^n] + dt^2 amp_p s[n] / (h^2 dz_k)
 *   q^{n+1} = 2q^n - q^{n-1} + dt^2 [nu_n^2 (Dxx + Dyy) p^n + nu_z^2 Dzz q^n] + dt^2 amp_q s[n] / (h^2 dz_k)
 * with nu_z = vz, nu_x = vz sqrt(1 + 2 eps), nu_n = vz sqrt(1 + 2 delta) (Sec. 1).
 *   - Dxx + Dyy: the symmetric radius-rxy xy stencil of Sec. 1 with spacing h, weights
 *     fd_weights(rxy) per axis (centre weight 2 w[0]).
 *   - Dzz: the per-plane z stencil of Sec. 1, 2rz+1 weights per plane (fd_vti_z_weights),
 *     which absorb a variable z spacing.
 *   - Zero values for rxy points outside the domain in x and y and rz planes in z.
 *   - dz_k = (z_{k+1} - z_{k-1}) / 2, the z extent of the cell of plane k (dz on a
 *     uniform grid).
 * Supported radius pairs (rxy, rz): rxy in {2, 4, 8, 12}, rz in {1, 2, 4, 8}, rz <= rxy.
 * Same conventions as the acoustic context: caller-owned device memory, one stream,
 * asynchronous stepping, fd_status codes. */

typedef struct fd_vti_ctx fd_vti_ctx;

/* Second-derivative weights of the z stencil of Sec. 1 for every plane: w[k*(2rz+1) + l+rz]
 * multiplies q at plane k+l (l = -rz..rz) and the row is exact for every polynomial of
 * degree <= 2rz at z_k.  Computed in FP64 with Fornberg's recursion (Math. Comp. 51, 1988).
 * zc: host, nz + 2rz strictly increasing plane coordinates (planes -rz .. nz+rz-1, in m).
 * w: host, nz * (2rz+1) doubles (1/m^2), written.  1 <= rz <= 8. */
int fd_vti_z_weights(const double *zc, int64_t nz, int rz, double *w);

/* Largest stable dt for a model bounded by vz <= vz_max, eps <= eps_max, delta <= delta_max
 * (delta <= eps point-wise): 2 / sqrt(lambda), lambda the largest eigenvalue of the 2x2
 * mode matrix [[nu_x^2 a, nu_z^2 b], [nu_n^2 a, nu_z^2 b]] at a = 2 S_xy / h^2 (Nyquist in
 * x and y) and b = the largest row sum of |Dzz| (exact for constant coefficients on a
 * uniform grid).  zc as in fd_vti_z_weights, or NULL for a uniform spacing h.
 * Returns -1 on invalid arguments. */
double fd_vti_dt_max(int rxy, int rz, double h, const double *zc, int64_t nz, double vz_max, double eps_max,
                     double delta_max);

/* Device workspace for fd_vti_create: seven padded fields (p, q at two time levels, three
 * coefficient fields), the z weight table and the source/receiver tables. */
int fd_vti_workspace_bytes(const fd_grid *g, int rxy, int rz, fd_dtype dtype, int64_t max_sources,
                           int64_t max_receivers, size_t *bytes);

/* Create a VTI context.  g: ndim 3.  zc: host, nz + 2rz plane coordinates, or NULL for a
 * uniform z spacing h.  vz, eps, delta: device, dtype, dense [nz][ny][nx], read during the
 * call only.  Errors: FD_E_INVAL (bad grid, radius pair, spacing, model: vz <= 0, 1 + 2 eps
 * <= 0, 1 + 2 delta < 0, non-finite); FD_E_UNSTABLE if delta > eps anywhere (the coupled
 * system then has a growing mode for every dt) or dt exceeds the limit of
 * fd_vti_dt_max evaluated point-wise; FD_E_NOMEM if ws_bytes is too small. */
int fd_vti_create(fd_vti_ctx **out, const fd_grid *g, int rxy, int rz, double h, const double *zc, double dt,
                  const void *vz, const void *eps, const void *delta, fd_dtype dtype, void *workspace,
                  size_t ws_bytes, int64_t max_sources, int64_t max_receivers, void *stream);
int fd_vti_destroy(fd_vti_ctx *ctx);

/* Point source: sample n of wavelet (device, dtype, nsamp samples, borrowed) enters the
 * step producing level n+1, scaled by dt^2 amp_p / (h^2 dz_k) in p and dt^2 amp_q /
 * (h^2 dz_k) in q.  Eq. (p) of Sec. 1 forces p only: amp_p = 1, amp_q = 0. */
int fd_vti_inject(fd_vti_ctx *ctx, const void *wavelet, int64_t nsamp, const int64_t pos[3], double amp_p,
                  double amp_q);

/* Receivers: pos host int32 [nrec][3]; traces_p[n][j] = p^{n+1} and traces_q[n][j] = q^{n+1}
 * at receiver j (device, dtype, time-major [cap][nrec]; either may be NULL), counted from
 * the step at which fd_vti_record is called. */
int fd_vti_record(fd_vti_ctx *ctx, const int32_t *pos, int64_t nrec, void *traces_p, void *traces_q,
                  int64_t cap);

/* nsteps steps, enqueued on the context stream. */
int fd_vti_step(fd_vti_ctx *ctx, int64_t nsteps);
int fd_vti_sync(fd_vti_ctx *ctx);
int fd_vti_get_step(const fd_vti_ctx *ctx, int64_t *step);

/* Dense copies (device, dtype, [nz][ny][nx]) of p^n, p^{n-1}, q^n, q^{n-1}; any may be NULL
 * (set_state: that field keeps its buffer, which is only valid if step has the parity of
 * the current step; otherwise all four are required, FD_E_INVAL). */
int fd_vti_get_state(fd_vti_ctx *ctx, void *p, void *p_prev, void *q, void *q_prev);
int fd_vti_set_state(fd_vti_ctx *ctx, const void *p, const void *p_prev, const void *q, const void *q_prev,
                     int64_t step);

/* Kernel tile configuration in use, and the tuning override (config index, z chunk; 0 = auto)
 * for contexts created afterwards. */
const char *fd_vti_kernel_config(const fd_vti_ctx *ctx);
int fd_vti_set_tuning(fd_dtype dtype, int rxy, int rz, int config, int zchunk);

#ifdef __cplusplus
}
#endif

#endif /* FDWAVE_H */
