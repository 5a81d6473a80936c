/* A C program that runs one forward shot through include/fdwave.h and libfdwave.so on the
 * GPU, with no Python and no torch: device memory comes from the HIP runtime's C API.
 *
 *   c_abi_device DTYPE(f32|f64) NX NY NZ R H DT NSTEPS SX SY SZ F0 T0 VEL.bin REC.bin NREC
 *                OUT_U.bin OUT_TRACES.bin [RESID.bin OUT_GRAD.bin]
 *
 * VEL.bin: dense velocity [NZ][NY][NX] in DTYPE; REC.bin: int32 [NREC][3] receiver
 * positions.  The program creates a context, computes Ricker samples on the device
 * (fd_ricker), registers the source and receivers, steps NSTEPS times, and writes the
 * dense u^NSTEPS and the traces [NSTEPS][NREC] (DTYPE) to the output files.  It prints
 * "step N" and "config NAME" and exits non-zero on any error.  With RESID.bin (the
 * residual [NSTEPS][NREC] in DTYPE) it instead runs the gradient with every forward
 * state kept: NSTEPS + 1 padded fields (fd_field_bytes each; ghosts cleared by
 * fd_clear_ghosts, the two starting fields zeroed), the forward pass by fd_step_record
 * into them (traces recorded), the adjoint by fd_adjoint_stored over the whole run, and
 * dJ/dv by fd_gradient_finish, written dense to OUT_GRAD.bin; OUT_U.bin then holds
 * u^{NSTEPS-1}.  Compiled and run by test_gpu_c_abi.py. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "fdwave.h"

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                  \
            return 10;                                                                  \
        }                                                                               \
    } while (0)
#define FD_OK_(call)                                                                    \
    do {                                                                                \
        int s_ = (call);                                                                \
        if (s_ != FD_OK) {                                                              \
            fprintf(stderr, "%s: status %d: %s\n", #call, s_, fd_last_error());         \
            return 11;                                                                  \
        }                                                                               \
    } while (0)

static void *read_file(const char *path, size_t bytes)
{
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    void *p = malloc(bytes);
    if (p && fread(p, 1, bytes, f) != bytes) {
        free(p);
        p = NULL;
    }
    fclose(f);
    return p;
}

static int write_file(const char *path, const void *p, size_t bytes)
{
    FILE *f = fopen(path, "wb");
    if (!f) return 1;
    const size_t n = fwrite(p, 1, bytes, f);
    fclose(f);
    return n != bytes;
}

/* The gradient mode (see the header comment): every forward state kept, no recompute. */
static int gradient(fd_ctx *ctx, const fd_grid *g, int r, fd_dtype dt_code, size_t es, size_t npts, int64_t T,
                    int64_t nrec, const void *d_v, void *d_u, const char *resid_path, const char *grad_path,
                    hipStream_t stream)
{
    size_t fb = 0;
    FD_OK_(fd_field_bytes(g, r, dt_code, &fb));
    char *states, *mu, *grad;
    void *d_resid, *d_gout;
    HIP_OK(hipMalloc((void **)&states, (size_t)(T + 1) * fb));
    HIP_OK(hipMalloc((void **)&mu, 2 * fb));
    HIP_OK(hipMalloc((void **)&grad, fb));
    HIP_OK(hipMalloc(&d_resid, (size_t)T * (size_t)nrec * es));
    HIP_OK(hipMalloc(&d_gout, npts * es));
    void *h_resid = read_file(resid_path, (size_t)T * (size_t)nrec * es);
    if (!h_resid) {
        fprintf(stderr, "cannot read the residual\n");
        return 3;
    }
    HIP_OK(hipMemcpy(d_resid, h_resid, (size_t)T * (size_t)nrec * es, hipMemcpyHostToDevice));
    HIP_OK(hipMemsetAsync(mu, 0, 2 * fb, stream));
    HIP_OK(hipMemsetAsync(grad, 0, fb, stream));
    /* field k holds u^k (k < T); field T holds u^{-1} = 0 and then takes u^T */
    HIP_OK(hipMemsetAsync(states, 0, fb, stream));
    HIP_OK(hipMemsetAsync(states + (size_t)T * fb, 0, fb, stream));
    FD_OK_(fd_clear_ghosts(ctx, states, T + 1));
    const char *prev = states + (size_t)T * fb, *cur = states;
    for (int64_t k = 0; k < T; ++k) {
        char *out = k + 1 < T ? states + (size_t)(k + 1) * fb : states + (size_t)T * fb;
        FD_OK_(fd_step_record(ctx, cur, prev, out, k));
        prev = cur;
        cur = out;
    }
    FD_OK_(fd_adjoint_stored(ctx, states, 0, T, mu, d_resid, 1.0, grad, NULL));
    FD_OK_(fd_gradient_finish(ctx, grad, d_v, d_gout, 1.0));
    int64_t step = -1;
    FD_OK_(fd_set_state(ctx, states + (size_t)(T - 1) * fb, NULL, T - 1, FD_PADDED));
    FD_OK_(fd_get_state(ctx, d_u, NULL, &step, FD_DENSE));
    FD_OK_(fd_sync(ctx));
    void *h_g = malloc(npts * es);
    if (!h_g) return 4;
    HIP_OK(hipMemcpy(h_g, d_gout, npts * es, hipMemcpyDeviceToHost));
    if (write_file(grad_path, h_g, npts * es)) {
        fprintf(stderr, "cannot write the gradient\n");
        return 5;
    }
    free(h_g);
    free(h_resid);
    HIP_OK(hipFree(states));
    HIP_OK(hipFree(mu));
    HIP_OK(hipFree(grad));
    HIP_OK(hipFree(d_resid));
    HIP_OK(hipFree(d_gout));
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 19 && argc != 21) {
        fprintf(stderr, "usage: see the header comment of c_abi_device.c\n");
        return 2;
    }
    const fd_dtype dt_code = strcmp(argv[1], "f64") == 0 ? FD_F64 : FD_F32;
    const size_t es = dt_code == FD_F64 ? 8 : 4;
    fd_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = 3;
    g.n[0] = atoll(argv[2]);
    g.n[1] = atoll(argv[3]);
    g.n[2] = atoll(argv[4]);
    const int r = atoi(argv[5]);
    const double h = atof(argv[6]), dt = atof(argv[7]);
    const int64_t T = atoll(argv[8]);
    const int64_t src[3] = {atoll(argv[9]), atoll(argv[10]), atoll(argv[11])};
    const double f0 = atof(argv[12]), t0 = atof(argv[13]);
    const int64_t nrec = atoll(argv[16]);
    const size_t npts = (size_t)(g.n[0] * g.n[1] * g.n[2]);

    void *h_v = read_file(argv[14], npts * es);
    int32_t *h_rec = (int32_t *)read_file(argv[15], (size_t)nrec * 3 * sizeof(int32_t));
    if (!h_v || !h_rec) {
        fprintf(stderr, "cannot read the input files\n");
        return 3;
    }
    size_t ws_bytes = 0;
    FD_OK_(fd_workspace_bytes(&g, r, dt_code, 1, nrec, &ws_bytes));

    void *d_v, *d_ws, *d_wav, *d_tr, *d_u;
    HIP_OK(hipMalloc(&d_v, npts * es));
    HIP_OK(hipMalloc(&d_ws, ws_bytes));  /* hipMalloc returns 256-byte aligned memory */
    HIP_OK(hipMalloc(&d_wav, (size_t)T * es));
    HIP_OK(hipMalloc(&d_tr, (size_t)T * (size_t)nrec * es));
    HIP_OK(hipMalloc(&d_u, npts * es));
    HIP_OK(hipMemcpy(d_v, h_v, npts * es, hipMemcpyHostToDevice));
    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));

    fd_ctx *ctx = NULL;
    FD_OK_(fd_create(&ctx, &g, r, h, dt, d_v, dt_code, FD_BC_ZERO, d_ws, ws_bytes, 1, nrec, stream));
    FD_OK_(fd_ricker(d_wav, T, dt, f0, t0, dt_code, stream));
    FD_OK_(fd_inject(ctx, d_wav, T, src, 1.0));
    FD_OK_(fd_record(ctx, h_rec, nrec, d_tr, T));
    int64_t step = -1;
    if (argc == 19) {
        FD_OK_(fd_step(ctx, T));
        FD_OK_(fd_get_state(ctx, d_u, NULL, &step, FD_DENSE));
        FD_OK_(fd_sync(ctx));
    } else {
        int st = gradient(ctx, &g, r, dt_code, es, npts, T, nrec, d_v, d_u, argv[19], argv[20], stream);
        if (st) return st;
        step = T;
    }
    printf("step %lld\nconfig %s\n", (long long)step, fd_kernel_config(ctx));

    void *h_u = malloc(npts * es), *h_tr = malloc((size_t)T * (size_t)nrec * es);
    if (!h_u || !h_tr) return 4;
    HIP_OK(hipMemcpy(h_u, d_u, npts * es, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_tr, d_tr, (size_t)T * (size_t)nrec * es, hipMemcpyDeviceToHost));
    if (write_file(argv[17], h_u, npts * es) || write_file(argv[18], h_tr, (size_t)T * (size_t)nrec * es)) {
        fprintf(stderr, "cannot write the output files\n");
        return 5;
    }
    FD_OK_(fd_destroy(ctx));
    HIP_OK(hipStreamDestroy(stream));
    HIP_OK(hipFree(d_v));
    HIP_OK(hipFree(d_ws));
    HIP_OK(hipFree(d_wav));
    HIP_OK(hipFree(d_tr));
    HIP_OK(hipFree(d_u));
    free(h_v);
    free(h_rec);
    free(h_u);
    free(h_tr);
    return 0;
}
