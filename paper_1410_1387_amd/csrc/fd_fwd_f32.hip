// fd_fwd_f32.hip -- explicit instantiations of the forward stencil kernels for float
// and the (radius, ndim) -> tile-configuration table the host side dispatches on.
// Written by gen_registry.py; edit the tile lists there.
#include "fd_stencil.h"

namespace fdw {
static const FwdEntry k3_r1[] = {
    fwd_entry<TileCfg<float, 1, 3, 16, 16, 1>>("f32 r1 3d tile 64x16 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 1, 3, 16, 16, 1, 4, 4>>("f32 r1 3d tile 64x16 (256 thr, 1 row/thr, built for 4 waves/SIMD)", FWD_SMALL_GRID),
};
static const FwdEntry k2_r1[] = {
    fwd_entry<TileCfg<float, 1, 2, 64, 1, 1>>("f32 r1 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r2[] = {
    fwd_entry<TileCfg<float, 2, 3, 16, 16, 1>>("f32 r2 3d tile 64x16 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 2, 3, 16, 16, 1, 4, 4>>("f32 r2 3d tile 64x16 (256 thr, 1 row/thr, built for 4 waves/SIMD)", FWD_SMALL_GRID),
};
static const FwdEntry k2_r2[] = {
    fwd_entry<TileCfg<float, 2, 2, 64, 1, 1>>("f32 r2 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r3[] = {
    fwd_entry<TileCfg<float, 3, 3, 16, 16, 1>>("f32 r3 3d tile 64x16 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 3, 3, 16, 16, 1, 4, 4>>("f32 r3 3d tile 64x16 (256 thr, 1 row/thr, built for 4 waves/SIMD)", FWD_SMALL_GRID),
};
static const FwdEntry k2_r3[] = {
    fwd_entry<TileCfg<float, 3, 2, 64, 1, 1>>("f32 r3 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r4[] = {
    fwd_entry<TileCfg<float, 4, 3, 16, 16, 1>>("f32 r4 3d tile 64x16 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 16, 16, 2>>("f32 r4 3d tile 64x32 (256 thr, 2 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 32, 8, 2>>("f32 r4 3d tile 128x16 (256 thr, 2 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 16, 8, 4>>("f32 r4 3d tile 64x32 (128 thr, 4 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 16, 32, 2>>("f32 r4 3d tile 64x64 (512 thr, 2 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 32, 16, 2>>("f32 r4 3d tile 128x32 (512 thr, 2 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 8, 32, 2>>("f32 r4 3d tile 32x64 (256 thr, 2 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 8, 32, 1>>("f32 r4 3d tile 32x32 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 4, 3, 16, 16, 1, 4, 4>>("f32 r4 3d tile 64x16 (256 thr, 1 row/thr, built for 4 waves/SIMD)", FWD_SMALL_GRID),
};
static const FwdEntry k2_r4[] = {
    fwd_entry<TileCfg<float, 4, 2, 64, 1, 1>>("f32 r4 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r5[] = {
    fwd_entry<TileCfg<float, 5, 3, 32, 16, 1>>("f32 r5 3d tile 128x16 (512 thr, 1 row/thr)"),
};
static const FwdEntry k2_r5[] = {
    fwd_entry<TileCfg<float, 5, 2, 64, 1, 1>>("f32 r5 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r6[] = {
    fwd_entry<TileCfg<float, 6, 3, 32, 16, 1>>("f32 r6 3d tile 128x16 (512 thr, 1 row/thr)"),
};
static const FwdEntry k2_r6[] = {
    fwd_entry<TileCfg<float, 6, 2, 64, 1, 1>>("f32 r6 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r7[] = {
    fwd_entry<TileCfg<float, 7, 3, 32, 16, 1>>("f32 r7 3d tile 128x16 (512 thr, 1 row/thr)"),
};
static const FwdEntry k2_r7[] = {
    fwd_entry<TileCfg<float, 7, 2, 64, 1, 1>>("f32 r7 2d tile 256x1 (64 thr, 1 row/thr)"),
};
static const FwdEntry k3_r8[] = {
    fwd_entry<TileCfg<float, 8, 3, 32, 16, 1>>("f32 r8 3d tile 128x16 (512 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 8, 3, 16, 16, 1>>("f32 r8 3d tile 64x16 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 8, 3, 32, 8, 1>>("f32 r8 3d tile 128x8 (256 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 8, 3, 16, 32, 1>>("f32 r8 3d tile 64x32 (512 thr, 1 row/thr)"),
    fwd_entry<TileCfg<float, 8, 3, 32, 16, 1, 2>>("f32 r8 3d tile 64x16 (512 thr, 1 row/thr, 8-byte vectors)"),
    fwd_entry<TileCfg<float, 8, 3, 32, 8, 1, 2>>("f32 r8 3d tile 64x8 (256 thr, 1 row/thr, 8-byte vectors)"),
    fwd_entry<TileCfg<float, 8, 3, 64, 8, 1, 2>>("f32 r8 3d tile 128x8 (512 thr, 1 row/thr, 8-byte vectors)"),
    fwd_entry<TileCfg<float, 8, 3, 16, 16, 1, 2>>("f32 r8 3d tile 32x16 (256 thr, 1 row/thr, 8-byte vectors)"),
    fwd_entry<TileCfg<float, 8, 3, 64, 4, 1, 2>>("f32 r8 3d tile 128x4 (256 thr, 1 row/thr, 8-byte vectors)"),
};
static const FwdEntry k2_r8[] = {
    fwd_entry<TileCfg<float, 8, 2, 64, 1, 1>>("f32 r8 2d tile 256x1 (64 thr, 1 row/thr)"),
};

const FwdEntry *fwd_configs_f32(int r, int ndim, int *count)
{
    switch (r * 10 + ndim) {
    case 12: *count = (int)(sizeof(k2_r1) / sizeof(FwdEntry)); return k2_r1;
    case 13: *count = (int)(sizeof(k3_r1) / sizeof(FwdEntry)); return k3_r1;
    case 22: *count = (int)(sizeof(k2_r2) / sizeof(FwdEntry)); return k2_r2;
    case 23: *count = (int)(sizeof(k3_r2) / sizeof(FwdEntry)); return k3_r2;
    case 32: *count = (int)(sizeof(k2_r3) / sizeof(FwdEntry)); return k2_r3;
    case 33: *count = (int)(sizeof(k3_r3) / sizeof(FwdEntry)); return k3_r3;
    case 42: *count = (int)(sizeof(k2_r4) / sizeof(FwdEntry)); return k2_r4;
    case 43: *count = (int)(sizeof(k3_r4) / sizeof(FwdEntry)); return k3_r4;
    case 52: *count = (int)(sizeof(k2_r5) / sizeof(FwdEntry)); return k2_r5;
    case 53: *count = (int)(sizeof(k3_r5) / sizeof(FwdEntry)); return k3_r5;
    case 62: *count = (int)(sizeof(k2_r6) / sizeof(FwdEntry)); return k2_r6;
    case 63: *count = (int)(sizeof(k3_r6) / sizeof(FwdEntry)); return k3_r6;
    case 72: *count = (int)(sizeof(k2_r7) / sizeof(FwdEntry)); return k2_r7;
    case 73: *count = (int)(sizeof(k3_r7) / sizeof(FwdEntry)); return k3_r7;
    case 82: *count = (int)(sizeof(k2_r8) / sizeof(FwdEntry)); return k2_r8;
    case 83: *count = (int)(sizeof(k3_r8) / sizeof(FwdEntry)); return k3_r8;
    default: *count = 0; return nullptr;
    }
}

}  // namespace fdw
