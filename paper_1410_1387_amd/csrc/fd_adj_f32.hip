// fd_adj_f32.hip -- explicit instantiations of the adjoint stencil kernels for float
// and the (radius, ndim) -> tile-configuration table the host side dispatches on.
// Written by gen_registry.py; edit the tile lists there.
#include "fd_stencil.h"

namespace fdw {
static const AdjEntry a3_r1[] = {
    adj_entry<TileCfg<float, 1, 3, 32, 16, 1>>("f32 r1 3d tile 128x16 (512 thr, 1 row/thr)"),
    adj_entry<TileCfg<float, 1, 3, 16, 16, 1>>("f32 r1 3d tile 64x16 (256 thr, 1 row/thr)", ADJ_RAGGED_X),
};
static const AdjEntry a2_r1[] = {adj_entry<TileCfg<float, 1, 2, 64, 1, 1>>("f32 r1 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r2[] = {
    adj_entry<TileCfg<float, 2, 3, 32, 16, 1>>("f32 r2 3d tile 128x16 (512 thr, 1 row/thr)"),
    adj_entry<TileCfg<float, 2, 3, 16, 16, 1>>("f32 r2 3d tile 64x16 (256 thr, 1 row/thr)", ADJ_RAGGED_X),
};
static const AdjEntry a2_r2[] = {adj_entry<TileCfg<float, 2, 2, 64, 1, 1>>("f32 r2 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r3[] = {
    adj_entry<TileCfg<float, 3, 3, 32, 16, 1>>("f32 r3 3d tile 128x16 (512 thr, 1 row/thr)"),
    adj_entry<TileCfg<float, 3, 3, 16, 16, 1>>("f32 r3 3d tile 64x16 (256 thr, 1 row/thr)", ADJ_RAGGED_X),
};
static const AdjEntry a2_r3[] = {adj_entry<TileCfg<float, 3, 2, 64, 1, 1>>("f32 r3 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r4[] = {
    adj_entry<TileCfg<float, 4, 3, 32, 16, 1>>("f32 r4 3d tile 128x16 (512 thr, 1 row/thr)"),
    adj_entry<TileCfg<float, 4, 3, 32, 16, 1, 2>>("f32 r4 3d tile 64x16 (512 thr, 1 row/thr, 8-byte vectors)"),
    adj_entry<TileCfg<float, 4, 3, 64, 8, 1, 2>>("f32 r4 3d tile 128x8 (512 thr, 1 row/thr, 8-byte vectors)"),
    adj_entry<TileCfg<float, 4, 3, 32, 8, 1, 2>>("f32 r4 3d tile 64x8 (256 thr, 1 row/thr, 8-byte vectors)"),
    adj_entry<TileCfg<float, 4, 3, 16, 16, 1, 2>>("f32 r4 3d tile 32x16 (256 thr, 1 row/thr, 8-byte vectors)"),
    adj_entry<TileCfg<float, 4, 3, 16, 16, 1>>("f32 r4 3d tile 64x16 (256 thr, 1 row/thr)", ADJ_RAGGED_X),
};
static const AdjEntry a2_r4[] = {adj_entry<TileCfg<float, 4, 2, 64, 1, 1>>("f32 r4 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r5[] = {
    adj_entry<TileCfg<float, 5, 3, 16, 16, 1>>("f32 r5 3d tile 64x16 (256 thr, 1 row/thr)"),
};
static const AdjEntry a2_r5[] = {adj_entry<TileCfg<float, 5, 2, 64, 1, 1>>("f32 r5 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r6[] = {
    adj_entry<TileCfg<float, 6, 3, 16, 16, 1>>("f32 r6 3d tile 64x16 (256 thr, 1 row/thr)"),
};
static const AdjEntry a2_r6[] = {adj_entry<TileCfg<float, 6, 2, 64, 1, 1>>("f32 r6 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r7[] = {
    adj_entry<TileCfg<float, 7, 3, 16, 16, 1>>("f32 r7 3d tile 64x16 (256 thr, 1 row/thr)"),
};
static const AdjEntry a2_r7[] = {adj_entry<TileCfg<float, 7, 2, 64, 1, 1>>("f32 r7 2d tile 256x1 (64 thr, 1 row/thr)")};
static const AdjEntry a3_r8[] = {
    adj_entry<TileCfg<float, 8, 3, 16, 16, 1>>("f32 r8 3d tile 64x16 (256 thr, 1 row/thr)"),
    adj_entry<TileCfg<float, 8, 3, 32, 16, 1, 2>>("f32 r8 3d tile 64x16 (512 thr, 1 row/thr, 8-byte vectors)"),
};
static const AdjEntry a2_r8[] = {adj_entry<TileCfg<float, 8, 2, 64, 1, 1>>("f32 r8 2d tile 256x1 (64 thr, 1 row/thr)")};

const AdjEntry *adj_configs_f32(int r, int ndim, int *count)
{
    switch (r * 10 + ndim) {
    case 12: *count = (int)(sizeof(a2_r1) / sizeof(AdjEntry)); return a2_r1;
    case 13: *count = (int)(sizeof(a3_r1) / sizeof(AdjEntry)); return a3_r1;
    case 22: *count = (int)(sizeof(a2_r2) / sizeof(AdjEntry)); return a2_r2;
    case 23: *count = (int)(sizeof(a3_r2) / sizeof(AdjEntry)); return a3_r2;
    case 32: *count = (int)(sizeof(a2_r3) / sizeof(AdjEntry)); return a2_r3;
    case 33: *count = (int)(sizeof(a3_r3) / sizeof(AdjEntry)); return a3_r3;
    case 42: *count = (int)(sizeof(a2_r4) / sizeof(AdjEntry)); return a2_r4;
    case 43: *count = (int)(sizeof(a3_r4) / sizeof(AdjEntry)); return a3_r4;
    case 52: *count = (int)(sizeof(a2_r5) / sizeof(AdjEntry)); return a2_r5;
    case 53: *count = (int)(sizeof(a3_r5) / sizeof(AdjEntry)); return a3_r5;
    case 62: *count = (int)(sizeof(a2_r6) / sizeof(AdjEntry)); return a2_r6;
    case 63: *count = (int)(sizeof(a3_r6) / sizeof(AdjEntry)); return a3_r6;
    case 72: *count = (int)(sizeof(a2_r7) / sizeof(AdjEntry)); return a2_r7;
    case 73: *count = (int)(sizeof(a3_r7) / sizeof(AdjEntry)); return a3_r7;
    case 82: *count = (int)(sizeof(a2_r8) / sizeof(AdjEntry)); return a2_r8;
    case 83: *count = (int)(sizeof(a3_r8) / sizeof(AdjEntry)); return a3_r8;
    default: *count = 0; return nullptr;
    }
}

}  // namespace fdw
