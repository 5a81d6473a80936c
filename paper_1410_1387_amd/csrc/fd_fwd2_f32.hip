// fd_fwd2_f32.hip -- instantiations of the two-step (temporally blocked) forward kernel
// for FP32 and the radius -> tile-configuration table the host side dispatches on.
// First entry: the default.
#include "fd_fwd2.h"

namespace fdw {

static const Fwd2Entry k2_r4[] = {
    fwd2_entry<Tile2Cfg<float, 4, 16, 32>>("f32 r4 3d two-step tile 64x32 (512 thr)"),
    fwd2_entry<Tile2Cfg<float, 4, 16, 16>>("f32 r4 3d two-step tile 64x16 (256 thr)"),
    fwd2_entry<Tile2Cfg<float, 4, 32, 16>>("f32 r4 3d two-step tile 128x16 (512 thr)"),
};

const Fwd2Entry *fwd2_configs_f32(int r, int *count)
{
    switch (r) {
    case 4: *count = (int)(sizeof(k2_r4) / sizeof(Fwd2Entry)); return k2_r4;
    default: *count = 0; return nullptr;
    }
}

}  // namespace fdw
