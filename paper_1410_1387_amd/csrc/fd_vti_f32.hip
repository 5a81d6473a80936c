// fd_vti_f32.hip -- explicit instantiations of the VTI stencil kernels for float
// and the (radius, ndim) -> tile-configuration table the host side dispatches on.
// Written by gen_registry.py; edit the tile lists there.
#include "fd_vti.h"

namespace fdw {
static const VtiEntry v_2_1[] = {
    vti_entry<VtiCfg<float, 2, 1, 16, 16>>("f32 vti rxy2 rz1 tile 64x16 (256 thr)"),
};
static const VtiEntry v_2_2[] = {
    vti_entry<VtiCfg<float, 2, 2, 16, 16>>("f32 vti rxy2 rz2 tile 64x16 (256 thr)"),
};
static const VtiEntry v_4_1[] = {
    vti_entry<VtiCfg<float, 4, 1, 16, 16>>("f32 vti rxy4 rz1 tile 64x16 (256 thr)"),
};
static const VtiEntry v_4_2[] = {
    vti_entry<VtiCfg<float, 4, 2, 16, 16>>("f32 vti rxy4 rz2 tile 64x16 (256 thr)"),
};
static const VtiEntry v_4_4[] = {
    vti_entry<VtiCfg<float, 4, 4, 16, 16>>("f32 vti rxy4 rz4 tile 64x16 (256 thr)"),
    vti_entry<VtiCfg<float, 4, 4, 32, 8>>("f32 vti rxy4 rz4 tile 128x8 (256 thr)"),
    vti_entry<VtiCfg<float, 4, 4, 16, 8>>("f32 vti rxy4 rz4 tile 64x8 (128 thr)"),
    vti_entry<VtiCfg<float, 4, 4, 32, 16>>("f32 vti rxy4 rz4 tile 128x16 (512 thr)"),
};
static const VtiEntry v_8_1[] = {
    vti_entry<VtiCfg<float, 8, 1, 16, 16>>("f32 vti rxy8 rz1 tile 64x16 (256 thr)"),
};
static const VtiEntry v_8_2[] = {
    vti_entry<VtiCfg<float, 8, 2, 16, 16>>("f32 vti rxy8 rz2 tile 64x16 (256 thr)"),
};
static const VtiEntry v_8_4[] = {
    vti_entry<VtiCfg<float, 8, 4, 16, 16>>("f32 vti rxy8 rz4 tile 64x16 (256 thr)"),
};
static const VtiEntry v_8_8[] = {
    vti_entry<VtiCfg<float, 8, 8, 16, 16>>("f32 vti rxy8 rz8 tile 64x16 (256 thr)"),
};
static const VtiEntry v_12_1[] = {
    vti_entry<VtiCfg<float, 12, 1, 16, 16>>("f32 vti rxy12 rz1 tile 64x16 (256 thr)"),
};
static const VtiEntry v_12_2[] = {
    vti_entry<VtiCfg<float, 12, 2, 16, 16>>("f32 vti rxy12 rz2 tile 64x16 (256 thr)"),
};
static const VtiEntry v_12_4[] = {
    vti_entry<VtiCfg<float, 12, 4, 16, 16>>("f32 vti rxy12 rz4 tile 64x16 (256 thr)"),
};
static const VtiEntry v_12_8[] = {
    vti_entry<VtiCfg<float, 12, 8, 16, 16>>("f32 vti rxy12 rz8 tile 64x16 (256 thr)"),
    vti_entry<VtiCfg<float, 12, 8, 32, 8>>("f32 vti rxy12 rz8 tile 128x8 (256 thr)"),
    vti_entry<VtiCfg<float, 12, 8, 16, 8>>("f32 vti rxy12 rz8 tile 64x8 (128 thr)"),
    vti_entry<VtiCfg<float, 12, 8, 32, 16>>("f32 vti rxy12 rz8 tile 128x16 (512 thr)"),
};

const VtiEntry *vti_configs_f32(int rxy, int rz, int *count)
{
    switch (rxy * 100 + rz) {
    case 201: *count = (int)(sizeof(v_2_1) / sizeof(VtiEntry)); return v_2_1;
    case 202: *count = (int)(sizeof(v_2_2) / sizeof(VtiEntry)); return v_2_2;
    case 401: *count = (int)(sizeof(v_4_1) / sizeof(VtiEntry)); return v_4_1;
    case 402: *count = (int)(sizeof(v_4_2) / sizeof(VtiEntry)); return v_4_2;
    case 404: *count = (int)(sizeof(v_4_4) / sizeof(VtiEntry)); return v_4_4;
    case 801: *count = (int)(sizeof(v_8_1) / sizeof(VtiEntry)); return v_8_1;
    case 802: *count = (int)(sizeof(v_8_2) / sizeof(VtiEntry)); return v_8_2;
    case 804: *count = (int)(sizeof(v_8_4) / sizeof(VtiEntry)); return v_8_4;
    case 808: *count = (int)(sizeof(v_8_8) / sizeof(VtiEntry)); return v_8_8;
    case 1201: *count = (int)(sizeof(v_12_1) / sizeof(VtiEntry)); return v_12_1;
    case 1202: *count = (int)(sizeof(v_12_2) / sizeof(VtiEntry)); return v_12_2;
    case 1204: *count = (int)(sizeof(v_12_4) / sizeof(VtiEntry)); return v_12_4;
    case 1208: *count = (int)(sizeof(v_12_8) / sizeof(VtiEntry)); return v_12_8;
    default: *count = 0; return nullptr;
    }
}

}  // namespace fdw
