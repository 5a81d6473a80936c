"""Writes the kernel-registry translation units fd_fwd_{f32,f64}.hip,
fd_adj_{f32,f64}.hip and fd_vti_{f32,f64}.hip: explicit template instantiations of the
stencil kernels and the (radius, ndim) -> tile-configuration tables (for the VTI
kernel: (xy radius, z radius) -> tiles) the host side dispatches on.

Tile shapes are (threads along x, threads along y, rows per thread); the first entry
of each list is the default.  Rerun after editing the lists:
    python paper_1410_1387_amd/csrc/gen_registry.py
"""

import os

HERE = os.path.dirname(os.path.abspath(__file__))

# 3-D forward tile shapes.  Radii in SWEEP_RADII get every shape; others the default.
# 64x16 with one row per thread first: 138 VGPRs and 41 KB of LDS give three 256-thread
# workgroups per CU, and at 512^3 r = 4 the chunker fills them with 768 workgroups of
# 171 planes (352 Gpts/s against 342 for 64x32 with two rows per thread)
F32_3D = [(16, 16, 1), (16, 16, 2), (32, 8, 2), (16, 8, 4), (16, 32, 2), (32, 16, 2), (8, 32, 2), (8, 32, 1)]
# radii above 4 keep one row per thread: two rows exceed 256 VGPRs and spill; 128x16
# (512 threads) first: measured fastest at 384^3, r = 8
F32_3D_BIG_R = [(32, 16, 1), (16, 16, 1), (32, 8, 1), (16, 32, 1),
                (32, 16, 1, 2), (32, 8, 1, 2), (64, 8, 1, 2), (16, 16, 1, 2), (64, 4, 1, 2)]
# FP64: 32x32 (two rows per thread) first for radii <= 4: 64x16 with 512 threads needs
# 83 KB of LDS at r = 4, one workgroup per CU (512^3 r = 4: 174.6 vs 129.2 Gpts/s);
# larger radii keep one row per thread (two rows spill at r >= 7); 32x16 measured fastest
# at 384^3 r = 8 (116.5 vs 110.0 Gpts/s for 64x16)
F64_3D = [(16, 16, 2), (32, 16, 1), (32, 8, 2), (16, 16, 1)]
F64_3D_BIG_R = [(16, 16, 1), (32, 16, 1), (32, 8, 1)]
F32_SWEEP_RADII = {4, 8}
# FP32 3-D, radii <= 4: the default tile built for 4 waves per SIMD (124 VGPRs, one set of
# prefetch registers, the early halo one plane later so that four workgroups' LDS fits a
# CU).  The library takes it by itself for grids whose default z chunk is 16-63 planes
# (fd_create): 1.05-1.06x at 256^3 and 320^3, 0.97-0.99x at 400^3 and 512^3.
F32_SMALL_GRID = (16, 16, 1, None, 4)
F64_SWEEP_RADII = {4, 8}
F2D = (64, 1, 1)          # 2-D forward and adjoint: one row of 64 threads
# adjoint: radii <= 4 128x16 first (measured 5-7 % faster than 64x16)
ADJ_F32_3D = [(32, 16, 1), (32, 16, 1, 2), (64, 8, 1, 2), (32, 8, 1, 2), (16, 16, 1, 2)]
# FP32 3-D adjoint, radii <= 4: a 64-wide tile (256 threads) for grids whose rows leave many
# of the default 128-wide tile's lanes idle; fd_create takes it by itself there (measured,
# 205 launches each: 320^3 190.0 vs 203.3 us, 192^3 47.2 vs 53.6, 160^3 32.0 vs 38.5; where
# 128 divides the row the default is faster: 256^3 92.8 vs 97.0, 512^3 700 vs 733)
ADJ_F32_RAGGED_X = (16, 16, 1)
ADJ_F32_3D_BIG_R = [(16, 16, 1), (32, 16, 1, 2)]  # radii > 4: two queues of 2r+2 planes
ADJ_F64_3D = [(32, 16, 1)]        # radii <= 4: 64x16, 512 threads (256^3: 176.0 vs 189.8 us for 64x8)
ADJ_F64_3D_BIG_R = [(32, 8, 1)]
ADJ_SWEEP_RADII = {4, 8}
# VTI kernel: (xy radius, z radius) pairs and tile shapes (threads along x, rows along y)
VTI_RADII = [(2, 1), (2, 2), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2), (8, 4), (8, 8),
             (12, 1), (12, 2), (12, 4), (12, 8)]
VTI_F32 = [(16, 16), (32, 8), (16, 8), (32, 16)]
VTI_F64 = [(16, 16), (32, 8)]
VTI_SWEEP = {(12, 8), (4, 4)}

HDR = """// {fname} -- explicit instantiations of the {what} stencil kernels for {T}
// and the (radius, ndim) -> tile-configuration table the host side dispatches on.
// Written by gen_registry.py; edit the tile lists there.
#include "fd_stencil.h"

namespace fdw {{
"""


def cfgname(T, R, nd, txn, tyn, ey, vec=None, occ=0):
    full = 4 if T == "float" else 2
    vec = vec or full
    bx = txn * vec
    by = tyn * ey if nd == 3 else 1
    nt = txn * (tyn if nd == 3 else 1)
    name = f"{'f32' if T == 'float' else 'f64'} r{R} {nd}d tile {bx}x{by} ({nt} thr, {ey if nd == 3 else 1} row/thr"
    if vec != full:
        name += f", {vec * (4 if T == 'float' else 8)}-byte vectors"
    if occ:
        name += f", built for {occ} waves/SIMD"
    return name + ")"


def tilecfg(T, R, nd, txn, tyn, ey, vec=None, occ=0):
    """TileCfg<...> for a tile tuple (threads along x, threads along y, rows per thread
    [, x points per thread (None: one 16-byte vector) [, waves per SIMD the forward
    kernel is built for (0: the compiler's choice)]])."""
    full = 4 if T == "float" else 2
    if occ:
        return f"TileCfg<{T}, {R}, {nd}, {txn}, {tyn}, {ey}, {vec or full}, {occ}>"
    return f"TileCfg<{T}, {R}, {nd}, {txn}, {tyn}, {ey}" + (f", {vec}>" if vec else ">")


def fwd_file(T, sweep3d, sweep_radii, sweep3d_big_r=None, small_grid=None):
    tag = "f32" if T == "float" else "f64"
    out = HDR.format(fname=f"fd_fwd_{tag}.hip", what="forward", T=T)
    for R in range(1, 9):
        lst = sweep3d_big_r if (sweep3d_big_r and R > 4) else sweep3d
        cfgs3 = lst if R in sweep_radii else lst[:1]
        out += f"static const FwdEntry k3_r{R}[] = {{\n"
        for cfg in cfgs3:
            out += f'    fwd_entry<{tilecfg(T, R, 3, *cfg)}>("{cfgname(T, R, 3, *cfg)}"),\n'
        if small_grid and R <= 4:
            out += (f'    fwd_entry<{tilecfg(T, R, 3, *small_grid)}>("{cfgname(T, R, 3, *small_grid)}", '
                    f'FWD_SMALL_GRID),\n')
        out += "};\n"
        txn = F2D[0]
        out += f"static const FwdEntry k2_r{R}[] = {{\n"
        out += f'    fwd_entry<TileCfg<{T}, {R}, 2, {txn}, 1, 1>>("{cfgname(T, R, 2, txn, 1, 1)}"),\n'
        out += "};\n"
    out += "\nconst FwdEntry *fwd_configs_" + tag + "(int r, int ndim, int *count)\n{\n    switch (r * 10 + ndim) {\n"
    for R in range(1, 9):
        for nd in (2, 3):
            out += f"    case {R * 10 + nd}: *count = (int)(sizeof(k{nd}_r{R}) / sizeof(FwdEntry)); return k{nd}_r{R};\n"
    out += "    default: *count = 0; return nullptr;\n    }\n}\n\n}  // namespace fdw\n"
    with open(os.path.join(HERE, f"fd_fwd_{tag}.hip"), "w") as f:
        f.write(out)


def adj_file(T, d3, d3_big_r=None, ragged_x=None):
    """Adjoint kernels: a list of 3-D tile shapes per radius (the first is the default),
    the ragged-row build for radii <= 4 (if given), and one 2-D shape."""
    tag = "f32" if T == "float" else "f64"
    out = HDR.format(fname=f"fd_adj_{tag}.hip", what="adjoint", T=T)
    for R in range(1, 9):
        lst = d3_big_r if (d3_big_r and R > 4) else d3
        lst = lst if R in ADJ_SWEEP_RADII else lst[:1]
        out += f"static const AdjEntry a3_r{R}[] = {{\n"
        for cfg in lst:
            out += f'    adj_entry<{tilecfg(T, R, 3, *cfg)}>("{cfgname(T, R, 3, *cfg)}"),\n'
        if ragged_x and R <= 4:
            out += (f'    adj_entry<{tilecfg(T, R, 3, *ragged_x)}>("{cfgname(T, R, 3, *ragged_x)}", '
                    f'ADJ_RAGGED_X),\n')
        out += "};\n"
        txn = F2D[0]
        out += (f"static const AdjEntry a2_r{R}[] = {{adj_entry<TileCfg<{T}, {R}, 2, {txn}, 1, 1>>"
                f'("{cfgname(T, R, 2, txn, 1, 1)}")}};\n')
    out += "\nconst AdjEntry *adj_configs_" + tag + "(int r, int ndim, int *count)\n{\n    switch (r * 10 + ndim) {\n"
    for R in range(1, 9):
        for nd in (2, 3):
            out += (f"    case {R * 10 + nd}: *count = (int)(sizeof(a{nd}_r{R}) / sizeof(AdjEntry)); "
                    f"return a{nd}_r{R};\n")
    out += "    default: *count = 0; return nullptr;\n    }\n}\n\n"
    out += "}  // namespace fdw\n"
    with open(os.path.join(HERE, f"fd_adj_{tag}.hip"), "w") as f:
        f.write(out)


def vti_file(T, tiles):
    tag = "f32" if T == "float" else "f64"
    vec = 4 if T == "float" else 2
    out = HDR.format(fname=f"fd_vti_{tag}.hip", what="VTI", T=T).replace('#include "fd_stencil.h"',
                                                                         '#include "fd_vti.h"')
    for (rxy, rz) in VTI_RADII:
        lst = tiles if (rxy, rz) in VTI_SWEEP else tiles[:1]
        out += f"static const VtiEntry v_{rxy}_{rz}[] = {{\n"
        for (txn, tyn) in lst:
            name = f"{tag} vti rxy{rxy} rz{rz} tile {txn * vec}x{tyn} ({txn * tyn} thr)"
            out += f'    vti_entry<VtiCfg<{T}, {rxy}, {rz}, {txn}, {tyn}>>("{name}"),\n'
        out += "};\n"
    out += "\nconst VtiEntry *vti_configs_" + tag + "(int rxy, int rz, int *count)\n{\n    switch (rxy * 100 + rz) {\n"
    for (rxy, rz) in VTI_RADII:
        out += (f"    case {rxy * 100 + rz}: *count = (int)(sizeof(v_{rxy}_{rz}) / sizeof(VtiEntry)); "
                f"return v_{rxy}_{rz};\n")
    out += "    default: *count = 0; return nullptr;\n    }\n}\n\n}  // namespace fdw\n"
    with open(os.path.join(HERE, f"fd_vti_{tag}.hip"), "w") as f:
        f.write(out)


if __name__ == "__main__":
    fwd_file("float", F32_3D, F32_SWEEP_RADII, F32_3D_BIG_R, F32_SMALL_GRID)
    fwd_file("double", F64_3D, F64_SWEEP_RADII, F64_3D_BIG_R)
    adj_file("float", ADJ_F32_3D, ADJ_F32_3D_BIG_R, ADJ_F32_RAGGED_X)
    adj_file("double", ADJ_F64_3D, ADJ_F64_3D_BIG_R)
    vti_file("float", VTI_F32)
    vti_file("double", VTI_F64)
