"""C-ABI contract tests that need no GPU: the library loads, exports every symbol
include/fdwave.h declares, and its host-only entry points validate arguments and
agree with the oracle's independent stencil and stability computations."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fdwave.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def F():
    from paper_1410_1387_amd import fdwave

    if not os.path.exists(fdwave.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    fdwave.lib()
    return fdwave


def test_exports_every_declared_symbol(F):
    declared = _declared_symbols()
    assert len(declared) >= 25
    L = ctypes.CDLL(F.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(F.EXPORTS) == declared


def test_noalloc_limit_matches_header(F):
    # the binding's copy of the no-allocation batch's shot limit is the header's
    import re

    with open(os.path.join(ROOT, "include", "fdwave.h")) as f:
        m = re.search(r"#define FD_BATCH_NOALLOC_MAX_SHOTS (\d+)", f.read())
    assert m and int(m.group(1)) == F.FD_BATCH_NOALLOC_MAX_SHOTS


def test_weights_match_oracle(F, oracle_mod):
    for r in range(1, 13):
        w = np.array(F.fd_weights(r))
        wo = oracle_mod.weights_f64(r)
        assert np.array_equal(w[1:], wo[1:])  # both correctly rounded from exact rationals
        assert abs(w[0] - wo[0]) <= 4e-16 * abs(wo[0])


def test_dt_max_matches_oracle(F, oracle_mod):
    for ndim in (2, 3):
        for r in range(1, 9):
            a = F.fd_dt_max(ndim, r, 10.0, 4500.0)
            b = oracle_mod.dt_max(ndim, r, 10.0, 4500.0)
            assert abs(a - b) <= 1e-14 * b


def test_invalid_arguments_rejected(F):
    with pytest.raises(F.FdError) as e:
        F.fd_weights(0)
    assert e.value.status == F.FD_E_INVAL
    with pytest.raises(F.FdError):
        F.fd_weights(13)
    with pytest.raises(F.FdError):
        F.fd_dt_max(3, 4, -1.0, 1.0)
    for bad_shape, r in [((0, 4, 4), 4), ((4, 4, 4), 0), ((4, 4, 4), 9), ((5,), 2)]:
        with pytest.raises((F.FdError, ValueError)):
            F.fd_field_bytes(bad_shape, r, "f32")
    with pytest.raises(F.FdError):
        F.fd_workspace_bytes((8, 8, 8), 4, "f32", -1, 0)
    with pytest.raises(F.FdError) as e:
        F.fd_set_tuning("f32", 4, 3, 99)
    assert e.value.status == F.FD_E_RANGE
    assert F.fd_batch_workspace_bytes(0) == 0


def test_null_context_rejected(F):
    # entry points that take a context refuse a null one with FD_E_INVAL before touching
    # any device; the configuration queries give an empty string
    calls = [
        lambda: F.fd_step_explicit(None, None, None, None, 0),
        lambda: F.fd_step_record(None, None, None, None, 0),
        lambda: F.fd_adjoint_segment(None, None, None, 0, 1, None, None, None, 1.0, None),
        lambda: F.fd_adjoint_stored(None, None, 0, 1, None, None, 1.0, None),
        lambda: F.fd_clear_ghosts(None, None, 1),
        lambda: F.fd_gradient_finish(None, None, None, None, 1.0),
    ]
    for call in calls:
        with pytest.raises(F.FdError) as e:
            call()
        assert e.value.status == F.FD_E_INVAL
    assert F.fd_kernel_config(None) == "" and F.fd_adjoint_config(None) == ""


def test_layout_sizes(F):
    # padded field: interior plus r ghost cells on every face plus alignment padding
    for shape, r, dt, es in [((512, 512, 512), 4, "f32", 4), ((384, 384, 384), 8, "f32", 4),
                             ((256, 256), 4, "f64", 8), ((7, 9, 11), 1, "f64", 8)]:
        fb = F.fd_field_bytes(shape, r, dt)
        dense = int(np.prod(shape)) * es
        assert fb % 256 == 0 and fb >= dense
        if len(shape) == 3:
            nz, ny, nx = shape
            assert fb >= (nx + 2 * r) * (ny + 2 * r) * (nz + 2 * r) * es
        ws = F.fd_workspace_bytes(shape, r, dt, 2, 100)
        assert ws >= 3 * fb
    # 512^3 FP32 r=4: the padding overhead stays modest
    assert F.fd_field_bytes((512, 512, 512), 4, "f32") < 1.2 * 512 ** 3 * 4


def test_tuning_table_accepts_known_configs(F):
    for cfg in range(9):
        F.fd_set_tuning("f32", 4, 3, cfg)
    F.fd_set_tuning("f32", 4, 3, -1)  # back to the library's own choice
    with pytest.raises(F.FdError) as e:
        F.fd_set_tuning("f32", 4, 3, -2)
    assert e.value.status == F.FD_E_RANGE
    for cfg in range(6):
        F.fd_set_adj_tuning("f32", 4, 3, cfg)
    F.fd_set_adj_tuning("f32", 4, 3, -1)  # back to the library's own choice
    for bad in (6, -2):
        with pytest.raises(F.FdError) as e:
            F.fd_set_adj_tuning("f32", 4, 3, bad)
        assert e.value.status == F.FD_E_RANGE
    with pytest.raises(F.FdError) as e:
        F.fd_set_adj_tuning("f32", 0, 3, 0)
    assert e.value.status == F.FD_E_INVAL


# ----------------------------------------------------------------------------- VTI host entry points


def _stretched(nz, rz, dz, a=0.35):
    k = np.arange(-rz, nz + rz, dtype=np.float64)
    return np.round(dz * k * (1.0 + a * (k / nz) ** 2) * 64.0) / 64.0


@pytest.mark.parametrize("rz", [1, 2, 4, 8])
def test_vti_z_weights_match_oracle(F, oracle_mod, rz):
    # library: Fornberg's recursion in FP64; oracle: exact moment equations over the rationals
    for zc in (oracle_mod.uniform_z(12, rz, 10.0), _stretched(12, rz, 9.0)):
        got = F.fd_vti_z_weights(zc, 12, rz)
        ref = oracle_mod.z_weights(zc, rz)
        scale = np.abs(ref).sum(axis=1, keepdims=True)
        assert np.max(np.abs(got - ref) / scale) <= 1e-13


def test_vti_dt_max_matches_oracle(F, oracle_mod):
    for (rxy, rz, dz) in [(12, 8, 10.0), (4, 2, 7.0), (8, 4, 12.5)]:
        zc = oracle_mod.uniform_z(10, rz, dz)
        for (e, d) in [(0.0, 0.0), (0.25, 0.1), (0.2, 0.2)]:
            a = F.fd_vti_dt_max(rxy, rz, 10.0, zc, 10, 3000.0, e, d)
            b = oracle_mod.vti_dt_max(rxy, rz, 10.0, oracle_mod.z_weights(zc, rz), np.full((10, 2, 2), 3000.0), e, d)
            assert abs(a - b) <= 1e-12 * b
    # NULL coordinates mean a uniform spacing h
    zc = oracle_mod.uniform_z(6, 4, 10.0)
    assert F.fd_vti_dt_max(12, 4, 10.0, None, 6, 2500.0, 0.1, 0.05) == F.fd_vti_dt_max(12, 4, 10.0, zc, 6, 2500.0,
                                                                                       0.1, 0.05)


def test_vti_invalid_arguments_rejected(F):
    with pytest.raises(F.FdError):
        F.fd_vti_z_weights([0.0, 1.0, 1.0, 2.0, 3.0], 3, 1)          # not strictly increasing
    with pytest.raises(F.FdError):
        F.fd_vti_dt_max(6, 2, 10.0, None, 8, 2000.0, 0.1, 0.0)        # unsupported xy radius
    with pytest.raises(F.FdError):
        F.fd_vti_dt_max(4, 8, 10.0, None, 8, 2000.0, 0.1, 0.0)        # rz > rxy
    with pytest.raises(F.FdError):
        F.fd_vti_workspace_bytes((8, 8), 4, 2, "f32", 1, 0)            # 2-D grid
    with pytest.raises(F.FdError) as e:
        F.fd_vti_set_tuning("f32", 12, 8, 99)
    assert e.value.status == F.FD_E_RANGE
    ws = F.fd_vti_workspace_bytes((64, 64, 64), 12, 8, "f32", 1, 10)
    assert ws >= 7 * 64 ** 3 * 4


def test_c_program_links_and_runs(F, oracle_mod, tmp_path):
    # the boundary is usable from plain C: a C program that includes include/fdwave.h
    # and links libfdwave.so gets the same weights, stability limit and sizes as the
    # Python binding, and the error codes and messages of refused arguments
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    exe = tmp_path / "c_abi_check"
    libdir = os.path.dirname(F.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-L", libdir, "-lfdwave",
                    "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    vals = dict(line.split(" ", 1) for line in out.strip().splitlines())
    w = [float(x) for x in vals["w4"].split()]
    assert w == list(F.fd_weights(4))
    assert np.array_equal(np.array(w[1:]), oracle_mod.weights_f64(4)[1:])
    assert float(vals["dtmax3_r4"]) == F.fd_dt_max(3, 4, 10.0, 4500.0)
    assert int(vals["field_bytes"]) == F.fd_field_bytes((512, 512, 512), 4, "f32")
    assert int(vals["workspace_bytes"]) == F.fd_workspace_bytes((512, 512, 512), 4, "f32", 1, 16384)
    assert vals["bad_radius"] == f"{F.FD_E_INVAL} msg" and vals["bad_grid"] == f"{F.FD_E_INVAL} msg"
