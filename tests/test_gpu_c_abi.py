"""The device entry points from plain C (needs an MI355X): tests/c_abi_device.c, compiled
with gcc against include/fdwave.h, libfdwave.so and the HIP runtime's C API, runs one
forward shot (fd_create, fd_ricker, fd_inject, fd_record, fd_step, fd_get_state), and in
its gradient mode a whole velocity gradient (fd_clear_ghosts, fd_step_record,
fd_adjoint_stored, fd_gradient_finish), with no Python in the process; wavefields,
traces and gradients are compared with the FP64 oracle."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def c_exe(tmp_path_factory):
    from paper_1410_1387_amd import fdwave as F

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    exe = tmp_path_factory.mktemp("cabi") / "c_abi_device"
    libdir = os.path.dirname(F.LIB_PATH)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(rocm, "include"), os.path.join(ROOT, "tests", "c_abi_device.c"),
                    "-L", libdir, "-lfdwave", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + libdir, "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", str(exe)], check=True)
    return exe


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f64", 1e-11)])
def test_c_program_runs_a_shot(oracle_mod, c_exe, tmp_path, dtype, tol):
    shape, r, h, T, f0 = (37, 45, 70), 4, 10.0, 80, 25.0
    nz, ny, nx = shape
    npdt = np.float32 if dtype == "f32" else np.float64
    v = workloads.layered_velocity(shape, seed=21)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, v.max())
    src = (nx // 2, ny // 2, 5)
    rec = np.array([[x, y, 5] for y in range(0, ny, 4) for x in range(0, nx, 3)], dtype=np.int32)
    (tmp_path / "v.bin").write_bytes(np.ascontiguousarray(v, dtype=npdt).tobytes())
    (tmp_path / "rec.bin").write_bytes(rec.tobytes())
    num = lambda x: f"{float(x):.17g}"  # noqa: E731  (round-trips a double exactly)
    args = [str(c_exe), dtype, str(nx), str(ny), str(nz), str(r), num(h), num(dt), str(T), *map(str, src),
            num(f0), num(1.5 / f0), str(tmp_path / "v.bin"), str(tmp_path / "rec.bin"), str(len(rec)),
            str(tmp_path / "u.bin"), str(tmp_path / "tr.bin")]
    say(f"c program: {dtype} {shape} r={r} T={T}")
    res = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    out = dict(line.split(" ", 1) for line in res.stdout.strip().splitlines())
    assert int(out["step"]) == T
    u = np.frombuffer((tmp_path / "u.bin").read_bytes(), dtype=npdt).reshape(shape)
    tr = np.frombuffer((tmp_path / "tr.bin").read_bytes(), dtype=npdt).reshape(T, len(rec))
    ref = oracle_mod.forward(v, h, dt, r, T, [(src, oracle_mod.ricker(T, dt, f0))], rec)
    eu, et = rel_l2(u, ref["u"]), rel_l2(tr, ref["traces"])
    say(f"c program {dtype} ({out['config']}): rel L2 u {eu:.2e} traces {et:.2e}")
    assert np.linalg.norm(ref["u"]) > 0 and eu <= tol and et <= tol


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-3), ("f64", 1e-9)])
def test_c_program_runs_a_gradient(oracle_mod, c_exe, tmp_path, dtype, tol):
    # the differentiation pattern from plain C: every forward state kept (fd_clear_ghosts,
    # fd_step_record), the adjoint over them (fd_adjoint_stored) and dJ/dv
    # (fd_gradient_finish), given the oracle's FP64 residual; checked against the oracle's
    # gradient, its traces and u^{T-1}
    shape, r, h, T, f0 = (29, 34, 45), 4, 10.0, 70, 25.0
    nz, ny, nx = shape
    npdt = np.float32 if dtype == "f32" else np.float64
    v0 = workloads.layered_velocity(shape, seed=23)
    rng = np.random.default_rng(23)
    v_true = np.clip(v0 * (1 + 0.04 * rng.standard_normal(shape)), 0.5 * v0.min(), 1.05 * v0.max())
    dt = 0.5 * oracle_mod.dt_max(3, r, h, 1.05 * v0.max())
    src = (nx // 2, ny // 2, 3)
    rec = np.array([[x, y, 3] for y in range(1, ny - 1, 3) for x in range(1, nx - 1, 3)], dtype=np.int32)
    wav = oracle_mod.ricker(T, dt, f0)
    obs = oracle_mod.forward(v_true, h, dt, r, T, [(src, wav)], rec)["traces"]
    ref = oracle_mod.gradient(v0, h, dt, r, T, [(src, wav)], rec, obs)
    fw = oracle_mod.forward(v0, h, dt, r, T, [(src, wav)], rec)
    (tmp_path / "v.bin").write_bytes(np.ascontiguousarray(v0, dtype=npdt).tobytes())
    (tmp_path / "rec.bin").write_bytes(rec.tobytes())
    (tmp_path / "resid.bin").write_bytes(np.ascontiguousarray(fw["traces"] - obs, dtype=npdt).tobytes())
    num = lambda x: f"{float(x):.17g}"  # noqa: E731
    args = [str(c_exe), dtype, str(nx), str(ny), str(nz), str(r), num(h), num(dt), str(T), *map(str, src),
            num(f0), num(1.5 / f0), str(tmp_path / "v.bin"), str(tmp_path / "rec.bin"), str(len(rec)),
            str(tmp_path / "u.bin"), str(tmp_path / "tr.bin"), str(tmp_path / "resid.bin"), str(tmp_path / "g.bin")]
    say(f"c program gradient: {dtype} {shape} r={r} T={T}")
    res = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    g = np.frombuffer((tmp_path / "g.bin").read_bytes(), dtype=npdt).reshape(shape)
    u = np.frombuffer((tmp_path / "u.bin").read_bytes(), dtype=npdt).reshape(shape)
    tr = np.frombuffer((tmp_path / "tr.bin").read_bytes(), dtype=npdt).reshape(T, len(rec))
    eg, et, eu = rel_l2(g, ref["grad_v"]), rel_l2(tr, fw["traces"]), rel_l2(u, fw["u_prev"])
    say(f"c program gradient {dtype}: rel L2 grad {eg:.2e} traces {et:.2e} u^(T-1) {eu:.2e}")
    assert np.linalg.norm(ref["grad_v"]) > 0 and eg <= tol
    assert et <= (1e-4 if dtype == "f32" else 1e-11) and eu <= (1e-4 if dtype == "f32" else 1e-11)
