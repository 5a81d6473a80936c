"""Parity at the stated workloads, full size and full step count (needs an MI355X).

* The 512^3 r = 4 FP32 layered shot, 1000 steps, Ricker 15 Hz at (256, 256, 16),
  128 x 128 receivers, in the benchmark's launch configuration: u^T, u^{T-1} and the
  traces against the FP64 oracle, relative L2 <= 1e-4 (Sec. 1 time scheme and stencil).
* The 256^3 r = 4 gradient workload (layered + 3 anomalies as the true model, layered
  start model, 2000 steps, checkpoints every 50): the FP32 GPU gradient against the
  oracle's checkpointed FP64 discrete adjoint, both given the oracle's FP64 residual
  (<= 1e-3) and end to end from FP64 observed data.
* The 384^3 r = 8 smoothed-noise shot, its stated 2000 steps (FD_PARITY_C3_STEPS sets
  fewer), against the oracle.
* The VTI benchmark workload's construction (layered vz, eps, delta; z spacing stretched
  with depth; R_xy = 12, R_z = 8) at 128^3 for 400 steps, full fields and traces.

The oracle runs in chunks and prints its progress outside pytest's capture, so a
long run shows that it is moving.  Named to run after the other GPU files: these are
the slowest tests (minutes of oracle time on the host)."""

import os
import time

import numpy as np
import pytest

import workloads
from gpu_util import oracle_forward_chunked, rel_l2, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture
def progress(capsys):
    t0 = time.time()

    def say(msg):
        with capsys.disabled():
            print(f"[full {time.time() - t0:7.1f} s] {msg}", flush=True)

    return say


def test_c2_full_shot_vs_oracle(oracle_mod, progress):
    shot = workloads.c2_3d_layered()
    v = shot.velocity()
    dt = shot.courant * oracle_mod.dt_max(3, shot.r, shot.h, v.max())
    T = shot.nsteps
    progress(f"{shot.name}: GPU FP32, {T} steps")
    got = run_gpu(v, shot.r, shot.h, dt, T, "f32", receivers=shot.receivers,
                  ricker=(shot.source, shot.f0, 1.5 / shot.f0), label=shot.name)
    assert got["step"] == T
    wav = oracle_mod.ricker(T, dt, shot.f0)
    ref = oracle_forward_chunked(oracle_mod, v, shot.h, dt, shot.r, T, [(shot.source, wav)], shot.receivers,
                                 progress)
    eu, ep = rel_l2(got["u"], ref["u"]), rel_l2(got["u_prev"], ref["u_prev"])
    et = rel_l2(got["traces"], ref["traces"])
    progress(f"{shot.name} x {T}: rel L2 u^T {eu:.2e} u^(T-1) {ep:.2e} traces {et:.2e} [{got['config']}]")
    assert np.linalg.norm(ref["u"]) > 0
    assert eu <= 1e-4 and ep <= 1e-4 and et <= 1e-4


def test_c3_shot_vs_oracle(oracle_mod, progress):
    shot = workloads.c3_3d_noise()
    T = int(os.environ.get("FD_PARITY_C3_STEPS", str(shot.nsteps)))
    assert 1 <= T <= shot.nsteps
    v = shot.velocity()
    dt = shot.courant * oracle_mod.dt_max(3, shot.r, shot.h, v.max())
    progress(f"{shot.name}: GPU FP32, {T} of the workload's {shot.nsteps} steps")
    got = run_gpu(v, shot.r, shot.h, dt, T, "f32", receivers=shot.receivers,
                  ricker=(shot.source, shot.f0, 1.5 / shot.f0), label=shot.name)
    wav = oracle_mod.ricker(T, dt, shot.f0)
    ref = oracle_forward_chunked(oracle_mod, v, shot.h, dt, shot.r, T, [(shot.source, wav)], shot.receivers,
                                 progress, chunk=200)
    eu, ep = rel_l2(got["u"], ref["u"]), rel_l2(got["u_prev"], ref["u_prev"])
    et = rel_l2(got["traces"], ref["traces"])
    progress(f"{shot.name} x {T}: rel L2 u^T {eu:.2e} u^(T-1) {ep:.2e} traces {et:.2e} [{got['config']}]")
    assert np.linalg.norm(ref["u"]) > 0
    assert eu <= 1e-4 and ep <= 1e-4 and et <= 1e-4


def test_vti_128_long_run_vs_oracle(oracle_mod, progress):
    import dataclasses

    from test_gpu_vti import run_vti_gpu

    shot = dataclasses.replace(workloads.VtiShot(), n=128, nsteps=400)
    vz, eps, delta = shot.models()
    zc = shot.zc()
    dt = shot.courant * oracle_mod.vti_dt_max(shot.rxy, shot.rz, shot.h, oracle_mod.z_weights(zc, shot.rz),
                                              vz, eps, delta)
    T, rec = shot.nsteps, shot.receivers()
    src = [(shot.source, oracle_mod.ricker(T, dt, shot.f0), 1.0, 0.0)]
    progress(f"VTI 128^3 rxy={shot.rxy} rz={shot.rz} x {T}: GPU FP32")
    out = run_vti_gpu(vz, eps, delta, shot.h, zc, dt, shot.rxy, shot.rz, T, "f32", sources=src, receivers=rec)
    progress("VTI 128^3: oracle")
    ref = oracle_mod.vti_forward(vz, eps, delta, shot.h, dt, shot.rxy, shot.rz, T, zc=zc, sources=src,
                                 receivers=rec)
    errs = {f: rel_l2(out[f], ref[f]) for f in ("p", "p_prev", "q", "q_prev", "traces_p", "traces_q")}
    progress(f"VTI 128^3 x {T}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) + f" [{out['config']}]")
    assert np.linalg.norm(ref["p"]) > 0
    assert all(e <= 1e-4 for e in errs.values()), errs


def test_c4_gradient_vs_oracle(oracle_mod, progress):
    import torch

    from paper_1410_1387_amd.autograd import GradientProblem, WaveProp, gradient

    case = workloads.GradientCase()
    v_true, v0 = case.models()
    dt = case.courant * oracle_mod.dt_max(3, case.r, case.h, float(max(v_true.max(), v0.max())))
    rec = case.receivers()
    T = case.nsteps
    wav = oracle_mod.ricker(T, dt, case.f0)
    obs = oracle_forward_chunked(oracle_mod, v_true, case.h, dt, case.r, T, [(case.source, wav)], rec, progress,
                                 chunk=250, what="oracle observed data (true model)")["traces"]
    ref = oracle_mod.gradient(v0, case.h, dt, case.r, T, [(case.source, wav)], rec, obs, checkpoint=case.ckpt,
                              progress=progress)
    g_ref = ref["grad_v"]
    pb = GradientProblem(r=case.r, h=case.h, dt=dt, nsteps=T, source=case.source, receivers=rec, f0=case.f0,
                         ckpt=case.ckpt, dtype="f32", states="all")
    progress("GPU FP32 gradient end to end (observed data from the oracle), every forward state kept")
    J32, g32 = gradient(torch.tensor(v0, dtype=torch.float32, device="cuda"), pb,
                        torch.tensor(obs, dtype=torch.float64, device="cuda"))
    e_e2e = rel_l2(g32.double().cpu().numpy(), g_ref)
    progress("the same gradient from checkpoints every 50 steps and recomputed segments")
    pb.states = "checkpoint"
    J32c, g32c = gradient(torch.tensor(v0, dtype=torch.float32, device="cuda"), pb,
                          torch.tensor(obs, dtype=torch.float64, device="cuda"))
    assert J32c == J32 and torch.equal(g32c, g32)
    del g32c
    torch.cuda.empty_cache()
    progress("GPU FP32 adjoint applied to the oracle's FP64 residual")
    resid = torch.tensor(ref["traces"] - obs, dtype=torch.float32, device="cuda")
    v32 = torch.tensor(v0, dtype=torch.float32, device="cuda").requires_grad_(True)
    tr32 = WaveProp.apply(v32, pb)
    (g_adj,) = torch.autograd.grad(tr32, v32, resid)
    e_adj = rel_l2(g_adj.double().cpu().numpy(), g_ref)
    eJ = abs(J32 - ref["J"]) / ref["J"]
    # how far the FP32 residual is from the FP64 one: the FP32 forward's rounding of the
    # traces (~sqrt(T) eps of their amplitude) over a misfit that is ~0.3 % of them
    tr32_np = tr32.detach().double().cpu().numpy()
    e_res = rel_l2(tr32_np - obs, ref["traces"] - obs)
    e_tr = rel_l2(tr32_np, ref["traces"])
    progress(f"256^3 x {T} gradient: J {J32:.6e} vs oracle {ref['J']:.6e} (rel {eJ:.1e}); "
             f"FP32 adjoint, oracle residual: rel L2 {e_adj:.2e}; FP32 end to end: rel L2 {e_e2e:.2e}; "
             f"FP32 traces rel L2 {e_tr:.2e}, FP32 residual rel L2 {e_res:.2e}")
    assert np.all(np.isfinite(g32.cpu().numpy()))
    assert e_tr <= 1e-4
    assert e_adj <= 1e-3
    # end to end the gradient inherits the residual's relative error (the adjoint is
    # linear in it); the bound leaves room for the adjoint's own amplification of it
    assert e_e2e <= 2e-2 and eJ <= 1e-3
