"""The no-allocation batch (fd_batch_create_noalloc; needs an MI355X).  Its shot table is
the library's fixed device array instead of a caller workspace; every result must be
bitwise that of a batch created with a workspace (fd_batch_create), on two calls in a
row, the second with a smaller input, and the batched result is the oracle's."""

import numpy as np
import pytest

import workloads
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


def _shot(shape, nsteps, seed):
    v = workloads.layered_velocity(shape, seed=seed).astype(np.float32)
    nz, ny, nx = shape
    return v, (nx // 2, ny // 2, 2), workloads.surface_receivers(nx, ny, 2, 3), nsteps


def _make_ctx(F, v, src, rec, T, dt, stream):
    import torch

    vt = torch.tensor(v, device="cuda")
    ws = torch.empty(F.fd_workspace_bytes(v.shape, 4, "f32", 1, len(rec)), dtype=torch.uint8, device="cuda")
    wav = torch.empty(T, dtype=torch.float32, device="cuda")
    tr = torch.zeros((T, len(rec)), dtype=torch.float32, device="cuda")
    sp = F.stream_ptr(stream)
    ctx = F.fd_create(v.shape, 4, 10.0, dt, vt, "f32", "zero", ws, 1, len(rec), sp)
    F.fd_ricker(wav, dt, 30.0, 0.03, sp)
    F.fd_inject(ctx, wav, src, 1.0)
    F.fd_record(ctx, rec, tr, T)
    return ctx, [vt, ws, wav], tr


def _run_batch(F, shots, dt, stream, noalloc, chunks):
    """All shots in one batch stepped by `chunks`; returns [(u^n, u^{n-1}, traces, step)]."""
    import torch

    ctxs = [_make_ctx(F, v, src, rec, T, dt, stream) for (v, src, rec, T) in shots]
    sp = F.stream_ptr(stream)
    bws = None
    if noalloc:
        b = F.fd_batch_create_noalloc(len(shots), sp)
    else:
        bws = torch.empty(F.fd_batch_workspace_bytes(len(shots)), dtype=torch.uint8, device="cuda")
        b = F.fd_batch_create(len(shots), bws, sp)
    out = []
    try:
        F.fd_batch_set(b, [c[0] for c in ctxs], [s[3] for s in shots])
        for n in chunks:
            F.fd_batch_step(b, n)
        for (ctx, keep, tr), (v, *_r) in zip(ctxs, shots):
            u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
            up = torch.empty_like(u)
            F.fd_get_state(ctx, u, up)
            F.fd_sync(ctx)
            out.append((u.cpu().numpy(), up.cpu().numpy(), tr.cpu().numpy(), F.fd_get_step(ctx)))
    finally:
        F.fd_batch_destroy(b)
        for ctx, keep, tr in ctxs:
            F.fd_destroy(ctx)
    return out


def test_noalloc_batch_matches_workspace_batch(oracle_mod):
    import torch

    from paper_1410_1387_amd import fdwave as F

    stream = torch.cuda.Stream()
    cases = [
        ("three shots", [_shot((33, 40, 37), 47, 2), _shot((20, 24, 28), 30, 1), _shot((16, 16, 70), 21, 3)]),
        ("one smaller shot", [_shot((12, 14, 20), 25, 4)]),
    ]
    chunks = (8, 7, 16, 3, 16)  # odd and even lengths, past every shot's target
    for name, shots in cases:
        dt = 0.45 * min(oracle_mod.dt_max(3, 4, 10.0, float(s[0].max())) for s in shots)
        say(f"no-allocation batch, {name}: workspace batch first")
        ref = _run_batch(F, shots, dt, stream, False, chunks)
        say(f"no-allocation batch, {name}: fixed shot table")
        got = _run_batch(F, shots, dt, stream, True, chunks)
        for j, ((u, up, tr, n), (u_r, up_r, tr_r, n_r)) in enumerate(zip(got, ref)):
            assert n == n_r == shots[j][3], (name, j)
            assert np.array_equal(u, u_r) and np.array_equal(up, up_r), (name, j)
            assert np.array_equal(tr, tr_r), (name, j)
        v, src, rec, T = shots[0]
        orc = oracle_mod.forward(v.astype(np.float64), 10.0, dt, 4, T,
                                 [(src, oracle_mod.ricker(T, dt, 30.0, 0.03))], rec)
        assert rel_l2(got[0][2], orc["traces"]) <= 1e-4 and rel_l2(got[0][0], orc["u"]) <= 1e-4


def test_noalloc_batch_errors():
    import torch

    from paper_1410_1387_amd import fdwave as F

    stream = torch.cuda.Stream()
    sp = F.stream_ptr(stream)
    with pytest.raises(F.FdError, match="FD_E_RANGE"):
        F.fd_batch_create_noalloc(F.FD_BATCH_NOALLOC_MAX_SHOTS + 1, sp)
    with pytest.raises(F.FdError, match="FD_E_RANGE"):
        F.fd_batch_create_noalloc(0, sp)
    b = F.fd_batch_create_noalloc(4, sp)
    try:
        with pytest.raises(F.FdError, match="FD_E_STATE"):   # the device's table is held
            F.fd_batch_create_noalloc(4, sp)
        v, src, rec, T = _shot((12, 14, 20), 10, 5)
        ctx, keep, tr = _make_ctx(F, v, src, rec, T, 4e-4, torch.cuda.Stream())
        try:
            with pytest.raises(F.FdError, match="FD_E_INVAL"):   # member on another stream
                F.fd_batch_set(b, [ctx], [T])
        finally:
            F.fd_destroy(ctx)
    finally:
        F.fd_batch_destroy(b)
    b = F.fd_batch_create_noalloc(F.FD_BATCH_NOALLOC_MAX_SHOTS, sp)  # released by destroy
    F.fd_batch_destroy(b)
