"""Batched (graph-replayed) stepping and the continuous-batching shot server (needs an
MI355X).  A shot must give bitwise the same traces and wavefield alone and in any mix,
because the per-point arithmetic of the batched kernel is that of the single-shot one."""

import numpy as np
import pytest

import workloads
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


def _shot(shape, nsteps, seed):
    v = workloads.layered_velocity(shape, seed=seed).astype(np.float32)
    nz, ny, nx = shape
    src = (nx // 2, ny // 2, 2)
    rec = workloads.surface_receivers(nx, ny, 2, 3)
    return v, src, rec, nsteps


def _make_ctx(v, src, rec, T, dt, stream):
    import torch

    from paper_1410_1387_amd import fdwave as F

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


def test_batched_graph_replays_match_single(oracle_mod):
    import torch

    from paper_1410_1387_amd import fdwave as F

    shots = [_shot((20, 24, 28), 30, 1), _shot((33, 40, 37), 47, 2), _shot((16, 16, 70), 21, 3)]
    dt = 0.45 * min(oracle_mod.dt_max(3, 4, 10.0, float(s[0].max())) for s in shots)
    stream = torch.cuda.Stream()
    chunk = 8
    # eager reference: each shot alone, state saved at every chunk boundary
    refs = []
    for (v, src, rec, T) in shots:
        ctx, keep, tr = _make_ctx(v, src, rec, T, dt, stream)
        states = []
        done = 0
        while done < T:
            n = min(chunk, T - done)
            F.fd_step(ctx, n)
            done += n
            u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
            F.fd_get_state(ctx, u, None)
            F.fd_sync(ctx)
            states.append(u.cpu().numpy())
        refs.append((states, tr.cpu().numpy()))
        F.fd_destroy(ctx)
    # batched: one launch per step for all three shots, graph-captured chunks
    ctxs = [_make_ctx(v, src, rec, T, dt, stream) for (v, src, rec, T) in shots]
    bws = torch.empty(F.fd_batch_workspace_bytes(4), dtype=torch.uint8, device="cuda")
    b = F.fd_batch_create(4, bws, F.stream_ptr(stream))
    F.fd_batch_set(b, [c[0] for c in ctxs], [s[3] for s in shots])
    for i in range(max(len(r[0]) for r in refs)):
        say(f"batched chunk {i}")
        F.fd_batch_step(b, chunk)
        stream.synchronize()
        for j, (ctx, keep, tr) in enumerate(ctxs):
            states = refs[j][0]
            k = min(i, len(states) - 1)
            u = torch.empty(shots[j][0].shape, dtype=torch.float32, device="cuda")
            F.fd_get_state(ctx, u, None)
            F.fd_sync(ctx)
            assert F.fd_get_step(ctx) == min((i + 1) * chunk, shots[j][3])
            assert np.array_equal(u.cpu().numpy(), states[k]), (i, j)
    for j, (ctx, keep, tr) in enumerate(ctxs):
        assert np.array_equal(tr.cpu().numpy(), refs[j][1])
        F.fd_destroy(ctx)
    F.fd_batch_destroy(b)
    # and the batched result is the oracle's
    v, src, rec, T = shots[1]
    ref = oracle_mod.forward(v.astype(np.float64), 10.0, dt, 4, T, [(src, oracle_mod.ricker(T, dt, 30.0, 0.03))], rec)
    assert rel_l2(refs[1][1], ref["traces"]) <= 1e-4


def test_batch_of_members_with_different_tile_builds(oracle_mod):
    # the library gives a 256^3 grid the 4-waves build of the tile and a small grid the
    # default one; a batch of both steps them with one kernel, bitwise as each alone
    import torch

    from paper_1410_1387_amd import fdwave as F

    shots = [_shot((256, 256, 256), 24, 21), _shot((40, 48, 64), 30, 22)]
    dt = 0.45 * min(oracle_mod.dt_max(3, 4, 10.0, float(s[0].max())) for s in shots)
    stream = torch.cuda.Stream()
    ref = []
    for (v, src, rec, T) in shots:
        ctx, keep, tr = _make_ctx(v, src, rec, T, dt, stream)
        F.fd_step(ctx, T)
        u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)
        F.fd_sync(ctx)
        ref.append((u.cpu().numpy(), tr.cpu().numpy(), F.fd_kernel_config(ctx)))
        F.fd_destroy(ctx)
    say(f"tile builds: {ref[0][2]} | {ref[1][2]}")
    assert ref[0][2].split(", zchunk")[0] != ref[1][2].split(", zchunk")[0]
    ctxs = [_make_ctx(v, src, rec, T, dt, stream) for (v, src, rec, T) in shots]
    bws = torch.empty(F.fd_batch_workspace_bytes(2), dtype=torch.uint8, device="cuda")
    b = F.fd_batch_create(2, bws, F.stream_ptr(stream))
    F.fd_batch_set(b, [c[0] for c in ctxs], [s[3] for s in shots])
    F.fd_batch_step(b, 16)
    F.fd_batch_step(b, 15)
    for j, ((ctx, keep, tr), (v, *_rest)) in enumerate(zip(ctxs, shots)):
        u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)
        F.fd_sync(ctx)
        assert F.fd_get_step(ctx) == shots[j][3]
        assert np.array_equal(u.cpu().numpy(), ref[j][0]), j
        assert np.array_equal(tr.cpu().numpy(), ref[j][1]), j
    F.fd_batch_destroy(b)
    for ctx, keep, tr in ctxs:
        F.fd_destroy(ctx)


def test_batch_orders_member_streams(oracle_mod):
    # Each member on a stream of its own and the batch on another: single steps still
    # queued on a member's stream finish before the batch steps it, and a state read
    # enqueued on the member's stream after fd_batch_step sees the batched steps; the
    # batch stream itself is never synchronised by the test.
    import torch

    from paper_1410_1387_amd import fdwave as F

    shots = [_shot((40, 48, 64), 60, 11), _shot((64, 64, 64), 50, 12), _shot((24, 90, 33), 44, 13)]
    dt = 0.45 * min(oracle_mod.dt_max(3, 4, 10.0, float(s[0].max())) for s in shots)
    pre = 7                                      # single steps queued before the batch
    ref = []
    s0 = torch.cuda.Stream()
    for (v, src, rec, T) in shots:
        ctx, keep, tr = _make_ctx(v, src, rec, T, dt, s0)
        F.fd_step(ctx, T)
        u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)
        F.fd_sync(ctx)
        ref.append((u.cpu().numpy(), tr.cpu().numpy()))
        F.fd_destroy(ctx)
    streams = [torch.cuda.Stream() for _ in shots]
    bstream = torch.cuda.Stream()
    ctxs = [_make_ctx(v, src, rec, T, dt, st) for (v, src, rec, T), st in zip(shots, streams)]
    for ctx, keep, tr in ctxs:
        F.fd_step(ctx, pre)                     # asynchronous, not waited for
    bws = torch.empty(F.fd_batch_workspace_bytes(4), dtype=torch.uint8, device="cuda")
    b = F.fd_batch_create(4, bws, F.stream_ptr(bstream))
    F.fd_batch_set(b, [c[0] for c in ctxs], [s[3] for s in shots])
    say("batch on its own stream, members on theirs")
    for _ in range(4):
        F.fd_batch_step(b, 16)
    outs = []
    for (ctx, keep, tr), (v, *_rest) in zip(ctxs, shots):
        u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)            # on the member's stream
        F.fd_sync(ctx)
        outs.append((u.cpu().numpy(), tr.cpu().numpy(), F.fd_get_step(ctx)))
    for j, ((u, tr, n), (u_ref, tr_ref)) in enumerate(zip(outs, ref)):
        assert n == shots[j][3]
        assert np.array_equal(u, u_ref), j
        assert np.array_equal(tr, tr_ref), j
    F.fd_batch_destroy(b)
    for ctx, keep, tr in ctxs:
        F.fd_destroy(ctx)


def _requests(n, seed, sides=(24, 32, 40), steps=(40, 90), spread=0.3):
    from paper_1410_1387_amd.serving import ShotRequest

    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        s = int(rng.choice(sides))
        v, src, rec, T = _shot((s, s, s), int(rng.integers(steps[0], steps[1] + 1)), seed * 100 + i)
        out.append(ShotRequest(rid=i, velocity=v, nsteps=T, source=src, receivers=rec, f0=30.0, t0=0.03,
                               arrival=float(rng.uniform(0, spread)), dt=4e-4))
    return out


def test_server_alone_vs_mix_bitwise(oracle_mod):
    from paper_1410_1387_amd.serving import ShotServer, run_sequential, summarize

    reqs = _requests(10, 5, steps=(300, 600), spread=0.02)  # arrivals overlap running shots
    say("sequential baseline")
    seq = {r.rid: r for r in run_sequential(reqs)}
    say("continuous batching")
    srv = ShotServer(r=4, chunk=8, max_shots=8)
    res = {r.rid: r for r in srv.serve_trace(reqs)}
    st = summarize(list(res.values()))
    say(f"served {st['completed']} p50 {st['p50_latency_s']:.3f}s p99 {st['p99_latency_s']:.3f}s; {srv.stats}")
    assert st["completed"] == len(reqs)
    assert srv.stats["max_stepping_shots"] > 1  # shots really shared launches
    for rid, r in res.items():
        assert r.status == "ok" and seq[rid].status == "ok"
        assert np.array_equal(r.traces.cpu().numpy(), seq[rid].traces.cpu().numpy()), rid
    q = reqs[3]
    ref = oracle_mod.forward(q.velocity.astype(np.float64), q.h, q.dt, 4, q.nsteps,
                             [(q.source, oracle_mod.ricker(q.nsteps, q.dt, q.f0, q.t0))], q.receivers)
    assert rel_l2(res[3].traces.cpu().numpy(), ref["traces"]) <= 1e-4


def test_server_budget_backpressure():
    import torch

    from paper_1410_1387_amd import fdwave as F
    from paper_1410_1387_amd.serving import ShotServer, run_sequential, shot_footprint, staging_bytes

    reqs = _requests(6, 6, sides=(32, 40), spread=0.0)
    need = max(shot_footprint(q.velocity.shape, q.nsteps, len(q.receivers), 4, "f32") +
               staging_bytes(q.velocity.shape, "f32") for q in reqs)
    budget = int(need * 1.6)  # room for one shot at a time, sometimes two
    say(f"budget {budget} B")
    srv = ShotServer(r=4, chunk=8, max_shots=8, budget_bytes=budget)
    torch.cuda.synchronize()
    # bytes the program asked the allocator for: the allocator's own bookkeeping rounds a
    # reused cached block up by as much as 1 MiB (it does not split off a small remainder),
    # which is not memory the server requested
    key = "requested_bytes.all.peak"
    assert key in torch.cuda.memory_stats(), "torch does not report requested bytes"
    base = torch.cuda.memory_stats()["requested_bytes.all.current"]
    torch.cuda.reset_peak_memory_stats()
    res = {r.rid: r for r in srv.serve_trace(reqs, realtime=False)}
    torch.cuda.synchronize()
    peak = torch.cuda.memory_stats()[key] - base
    seq = {r.rid: r for r in run_sequential(reqs, realtime=False)}
    assert all(r.status == "ok" for r in res.values())
    assert srv.stats["max_resident_bytes"] <= budget
    assert srv.stats["max_admission_bytes"] <= budget
    # the device memory the server really requested, staged models included, stays within the
    # budget plus its own batch table and the traces it has already handed back (they belong
    # to the caller once a shot completes)
    handed_back = sum(r.traces.numel() * r.traces.element_size() for r in res.values())
    slack = F.fd_batch_workspace_bytes(8) + 64 * 1024
    say(f"peak requested device memory {peak} B against budget {budget} B (+ {handed_back} B of returned traces)")
    assert peak <= budget + handed_back + slack
    for rid in res:
        assert np.array_equal(res[rid].traces.cpu().numpy(), seq[rid].traces.cpu().numpy())


def test_server_isolates_bad_requests():
    from paper_1410_1387_amd.serving import ShotRequest, ShotServer, run_sequential

    reqs = _requests(4, 7, spread=0.0)
    v = reqs[0].velocity
    reqs.append(ShotRequest(rid=90, velocity=v, nsteps=20, source=(1, 1, 1), receivers=reqs[0].receivers,
                            dt=1.0))                                   # unstable time step
    reqs.append(ShotRequest(rid=91, velocity=v, nsteps=20, source=(999, 1, 1), receivers=reqs[0].receivers,
                            dt=4e-4))                                  # source outside the grid
    big = np.full((400, 400, 400), 2000.0, dtype=np.float32)
    reqs.append(ShotRequest(rid=92, velocity=big, nsteps=10, source=(1, 1, 1), receivers=reqs[0].receivers))
    def broken_model():
        raise ValueError("model file unreadable")

    reqs.append(ShotRequest(rid=93, velocity=broken_model, shape=v.shape, nsteps=10, source=(1, 1, 1),
                            receivers=reqs[0].receivers))              # the model cannot be built
    srv = ShotServer(r=4, chunk=8, max_shots=8, budget_bytes=1 << 30)  # 400^3 does not fit 1 GiB
    res = {r.rid: r for r in srv.serve_trace(reqs, realtime=False)}
    assert res[90].status == "failed" and "UNSTABLE" in res[90].error
    assert res[91].status == "failed" and "RANGE" in res[91].error
    assert res[92].status == "failed" and "budget" in res[92].error
    assert res[93].status == "failed" and "ValueError" in res[93].error
    assert all(res[i].status == "ok" for i in range(4))
    seq = {r.rid: r for r in run_sequential(reqs, realtime=False)}
    assert seq[93].status == "failed" and all(seq[i].status == "ok" for i in range(4))


def test_server_zero_and_negative_steps():
    # a shot of zero steps is served at once with an empty trace set (nothing to inject or
    # record) and leaves the others bitwise unchanged; a negative step count fails alone
    import dataclasses

    from paper_1410_1387_amd.serving import ShotServer, run_sequential

    reqs = _requests(3, 11, spread=0.0)
    zero = dataclasses.replace(reqs[0], rid=80, nsteps=0)
    neg = dataclasses.replace(reqs[1], rid=81, nsteps=-5)
    ref = {r.rid: r for r in run_sequential(reqs, realtime=False)}
    for name, res in (("batched", ShotServer(r=4, chunk=8, max_shots=8).serve_trace(reqs + [zero, neg], realtime=False)),
                      ("one at a time", run_sequential(reqs + [zero, neg], realtime=False))):
        res = {r.rid: r for r in res}
        say(f"{name}: zero-step {res[80].status}, negative {res[81].status} ({res[81].error})")
        assert res[80].status == "ok" and tuple(res[80].traces.shape) == (0, len(zero.receivers))
        assert res[81].status == "failed" and "nsteps" in res[81].error
        for i in range(3):
            assert res[i].status == "ok" and torch_equal(res[i].traces, ref[i].traces)


def torch_equal(a, b):
    import torch

    return bool(torch.equal(a, b))


def test_server_real_sizes_alone_vs_mix_bitwise(oracle_mod):
    # the serving workload's own requests (sides 128-400, layered models built on the GPU,
    # surface receivers), with their step counts cut to 37-96 so the test stays short:
    # batched with the default stepping window and graph chunks, every shot's traces are
    # bitwise those of the same shot served alone
    import dataclasses

    import torch

    from paper_1410_1387_amd import fdwave as F
    from paper_1410_1387_amd.serving import ShotRequest, ShotServer, run_sequential

    sides = {}
    reqs = []
    for q in workloads.serving_trace(24):
        if q.n in sides and len(reqs) >= 5:
            continue
        sides[q.n] = True
        prof = q.profile().astype("float32")
        dt = 0.5 * F.fd_dt_max(3, 4, 10.0, float(prof.max()))

        def make(prof=prof, n=q.n):
            return torch.tensor(prof, device="cuda").view(n, 1, 1).expand(n, n, n).contiguous()

        reqs.append(ShotRequest(rid=q.rid, velocity=make, shape=q.shape, nsteps=(37, 64, 96)[len(reqs) % 3],
                                source=q.source, receivers=q.receivers(), dt=dt))
        if len(reqs) == 7:
            break
    say("real sizes: " + ", ".join(f"{r.shape[0]}^3 x {r.nsteps}" for r in reqs))
    assert {400, 128} <= {r.shape[0] for r in reqs}
    seq = {r.rid: r for r in run_sequential(reqs, realtime=False)}
    srv = ShotServer(r=4, budget_bytes=64 << 30, max_shots=8)
    res = {r.rid: r for r in srv.serve_trace([dataclasses.replace(r, arrival=0.0) for r in reqs], realtime=False)}
    say(f"stats {srv.stats}")
    assert srv.stats["max_stepping_shots"] > 1
    for rid in seq:
        assert res[rid].status == "ok" and seq[rid].status == "ok"
        assert np.array_equal(res[rid].traces.cpu().numpy(), seq[rid].traces.cpu().numpy()), rid


def test_server_cancellation():
    # requests cancelled while queued are dropped; the others are served; a request that
    # has been admitted can no longer be cancelled and completes
    from paper_1410_1387_amd.serving import ShotServer

    reqs = _requests(6, 11, sides=(32,), steps=(200, 200), spread=0.0)
    need = 1 << 30
    srv = ShotServer(r=4, chunk=8, max_shots=1, budget_bytes=need)   # one shot at a time
    futs = [srv.submit(q) for q in reqs]
    cancelled = [futs[i].cancel() for i in (3, 5)]
    srv.start()
    res = {}
    for q, f in zip(reqs, futs):
        if not f.cancelled():
            res[q.rid] = f.result(timeout=120)
    late = futs[0].cancel()                  # admitted (and finished) already
    srv.stop()
    say(f"cancelled {cancelled}, late cancel {late}, served {sorted(res)}")
    assert all(cancelled) and not late
    assert sorted(res) == [0, 1, 2, 4] and all(r.status == "ok" for r in res.values())


@pytest.mark.parametrize("seed", range(4))
def test_batch_random_mixes_bitwise(seed):
    # random mixes of 2-6 shots (ragged 3-D sizes, different step counts and targets,
    # random chunk lengths odd and even, membership changes mid-run): every shot's state
    # and traces are bitwise those of the same shot stepped alone
    import torch

    from paper_1410_1387_amd import fdwave as F

    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 7))
    shots = []
    for k in range(n):
        shape = tuple(int(x) for x in rng.integers(3, [40, 50, 90]))
        v = rng.uniform(1500.0, 4000.0, shape).astype(np.float32)
        src = tuple(int(rng.integers(0, s)) for s in shape[::-1])
        rec = np.array([tuple(int(rng.integers(0, s)) for s in shape[::-1]) for _ in range(int(rng.integers(1, 20)))])
        shots.append((v, src, rec, int(rng.integers(5, 60))))
    dt = 0.45 * F.fd_dt_max(3, 4, 10.0, 4000.0)
    stream = torch.cuda.Stream()
    alone = []
    for (v, src, rec, T) in shots:
        ctx, keep, tr = _make_ctx(v, src, rec, T, dt, stream)
        F.fd_step(ctx, T)
        u = torch.empty(v.shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)
        F.fd_sync(ctx)
        alone.append((u.cpu().numpy(), tr.cpu().numpy()))
        F.fd_destroy(ctx)
    ctxs = [_make_ctx(v, src, rec, T, dt, stream) for (v, src, rec, T) in shots]
    bws = torch.empty(F.fd_batch_workspace_bytes(8), dtype=torch.uint8, device="cuda")
    b = F.fd_batch_create(8, bws, F.stream_ptr(stream))
    members = list(range(n))
    first = members[: max(1, n // 2)]          # start with half, add the rest later
    F.fd_batch_set(b, [ctxs[j][0] for j in first], [shots[j][3] for j in first])
    steps = 0
    while steps < 7:
        c = int(rng.integers(1, 12))
        F.fd_batch_step(b, c)
        steps += c
    F.fd_batch_set(b, [ctxs[j][0] for j in members], [shots[j][3] for j in members])
    while any(F.fd_get_step(ctxs[j][0]) < shots[j][3] for j in members) and steps < 1000:
        c = int(rng.integers(1, 12))
        F.fd_batch_step(b, c)
        steps += c
    stream.synchronize()
    say(f"mix of {n} shots, {steps} batched steps")
    for j, (ctx, keep, tr) in enumerate(ctxs):
        u = torch.empty(shots[j][0].shape, dtype=torch.float32, device="cuda")
        F.fd_get_state(ctx, u, None)
        F.fd_sync(ctx)
        assert F.fd_get_step(ctx) == shots[j][3]
        assert np.array_equal(u.cpu().numpy(), alone[j][0]), j
        assert np.array_equal(tr.cpu().numpy(), alone[j][1]), j
        F.fd_destroy(ctx)
    F.fd_batch_destroy(b)
