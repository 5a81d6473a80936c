"""Host logic of the serving loop's stepping window (no GPU): which resident shots a
batched launch advances."""
import concurrent.futures as cf
import types

from paper_1410_1387_amd.serving import ShotServer, _Live


def live(n, nsteps=100, done=False, queued_done=False):
    fut = cf.Future()
    if done:
        fut.set_result(None)
    req = types.SimpleNamespace(nsteps=nsteps)
    s = _Live(req, 0, [], None, 0, n ** 3 * nsteps, 0.0, 0.0, fut)
    if queued_done:
        s._queued_done = True
    return s


def window(fill, shots):
    return ShotServer._window(types.SimpleNamespace(fill_points=fill), shots)


def test_window_stops_once_filled():
    shots = [live(128), live(128), live(128), live(128)]  # 2.1 M points per step each
    assert window(4_000_000, shots) == shots[:2]
    assert window(4_200_000, shots) == shots[:3]


def test_large_shot_steps_alone():
    # a shot at or above the fill target is a window of one, whatever follows it
    shots = [live(256), live(64), live(64)]
    assert window(16_000_000, shots) == shots[:1]
    # ... and one that is not first ends the window after it
    shots = [live(64), live(256), live(64)]
    assert window(16_000_000, shots) == shots[:2]


def test_window_has_at_least_one_shot():
    shots = [live(400), live(128)]
    assert window(1, shots) == shots[:1]


def test_finished_shots_leave_the_window():
    shots = [live(128, done=True), live(128, queued_done=True), live(128), live(128)]
    assert window(10 ** 12, shots) == shots[2:]
    assert window(1, shots) == shots[2:3]
    assert window(10 ** 12, [live(64, done=True)]) == []


def test_no_fill_target_steps_every_live_shot():
    shots = [live(400), live(320), live(64, done=True), live(128)]
    assert window(None, shots) == [shots[0], shots[1], shots[3]]


def test_default_window_fits_the_last_level_cache():
    # three FP32 fields (u^n, u^(n-1), c) of the default window's points fit in 256 MB
    import inspect
    fill = inspect.signature(ShotServer.__init__).parameters["fill_points"].default
    assert 12 * fill <= 256 * 10 ** 6
    # and a 256^3 shot fills it alone
    assert 256 ** 3 >= fill


def test_window_keeps_to_one_kernel():
    # one launch runs one stencil kernel: shots whose grid got another tile shape wait for
    # a window led by a shot of their own kind
    a, b, c, d = live(64), live(64), live(64), live(64)
    a.kernel, b.kernel, c.kernel, d.kernel = "k1", "k2", "k1", "k2"
    assert window(16_000_000, [a, b, c, d]) == [a, c]
    assert window(None, [a, b, c, d]) == [a, c]
    a.future.set_result(None)
    assert window(16_000_000, [a, b, c, d]) == [b, d]


def test_window_invariants_random():
    # for any resident set: the oldest live shot always steps; the window holds only shots
    # of its kernel, in admission order, none finished; it stops at the first shot after
    # which the fill target is met
    import random

    rng = random.Random(7)
    for _ in range(300):
        shots = []
        for _k in range(rng.randint(0, 12)):
            s = live(rng.choice((64, 96, 128, 192, 256, 320)), done=rng.random() < 0.2,
                     queued_done=rng.random() < 0.1)
            s.kernel = rng.choice(("k1", "k2"))
            shots.append(s)
        fill = rng.choice((None, 1_000_000, 16_000_000, 64_000_000))
        win = window(fill, shots)
        livs = [s for s in shots if not s.future.done() and not getattr(s, "_queued_done", False)]
        if not livs:
            assert win == []
            continue
        assert win[0] is livs[0]
        assert all(s.kernel == livs[0].kernel for s in win)
        same = [s for s in livs if s.kernel == livs[0].kernel]
        assert win == same[: len(win)]
        if fill is not None:
            per_step = [s.npoints // s.req.nsteps for s in win]
            assert sum(per_step[:-1]) < fill           # it did not stop too late
            assert len(win) == len(same) or sum(per_step) >= fill  # nor too early
