"""Pins of the oracle's absorbing sponge (CPU only).

The sponge (Sec. 1, after Cerjan et al.) may change the solution only through the
strip where G < 1: outside that strip's domain of influence the damped and undamped
solutions are bitwise equal, a zero-width sponge changes nothing, and a wave that
has crossed the sponge leaves far less energy behind than the reflecting bare
boundary does."""

import math

import numpy as np
import pytest


def test_profile_shape(oracle_mod):
    g = oracle_mod.cerjan(50, 20, 0.015)
    assert g[0] == pytest.approx(math.exp(-(0.015 * 20) ** 2), rel=1e-15)
    assert np.all(np.diff(g[:20]) > 0) and np.all(g[20:30] == 1.0)
    assert np.array_equal(g, g[::-1])
    lo = oracle_mod.cerjan(50, 20, 0.015, hi=False)
    assert np.all(lo[20:] == 1.0) and np.array_equal(lo[:20], g[:20])
    G = oracle_mod.damping_field((30, 40), 5, 0.05, faces=(True, False, False, True))
    # x+ and y- are undamped (outside the other axis' strip), x- and y+ are
    assert np.all(G[:-5, -1] == 1.0) and np.all(G[0, 5:] == 1.0) and G[-1, 0] < G[-1, 10] < 1.0


def _run(oracle_mod, shape, r, T, damping, src=None):
    h = 10.0
    v = np.full(shape, 2000.0)
    dt = 0.5 * oracle_mod.dt_max(len(shape), r, h, 2000.0)
    wav = oracle_mod.ricker(T, dt, 25.0, 0.05)
    src = src or tuple(s // 2 for s in shape[::-1])
    return oracle_mod.forward(v, h, dt, r, T, [(src, wav)], damping=damping)


def test_zero_width_is_undamped(oracle_mod):
    a = _run(oracle_mod, (31, 37), 4, 60, None)
    b = _run(oracle_mod, (31, 37), 4, 60, (0, 0.015))
    c = _run(oracle_mod, (31, 37), 4, 60, (8, 0.0))
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["u"], c["u"])


@pytest.mark.parametrize("shape,r,width,T", [((61, 67), 4, 6, 5), ((25, 27, 29), 2, 4, 3)])
def test_sponge_acts_only_through_its_strip(oracle_mod, shape, r, width, T):
    # from a random state, the damped update differs from the undamped one only where
    # G < 1; a difference travels at most r points per step, so after T steps every point
    # farther than T r from the strip is bitwise the undamped value, and points closer
    # than that have been reached
    h = 10.0
    v = np.full(shape, 2000.0)
    dt = 0.5 * oracle_mod.dt_max(len(shape), r, h, 2000.0)
    rng = np.random.default_rng(1)
    u0, um1 = rng.standard_normal(shape), rng.standard_normal(shape)
    a = oracle_mod.forward(v, h, dt, r, T, u0=u0, um1=um1)
    b = oracle_mod.forward(v, h, dt, r, T, u0=u0, um1=um1, damping=(width, 0.08))
    d = width + T * r
    core = tuple(slice(d, n - d) for n in shape)
    assert all(sl.start < sl.stop for sl in core)
    assert np.array_equal(a["u"][core], b["u"][core])
    assert np.array_equal(a["u_prev"][core], b["u_prev"][core])
    reach = tuple(slice(width, n - width) for n in shape)      # inside the strip ...
    diff = a["u"][reach] != b["u"][reach]
    assert diff.any()                                            # ... reached by the change


def test_sponge_absorbs(oracle_mod):
    # a pulse from the centre of a 2-D box: after the direct wave has reached the walls
    # and come back, the bare zero boundary has reflected it into the interior while the
    # sponge has absorbed most of it
    shape, r, width = (161, 161), 4, 30
    h, c = 10.0, 2000.0
    dt = 0.5 * oracle_mod.dt_max(2, r, h, c)
    T = int(1.6 * 80 * h / c / dt)
    bare = _run(oracle_mod, shape, r, T, None)["u"]
    damp = _run(oracle_mod, shape, r, T, (width, 0.015))["u"]
    core = (slice(width, -width), slice(width, -width))
    e_bare = float(np.sum(bare[core] ** 2))
    e_damp = float(np.sum(damp[core] ** 2))
    assert e_bare > 0 and e_damp < 0.05 * e_bare, (e_damp, e_bare)
