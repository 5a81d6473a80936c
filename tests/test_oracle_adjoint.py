"""Pins of the oracle's discrete adjoint gradient (CPU only): central finite
differences of the misfit, the Taylor remainder, and a check of the gradient's
scaling in v."""

import numpy as np
import pytest


def _setup(shape, r, T, seed):
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    v = 2000 + 1500 * rng.random(shape)
    import oracle

    h = 10.0
    dt = 0.5 * oracle.dt_max(ndim, r, h, v.max())
    wav = oracle.ricker(T, dt, 40.0, t0=0.03)
    centre = tuple(s // 2 for s in shape[::-1])
    src = [(centre, wav)]
    # a line of receivers along x at the second index of every other axis
    rec = [tuple([x] + [1] * (ndim - 1)) for x in range(1, shape[-1] - 1, 2)]
    v_true = v * (1 + 0.05 * rng.standard_normal(shape))
    obs = oracle.forward(v_true, h, dt, r, T, src, rec)["traces"]
    return rng, v, h, dt, src, rec, obs


@pytest.mark.parametrize("shape,r,T", [((18, 20), 2, 90), ((9, 10, 11), 4, 50)])
def test_gradient_central_fd(oracle_mod, shape, r, T):
    rng, v, h, dt, src, rec, obs = _setup(shape, r, T, 11)
    g = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs)
    gv = g["grad_v"]
    flat = rng.choice(v.size, size=6, replace=False)
    scale = np.abs(gv).max()
    for f in flat:
        idx = np.unravel_index(f, v.shape)
        eps = 1e-3 * v[idx]
        vp, vm = v.copy(), v.copy()
        vp[idx] += eps
        vm[idx] -= eps
        Jp = oracle_mod.misfit(oracle_mod.forward(vp, h, dt, r, T, src, rec)["traces"], obs)
        Jm = oracle_mod.misfit(oracle_mod.forward(vm, h, dt, r, T, src, rec)["traces"], obs)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - gv[idx]) <= 1e-6 * scale, (idx, fd, gv[idx], scale)


def test_gradient_taylor_remainder(oracle_mod):
    # J(v + e d) - J(v) - e <g, d> = O(e^2): halving e quarters the remainder
    shape, r, T = (16, 14), 3, 80
    rng, v, h, dt, src, rec, obs = _setup(shape, r, T, 12)
    g = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs)
    d = rng.standard_normal(shape) * 20.0
    J0 = g["J"]
    gd = float(np.sum(g["grad_v"] * d))
    rem = []
    for e in (0.4, 0.2, 0.1):
        Je = oracle_mod.misfit(oracle_mod.forward(v + e * d, h, dt, r, T, src, rec)["traces"], obs)
        rem.append(abs(Je - J0 - e * gd))
    ratios = np.array(rem[:-1]) / np.array(rem[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.3), ratios
    # the first-order term dominates the remainder at the smallest step
    assert rem[-1] < 0.05 * abs(0.1 * gd)


def test_gradient_zero_at_true_model(oracle_mod):
    shape, r, T = (12, 13), 2, 60
    rng, v, h, dt, src, rec, _ = _setup(shape, r, T, 13)
    obs = oracle_mod.forward(v, h, dt, r, T, src, rec)["traces"]
    g = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs)
    assert g["J"] == 0.0 and np.all(g["grad_v"] == 0.0)


def test_gradient_is_linear_in_residual(oracle_mod):
    # dJ/dv = J'(v)^T resid: doubling the residual doubles the gradient exactly
    shape, r, T = (12, 11), 2, 50
    rng, v, h, dt, src, rec, obs = _setup(shape, r, T, 14)
    fw = oracle_mod.forward(v, h, dt, r, T, src, rec)["traces"]
    g1 = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs)["grad_v"]
    obs2 = fw - 2.0 * (fw - obs)
    g2 = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs2)["grad_v"]
    assert np.abs(g2 - 2.0 * g1).max() <= 1e-13 * np.abs(g1).max()


@pytest.mark.parametrize("shape,r,T", [((14, 17), 2, 61), ((7, 9, 11), 4, 37)])
def test_checkpointed_gradient_equals_store_all(oracle_mod, shape, r, T):
    # recomputing each segment from its checkpoint repeats the forward arithmetic, and the
    # multiplier recursion carried across segments is the same recursion: the gradient,
    # the misfit and the traces are bit for bit those of the path that stores every state,
    # for intervals that divide T, that do not, of one step, and longer than the run
    rng, v, h, dt, src, rec, obs = _setup(shape, r, T, 15)
    ref = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs)
    seen = []
    for K in (1, 5, T // 3, T - 1, T, T + 7):
        g = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs, checkpoint=K, progress=seen.append)
        assert np.array_equal(g["grad_v"], ref["grad_v"]), K
        assert np.array_equal(g["traces"], ref["traces"]) and g["J"] == ref["J"], K
    assert seen and np.abs(ref["grad_v"]).max() > 0


def test_checkpointed_gradient_central_fd(oracle_mod):
    # the checkpointed path against central differences of the misfit directly (not only
    # through the store-all path)
    shape, r, T = (10, 12, 13), 3, 45
    rng, v, h, dt, src, rec, obs = _setup(shape, r, T, 16)
    gv = oracle_mod.gradient(v, h, dt, r, T, src, rec, obs, checkpoint=8)["grad_v"]
    scale = np.abs(gv).max()
    for f in rng.choice(v.size, size=4, replace=False):
        idx = np.unravel_index(f, v.shape)
        eps = 1e-3 * v[idx]
        vp, vm = v.copy(), v.copy()
        vp[idx] += eps
        vm[idx] -= eps
        Jp = oracle_mod.misfit(oracle_mod.forward(vp, h, dt, r, T, src, rec)["traces"], obs)
        Jm = oracle_mod.misfit(oracle_mod.forward(vm, h, dt, r, T, src, rec)["traces"], obs)
        assert abs((Jp - Jm) / (2 * eps) - gv[idx]) <= 1e-6 * scale
