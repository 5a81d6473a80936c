"""Pins of the oracle's time stepping (CPU only).

Each test checks the FP64 oracle against something the mathematics fixes
independently of its code: an exact discrete solution, a textbook special case,
an invariant of the scheme, a symmetry, or a convergence rate.
"""

import math

import numpy as np
import pytest


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ----------------------------------------------------------------------------- exact solutions


@pytest.mark.parametrize("shape,r", [((24, 32), 4), ((20, 12, 16), 2), ((16, 16, 16), 8)])
def test_standing_wave_exact(oracle_mod, shape, r):
    # phi = prod sin(k_a x_a) on a periodic box is an eigenvector of L with eigenvalue
    # -kappa_h^2 = h^-2 sum_a (w0 + 2 sum_l w_l cos(l k_a h)); with u^0 = phi and
    # u^{-1} = cos(w dt) phi, cos(w dt) = 1 - dt^2 v^2 kappa_h^2 / 2, the leapfrog
    # solution is exactly u^n = cos(w n dt) phi.
    h, v = 10.0, 2000.0
    ndim = len(shape)
    dt = 0.8 * oracle_mod.dt_max(ndim, r, h, v)
    w = [float(x) for x in oracle_mod.weights(r)]
    modes = [1, 2, 3][:ndim]
    axes = []
    kap2 = 0.0
    for a, m in enumerate(modes):
        n_a = shape[::-1][a]
        k = 2 * math.pi * m / (n_a * h)
        axes.append(np.sin(k * np.arange(n_a) * h))
        kap2 -= (w[0] + 2 * sum(w[l] * math.cos(l * k * h) for l in range(1, r + 1))) / h ** 2
    phi = axes[0]
    for a in range(1, ndim):
        phi = np.multiply.outer(axes[a], phi)
    cwdt = 1 - dt * dt * v * v * kap2 / 2
    omega_dt = math.acos(cwdt)
    T = 300
    out = oracle_mod.forward(np.full(shape, v), h, dt, r, T, periodic=True, u0=phi, um1=cwdt * phi)
    expect = math.cos(omega_dt * T) * phi
    assert np.abs(out["u"] - expect).max() < 1e-11
    assert np.abs(out["u_prev"] - math.cos(omega_dt * (T - 1)) * phi).max() < 1e-11


def test_dalembert_courant_one_bitwise(oracle_mod):
    # r = 1, v dt = h: the scheme reduces to u^{n+1}_i = u^n_{i+1} + u^n_{i-1} - u^{n-1}_i,
    # which carries any right-moving pulse f(x - t) exactly (d'Alembert).
    n = 64
    f = np.zeros(n)
    f[5:12] = [1, 3, 6, 7, 6, 3, 1]
    out = oracle_mod.forward(np.ones(n), 1.0, 1.0, 1, 150, periodic=True, u0=f, um1=np.roll(f, -1))
    assert np.array_equal(out["u"], np.roll(f, 150))
    assert np.array_equal(out["u_prev"], np.roll(f, 149))


@pytest.mark.parametrize("r", [1, 2])
def test_full_solution_h_slope(oracle_mod, r):
    # With dt fixed, compare with the time-discrete, space-exact solution
    # cos(w~ n dt) sin(kx), cos(w~ dt) = 1 - (v dt k)^2 / 2.  The time error cancels and
    # what remains is the spatial error, which must fall like h^{2r}.
    L, v, T = 1.0, 1.0, 400
    k = 2 * math.pi / L
    dt = 0.002
    errs, hs = [], []
    for n in (16, 32, 64):
        h = L / n
        x = np.arange(n) * h
        phi = np.sin(k * x)
        w = [float(q) for q in oracle_mod.weights(r)]
        kap2 = -(w[0] + 2 * sum(w[l] * math.cos(l * k * h) for l in range(1, r + 1))) / h ** 2
        cwdt = 1 - dt * dt * v * v * kap2 / 2
        out = oracle_mod.forward(np.full(n, v), h, dt, r, T, periodic=True, u0=phi, um1=cwdt * phi)
        wt = math.acos(1 - (v * dt * k) ** 2 / 2)
        errs.append(np.abs(out["u"] - math.cos(wt * T) * phi).max())
        hs.append(h)
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(np.abs(slopes - 2 * r) < 0.2), slopes


# ----------------------------------------------------------------------------- invariants


def _smooth_field(rng, shape, scale=3.0):
    f = rng.standard_normal(shape)
    for ax in range(len(shape)):
        for _ in range(3):
            f = 0.25 * np.roll(f, 1, ax) + 0.5 * f + 0.25 * np.roll(f, -1, ax)
    return f * scale


@pytest.mark.parametrize("periodic", [False, True])
def test_energy_conserved(oracle_mod, periodic):
    # E^{n+1/2} = ||u^{n+1} - u^n||^2_{1/v^2} / dt^2 - <u^{n+1}, L u^n> is constant without
    # a source, for any v and either boundary, because L is symmetric.
    rng = np.random.default_rng(1)
    shape, r, h = (14, 12, 10), 4, 10.0
    v = 1500 + 3000 * rng.random(shape)
    dt = 0.9 * oracle_mod.dt_max(3, r, h, v.max())
    u0 = _smooth_field(rng, shape)
    out = oracle_mod.forward(v, h, dt, r, 120, periodic=periodic, u0=u0, um1=0.9 * u0, store_states=True)
    st = out["states"]
    E = []
    for nn in range(0, 120):
        du = st[nn + 1] - st[nn]
        E.append(np.sum(du * du / (v * v)) / dt ** 2
                 - np.sum(st[nn + 1] * oracle_mod.laplacian(st[nn], r, h, periodic)))
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-12 * abs(E[0])


def test_reciprocity_variable_velocity(oracle_mod):
    # G(r <- s) m_s = G(s <- r) m_r, because (M L)^T = M^{-1} (M L) M.
    rng = np.random.default_rng(2)
    shape, r, h, T = (11, 13, 12), 4, 10.0, 90
    v = 1500 + 3000 * rng.random(shape)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, v.max())
    wav = oracle_mod.ricker(T, dt, 30.0)
    a, b = (2, 3, 4), (9, 7, 8)  # (x, y, z)
    g_ab = oracle_mod.forward(v, h, dt, r, T, [(a, wav)], [b])["traces"][:, 0]
    g_ba = oracle_mod.forward(v, h, dt, r, T, [(b, wav)], [a])["traces"][:, 0]
    m = lambda p: v[p[2], p[1], p[0]] ** 2
    lhs, rhs = g_ab * m(a), g_ba * m(b)
    assert _rel(lhs, rhs) < 1e-13
    assert _rel(g_ab, g_ba) > 1e-3  # the unscaled swap does not hold


def test_centred_source_symmetry(oracle_mod):
    # constant v, odd cube, centred source: mirror images are bitwise equal,
    # axis permutations equal to roundoff
    n, r, h, T = 15, 4, 10.0, 70
    v = np.full((n, n, n), 2500.0)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, 2500.0)
    wav = oracle_mod.ricker(T, dt, 40.0, t0=0.02)
    u = oracle_mod.forward(v, h, dt, r, T, [((7, 7, 7), wav)])["u"]
    assert np.abs(u).max() > 0
    for ax in range(3):
        assert np.array_equal(u, np.flip(u, ax))
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
        assert np.abs(u - np.transpose(u, perm)).max() <= 1e-14 * np.abs(u).max()


def test_superposition_and_scaling(oracle_mod):
    rng = np.random.default_rng(3)
    shape, r, h, T = (12, 10, 14), 3, 10.0, 60
    v = 1500 + 3000 * rng.random(shape)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, v.max())
    wa, wb = oracle_mod.ricker(T, dt, 25.0), rng.standard_normal(T)
    pa, pb = (3, 4, 5), (8, 2, 9)
    ua = oracle_mod.forward(v, h, dt, r, T, [(pa, wa)])["u"]
    ub = oracle_mod.forward(v, h, dt, r, T, [(pb, wb)])["u"]
    uab = oracle_mod.forward(v, h, dt, r, T, [(pa, wa), (pb, wb)])["u"]
    assert np.abs(uab - (ua + ub)).max() <= 1e-14 * np.abs(uab).max()
    u8 = oracle_mod.forward(v, h, dt, r, T, [(pa, 8.0 * wa)])["u"]
    assert np.array_equal(u8, 8.0 * ua)  # power-of-two scaling is exact


def test_periodic_translation_bitwise(oracle_mod):
    shape, r, h, T = (10, 12, 14), 4, 10.0, 50
    v = np.full(shape, 3000.0)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, 3000.0)
    wav = oracle_mod.ricker(T, dt, 30.0)
    u1 = oracle_mod.forward(v, h, dt, r, T, [((2, 3, 4), wav)], periodic=True)["u"]
    u2 = oracle_mod.forward(v, h, dt, r, T, [((7, 5, 1), wav)], periodic=True)["u"]
    assert np.array_equal(np.roll(u1, (-3, 2, 5), axis=(0, 1, 2)), u2)


def test_time_reversibility(oracle_mod):
    # feeding (cur = u^{T-1}, prev = u^T) back into the same scheme retraces the
    # trajectory to (u^{-1}, u^0)
    rng = np.random.default_rng(4)
    shape, r, h, T = (16, 14, 12), 4, 10.0, 150
    v = 1500 + 3000 * rng.random(shape)
    dt = 0.6 * oracle_mod.dt_max(3, r, h, v.max())
    u0, um1 = _smooth_field(rng, shape), _smooth_field(rng, shape)
    fw = oracle_mod.forward(v, h, dt, r, T, u0=u0, um1=um1)
    bw = oracle_mod.forward(v, h, dt, r, T, u0=fw["u_prev"], um1=fw["u"])
    assert np.abs(bw["u"] - um1).max() <= 1e-9 * np.abs(um1).max()
    assert np.abs(bw["u_prev"] - u0).max() <= 1e-9 * np.abs(u0).max()


# ----------------------------------------------------------------------------- stability, source


def test_stability_limit(oracle_mod):
    # constant v on an even periodic box contains the theta = pi mode: just below
    # dt_max the solution stays bounded, just above it grows geometrically
    rng = np.random.default_rng(6)
    shape, r, h, v = (16, 16), 4, 10.0, 3000.0
    u0 = rng.standard_normal(shape)
    dtm = oracle_mod.dt_max(2, r, h, v)
    lo = oracle_mod.forward(np.full(shape, v), h, 0.999 * dtm, r, 2000, periodic=True, u0=u0, um1=u0)
    hi = oracle_mod.forward(np.full(shape, v), h, 1.01 * dtm, r, 200, periodic=True, u0=u0, um1=u0)
    assert np.abs(lo["u"]).max() < 50 * np.abs(u0).max()
    assert np.abs(hi["u"]).max() > 1e6 * np.abs(u0).max()


def test_ricker_closed_form_points(oracle_mod):
    f = 15.0
    assert oracle_mod.ricker(1, 0.001, f, t0=0.0)[0] == 1.0  # peak at tau = 0
    dz = 1 / (math.pi * f * math.sqrt(2))  # zero crossing
    assert abs(oracle_mod.ricker(2, dz, f, t0=0.0)[1]) < 1e-15
    dm = math.sqrt(1.5) / (math.pi * f)  # side lobes, value -2 e^{-3/2}
    assert abs(oracle_mod.ricker(2, dm, f, t0=0.0)[1] + 2 * math.exp(-1.5)) < 1e-15
    s = oracle_mod.ricker(401, 0.0005, f, t0=0.1)
    assert np.abs(s[:200][::-1] - s[201:]).max() < 1e-12  # symmetric about t0
    assert abs(oracle_mod.ricker(1, 0.001, f)[0]) < 2e-8  # default shift t0 = 1.5 / f


def test_source_scaling_and_time_level(oracle_mod):
    # reading of the source term: sample n enters u^{n+1} as dt^2 s[n] / h^ndim at one
    # point (discrete delta, no v^2 factor); traces[n] samples u^{n+1}
    shape, r, h = (9, 8, 7), 2, 4.0
    v = np.full(shape, 1000.0)
    dt = 1e-3
    wav = np.zeros(3)
    wav[0] = 1.0
    p = (3, 4, 5)
    out = oracle_mod.forward(v, h, dt, r, 1, [(p, wav)], [p, (0, 0, 0)])
    u1 = out["u"]
    assert u1[5, 4, 3] == dt * dt / h ** 3
    assert np.count_nonzero(u1) == 1
    assert out["traces"][0, 0] == dt * dt / h ** 3 and out["traces"][0, 1] == 0.0


def test_chunked_forward_bitwise(oracle_mod):
    # a run split into chunks, each restarted from the previous chunk's (u, u_prev) with
    # the wavelet shifted, is the one-call run bit for bit (how the full-size parity tests
    # run the oracle)
    from gpu_util import oracle_forward_chunked

    shape, r, h, T = (9, 11, 13), 3, 10.0, 37
    v = 1800.0 + 900.0 * np.random.default_rng(5).random(shape)
    dt = 0.5 * oracle_mod.dt_max(3, r, h, v.max())
    src = [((6, 5, 4), oracle_mod.ricker(T, dt, 40.0, 0.03)), ((0, 10, 8), np.random.default_rng(6).random(T))]
    rec = np.array([(1, 2, 3), (12, 10, 8), (6, 5, 4)])
    one = oracle_mod.forward(v, h, dt, r, T, src, rec)
    for chunk in (1, 5, 36, 40):
        got = oracle_forward_chunked(oracle_mod, v, h, dt, r, T, src, rec, lambda m: None, chunk=chunk)
        for key in ("u", "u_prev", "traces"):
            assert np.array_equal(got[key], one[key]), (chunk, key)
