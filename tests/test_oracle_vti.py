"""Pins of the oracle's two-field VTI propagator (CPU only).

Each test checks the FP64 oracle against something fixed independently of its
code: the isotropic oracle (itself pinned by closed forms) in the isotropic
limit, an exact discrete standing wave of the coupled p/q system, the sharp
stability limit, the Lagrange-basis construction of the z weights, exactness of
the z stencil on polynomials over a stretched grid, and reflection symmetry.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import workloads


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _stretched_z(nz, rz, dz, a=0.35):
    """Strictly increasing plane coordinates -rz .. nz+rz-1 with spacing growing with
    depth, rounded to multiples of 1/64 m (so that the exact weights stay cheap)."""
    k = np.arange(-rz, nz + rz, dtype=np.float64)
    z = dz * k * (1.0 + a * (k / nz) ** 2)
    z = np.round(z * 64.0) / 64.0
    assert np.all(np.diff(z) > 0)
    return z


# ----------------------------------------------------------------------------- z weights


@pytest.mark.parametrize("rz", [1, 2, 4, 8])
def test_z_weights_uniform_are_the_central_weights(oracle_mod, rz):
    # on a uniform grid the unique (2rz+1)-point stencil exact to degree 2rz is the
    # symmetric central one (pinned in test_oracle_weights), scaled by 1/dz^2
    dz = Fraction(5, 2)
    zc = [float(dz * k) for k in range(-rz, 6 + rz)]
    tab = oracle_mod.z_weights_exact(zc, rz)
    w = oracle_mod.weights(rz)
    for row in tab:
        assert [row[l + rz] for l in range(-rz, rz + 1)] == [w[abs(l)] / dz ** 2 for l in range(-rz, rz + 1)]


def _lagrange_second_derivative(nodes, c):
    """Weights l_j''(x_c) of the Lagrange basis of `nodes` at node index c: with
    l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m), the second derivative of the product
    is the sum over ordered pairs a != b (both != j) of prod_{m != j, a, b} (x - x_m)."""
    n = len(nodes)
    x = nodes[c]
    out = []
    for j in range(n):
        others = [m for m in range(n) if m != j]
        num = Fraction(0)
        for a in others:
            for b in others:
                if a == b:
                    continue
                t = Fraction(1)
                for m in others:
                    if m != a and m != b:
                        t *= x - nodes[m]
                num += t
        den = Fraction(1)
        for m in others:
            den *= nodes[j] - nodes[m]
        out.append(num / den)
    return out


@pytest.mark.parametrize("rz", [2, 3])
def test_z_weights_match_lagrange_basis(oracle_mod, rz):
    zc = _stretched_z(9, rz, 7.5)
    tab = oracle_mod.z_weights_exact(zc, rz)
    zf = [Fraction(float(z)) for z in zc]
    for k in (0, 1, 4, 8):
        nodes = zf[k: k + 2 * rz + 1]
        assert list(tab[k]) == _lagrange_second_derivative(nodes, rz), k


# ----------------------------------------------------------------------------- isotropic limit


@pytest.mark.parametrize("r", [2, 4])
def test_isotropic_limit_equals_acoustic_oracle(oracle_mod, r):
    # eps = delta = 0, equal radii, dz = h and the source in both equations: p = q = u,
    # the solution of the isotropic scheme
    shape = (13, 14, 15)
    h = 10.0
    vz = workloads.layered_velocity(shape, seed=3)
    dt = 0.6 * oracle_mod.dt_max(3, r, h, vz.max())
    T = 60
    wav = oracle_mod.ricker(T, dt, 30.0, 0.03)
    src = (7, 6, 5)
    rec = np.array([[1, 2, 3], [7, 7, 7], [14, 13, 12]])
    ref = oracle_mod.forward(vz, h, dt, r, T, [(src, wav)], rec)
    out = oracle_mod.vti_forward(vz, 0.0, 0.0, h, dt, r, r, T, sources=[(src, wav, 1.0, 1.0)], receivers=rec)
    assert np.array_equal(out["p"], out["q"]) and np.array_equal(out["p_prev"], out["q_prev"])
    assert _rel(out["p"], ref["u"]) <= 1e-13
    assert _rel(out["p_prev"], ref["u_prev"]) <= 1e-13
    assert _rel(out["traces_p"], ref["traces"]) <= 1e-13


# ----------------------------------------------------------------------------- exact discrete solution


def _symbol(w, theta):
    """-(w0 + 2 sum_l w_l cos(l theta)): the 1-D stencil acting on a mode of angle theta."""
    return -(w[0] + 2.0 * sum(w[l] * math.cos(l * theta) for l in range(1, len(w))))


@pytest.mark.parametrize("branch", [0, 1])
def test_standing_wave_exact(oracle_mod, branch):
    # On a periodic box phi = f(x) g(y) e(z), each factor a sine/cosine of a grid
    # frequency, is an eigenfunction of -(Dxx + Dyy) and -Dzz with eigenvalues a_xy, a_z.
    # (p, q) = (e_p, e_q) phi, with (e_p, e_q) an eigenvector of
    # M = [[nux2 a_xy, nuz2 a_z], [nun2 a_xy, nuz2 a_z]] for eigenvalue lam, evolves as
    # cos(omega n dt) (e_p, e_q) phi, cos(omega dt) = 1 - dt^2 lam / 2, exactly.
    nz, ny, nx = 16, 12, 20
    rxy, rz = 4, 2
    h, dz = 10.0, 8.0
    vz, eps, delta = 2000.0, 0.25, 0.1
    mx, my, mz = 2, 1, 3
    tx, ty, tz = 2 * math.pi * mx / nx, 2 * math.pi * my / ny, 2 * math.pi * mz / nz
    i, j, k = np.arange(nx), np.arange(ny), np.arange(nz)
    phi = (np.sin(tz * k + 0.7)[:, None, None] * np.cos(ty * j)[None, :, None] *
           (np.sin(tx * i + 0.3) + 0.5 * np.cos(tx * i))[None, None, :])
    wxy = oracle_mod.weights_f64(rxy)
    wzs = oracle_mod.weights_f64(rz)
    a_xy = (_symbol(wxy, tx) + _symbol(wxy, ty)) / h ** 2
    a_z = _symbol(wzs, tz) / dz ** 2
    nuz2 = vz ** 2
    nux2, nun2 = nuz2 * (1 + 2 * eps), nuz2 * (1 + 2 * delta)
    M = np.array([[nux2 * a_xy, nuz2 * a_z], [nun2 * a_xy, nuz2 * a_z]])
    lam, vec = np.linalg.eig(M)
    lam, e = float(lam[branch].real), vec[:, branch].real
    zc = oracle_mod.uniform_z(nz, rz, dz)
    shape = (nz, ny, nx)
    vzf = np.full(shape, vz)
    dt = 0.9 * oracle_mod.vti_dt_max(rxy, rz, h, oracle_mod.z_weights(zc, rz), vzf, eps, delta)
    c1 = 1 - 0.5 * dt * dt * lam
    assert abs(c1) < 1
    om = math.acos(c1)
    T = 70
    st = (e[0] * phi, e[0] * c1 * phi, e[1] * phi, e[1] * c1 * phi)
    out = oracle_mod.vti_forward(vzf, eps, delta, h, dt, rxy, rz, T, zc=zc, periodic_xy=True, periodic_z=True,
                                 state=st)
    assert _rel(out["p"], e[0] * math.cos(om * T) * phi) <= 1e-11
    assert _rel(out["q"], e[1] * math.cos(om * T) * phi) <= 1e-11
    assert _rel(out["q_prev"], e[1] * math.cos(om * (T - 1)) * phi) <= 1e-11


@pytest.mark.parametrize("factor,grows", [(0.995, False), (1.005, True)])
def test_dt_max_is_sharp(oracle_mod, factor, grows):
    # the Nyquist mode (-1)^(i+j+k) is the first to go unstable; just below the limit
    # it oscillates with constant amplitude, just above it grows geometrically
    nz, ny, nx = 8, 8, 10
    rxy, rz = 4, 3
    h, dz = 10.0, 7.0
    shape = (nz, ny, nx)
    vz, eps, delta = np.full(shape, 2500.0), 0.2, 0.05
    zc = oracle_mod.uniform_z(nz, rz, dz)
    dt = factor * oracle_mod.vti_dt_max(rxy, rz, h, oracle_mod.z_weights(zc, rz), vz, eps, delta)
    i, j, k = np.indices(shape)
    phi = (-1.0) ** (i + j + k)
    a = oracle_mod.vti_forward(vz, eps, delta, h, dt, rxy, rz, 400, zc=zc, periodic_xy=True, periodic_z=True,
                               state=(phi, phi, 0.3 * phi, 0.3 * phi))
    amp = max(np.abs(a["p"]).max(), np.abs(a["q"]).max())
    assert (amp > 1e3) == grows, amp


def test_no_stable_step_when_delta_exceeds_eps(oracle_mod):
    zc = oracle_mod.uniform_z(4, 2, 10.0)
    assert oracle_mod.vti_dt_max(4, 2, 10.0, oracle_mod.z_weights(zc, 2), np.full((4, 4, 4), 2000.0), 0.05,
                                 0.1) == 0.0


# ----------------------------------------------------------------------------- stretched z grid


@pytest.mark.parametrize("rz,deg", [(2, 2), (2, 4), (3, 5), (4, 8)])
def test_stretched_z_step_exact_on_polynomials(oracle_mod, rz, deg):
    # fields constant in x and y (periodic xy): one step from p^0 = p^{-1} = q^0 = q^{-1}
    # = f(z) gives p^1 - p^0 = q^1 - q^0 = dt^2 vz^2 f''(z_k) wherever the 2rz+1 planes
    # around z_k are inside the domain, for every polynomial of degree <= 2rz
    nz, ny, nx = 20, 5, 6
    h, dz, v = 10.0, 9.0, 1800.0
    zc = _stretched_z(nz, rz, dz)
    z = zc[rz: rz + nz]
    zm, L = z.mean(), z.max() - z.min()
    f = ((z - zm) / L) ** deg
    f2 = deg * (deg - 1) * ((z - zm) / L) ** max(deg - 2, 0) / L ** 2
    field = np.broadcast_to(f[:, None, None], (nz, ny, nx)).copy()
    shape = (nz, ny, nx)
    vz = np.full(shape, v)
    dt = 1e-3
    out = oracle_mod.vti_forward(vz, 0.15, 0.05, h, dt, 4, rz, 1, zc=zc, periodic_xy=True,
                                 state=(field, field, field, field))
    for fld in ("p", "q"):
        got = (out[fld] - field)[:, 2, 3] / (dt * dt * v * v)
        inner = slice(rz, nz - rz)
        assert np.max(np.abs(got[inner] - f2[inner])) <= 1e-8 * np.max(np.abs(f2)), fld


# ----------------------------------------------------------------------------- symmetry


def test_centred_source_symmetry(oracle_mod):
    # constant model, odd cube-like box, source at the centre, in p only (the form of
    # eq. (p)): p and q are invariant under x and y reflections and the x <-> y swap;
    # the x reflection only swaps the operands of one addition and is bitwise
    shape = (15, 13, 13)
    h = 10.0
    rxy, rz = 4, 3
    vz = np.full(shape, 2200.0)
    zc = oracle_mod.uniform_z(shape[0], rz, 8.0)
    dt = 0.5 * oracle_mod.vti_dt_max(rxy, rz, h, oracle_mod.z_weights(zc, rz), vz, 0.2, 0.05)
    T = 45
    wav = oracle_mod.ricker(T, dt, 40.0, 0.02)
    out = oracle_mod.vti_forward(vz, 0.2, 0.05, h, dt, rxy, rz, T, zc=zc, sources=[((6, 6, 7), wav, 1.0, 0.0)])
    for f in ("p", "q"):
        u = out[f]
        assert np.abs(u).max() > 0
        assert np.array_equal(u, u[:, :, ::-1])
        assert _rel(u[:, ::-1, :], u) <= 1e-14
        assert _rel(np.swapaxes(u, 1, 2), u) <= 1e-14
        assert _rel(u[::-1, :, :], u) <= 1e-14


def test_source_has_unit_integral(oracle_mod):
    # the discrete delta integrates to one under the grid's own quadrature (cell volume
    # h^2 dz_k with dz_k the half-distance of plane k's neighbours): one step from rest
    # leaves dt^2 amp s[0] / (h^2 dz_k) at the source point, whatever the z spacing
    shape = (12, 7, 8)
    rz = 3
    zc = _stretched_z(shape[0], rz, 6.0)
    dzc = 0.5 * (zc[rz + 1: rz + 1 + shape[0]] - zc[rz - 1: rz - 1 + shape[0]])
    h, dt = 10.0, 1e-3
    for k in (0, 5, 11):
        out = oracle_mod.vti_forward(np.full(shape, 2000.0), 0.1, 0.0, h, dt, 2, rz, 1, zc=zc,
                                     sources=[((3, 4, k), [0.75], 1.0, -2.0)])
        vol = h * h * dzc[:, None, None]
        assert math.isclose(float(np.sum(out["p"] * vol)), dt * dt * 0.75, rel_tol=1e-12)
        assert math.isclose(float(np.sum(out["q"] * vol)), -2.0 * dt * dt * 0.75, rel_tol=1e-12)
