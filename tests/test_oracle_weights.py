"""Pins of the oracle's stencil weights, symbol and stability limit (CPU only).

The oracle solves the Taylor conditions for the weights; these tests pin the
result against things that do not come from that solve: a published table,
a closed form derived independently, polynomial exactness on a grid (through the
C Laplacian), the dispersion constant and a dense scan of the symbol.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "central_fd_weights.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[int(parts[0])] = tuple(Fraction(p) for p in parts[1:])
    return out


def test_weights_match_published_table(oracle_mod):
    golden = _golden()
    assert sorted(golden) == [1, 2, 3, 4]
    for r, w in golden.items():
        assert oracle_mod.weights(r) == w


@pytest.mark.parametrize("r", range(1, 9))
def test_weights_closed_form(oracle_mod, r):
    # w_l = 2 (-1)^{l+1} (r!)^2 / (l^2 (r-l)! (r+l)!),  w0 = -2 sum_l w_l
    fr = math.factorial(r)
    expect = [Fraction(2 * (-1) ** (l + 1) * fr * fr, l * l * math.factorial(r - l) * math.factorial(r + l))
              for l in range(1, r + 1)]
    w = oracle_mod.weights(r)
    assert list(w[1:]) == expect
    assert w[0] == -2 * sum(expect)


@pytest.mark.parametrize("r", [1, 2, 4, 8])
def test_weight_moments(oracle_mod, r):
    # sum w_l l^2 = 1, sum w_l l^{2k} = 0 (k=2..r), sum w_l l^{2r+2} = (-1)^{r+1} (r!)^2
    w = oracle_mod.weights(r)
    mom = lambda p: sum(w[l] * l ** p for l in range(1, r + 1))
    assert mom(2) == 1
    for k in range(2, r + 1):
        assert mom(2 * k) == 0
    assert mom(2 * r + 2) == (-1) ** (r + 1) * math.factorial(r) ** 2


def test_r8_values(oracle_mod):
    # radius 8 (16th order): spelled out so a wrong solve shows up as a readable diff
    expect = [Fraction(-1077749, 352800), Fraction(16, 9), Fraction(-14, 45), Fraction(112, 1485),
              Fraction(-7, 396), Fraction(112, 32175), Fraction(-2, 3861), Fraction(16, 315315),
              Fraction(-1, 411840)]
    assert list(oracle_mod.weights(8)) == expect


@pytest.mark.parametrize("r", [1, 2, 3, 4, 6, 8])
def test_symbol_max_is_at_pi(oracle_mod, r):
    w = oracle_mod.weights_f64(r)
    th = np.linspace(0, math.pi, 20001)
    sym = -(w[0] + 2 * sum(w[l] * np.cos(l * th) for l in range(1, r + 1)))
    assert np.all(np.diff(sym) >= -1e-14)  # monotone on [0, pi]
    assert abs(sym.max() - oracle_mod.symbol_max(r)) < 1e-12
    # -w0 + 2 sum |w_l|, since the weights alternate in sign
    assert abs(oracle_mod.symbol_max(r) - (-w[0] + 2 * np.abs(w[1:]).sum())) < 1e-12


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_dispersion_constant(oracle_mod, r):
    # 1-D symbol: kappa_h^2 = k^2 (1 - c_r (kh)^{2r} + ...), c_r = 2 (r!)^2 / (2r+2)!
    c_r = 2 * math.factorial(r) ** 2 / math.factorial(2 * r + 2)
    w = [Fraction(x) for x in oracle_mod.weights(r)]
    # evaluate with exact rationals on a truncated Taylor series of cos
    theta = Fraction(1, 64)

    def cos_series(x, terms=40):
        s, term = Fraction(0), Fraction(1)
        for j in range(terms):
            s += term
            term *= -x * x / ((2 * j + 1) * (2 * j + 2))
        return s

    kap2 = -(w[0] + 2 * sum(w[l] * cos_series(l * theta) for l in range(1, r + 1)))
    rel = (theta ** 2 - kap2) / theta ** 2 / theta ** (2 * r)
    assert abs(float(rel) - c_r) / c_r < 1e-2


def test_dt_max_closed_forms(oracle_mod):
    # r = 1: the classic Courant limit dt <= h / (v sqrt(ndim))
    for ndim in (1, 2, 3):
        assert abs(oracle_mod.dt_max(ndim, 1, 10.0, 2000.0) - 10.0 / (2000.0 * math.sqrt(ndim))) < 1e-15
    # r = 4 Courant numbers quoted for the 2-D and 3-D workloads
    assert abs(oracle_mod.dt_max(2, 4, 1.0, 1.0) - 0.55463) < 5e-6
    assert abs(oracle_mod.dt_max(3, 4, 1.0, 1.0) - 0.45286) < 5e-6
    assert abs(oracle_mod.dt_max(3, 8, 1.0, 1.0) - 0.42371) < 5e-6


@pytest.mark.parametrize("r", [1, 2, 3, 4, 8])
def test_polynomial_exactness_1d(oracle_mod, r):
    # L x^p is exact at interior points for p <= 2r+1; for p = 2r+2 the error is the
    # constant 2 (-1)^{r+1} (r!)^2 h^{2r} (leading Taylor remainder).
    h = 0.5
    n = 4 * r + 9
    x = (np.arange(n) - n // 2) * h
    interior = slice(r, n - r)
    for p in range(0, 2 * r + 3):
        u = x ** p
        lap = oracle_mod.laplacian(u, r, h)
        exact = p * (p - 1) * x ** (p - 2) if p >= 2 else np.zeros_like(x)
        err = (lap - exact)[interior]
        scale = max(1.0, np.abs(exact[interior]).max(), np.abs(u).max() / h ** 2)
        if p <= 2 * r + 1:
            assert np.abs(err).max() <= 1e-11 * scale, (r, p)
        else:
            c = 2 * (-1) ** (r + 1) * math.factorial(r) ** 2 * h ** (2 * r)
            assert np.allclose(err, c, rtol=1e-8, atol=1e-10 * scale), (r, p, err[:3], c)


@pytest.mark.parametrize("r", [1, 2, 4])
def test_polynomial_exactness_3d(oracle_mod, r):
    # mixed monomial x^a y^b z^c, each degree <= 2r+1; the Laplacian is exact at points
    # at least r cells from every face.
    h = 0.25
    n = 2 * r + 5
    ax = (np.arange(n) - n // 2) * h
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    a, b, c = 2 * r + 1, 2 * r, 3
    u = x ** a * y ** b * z ** c
    exact = (a * (a - 1) * x ** (a - 2) * y ** b * z ** c + b * (b - 1) * x ** a * y ** (b - 2) * z ** c
             + c * (c - 1) * x ** a * y ** b * z ** (c - 2))
    lap = oracle_mod.laplacian(u, r, h)
    s = slice(r, n - r)
    err = np.abs(lap - exact)[s, s, s]
    assert err.max() <= 1e-9 * max(1.0, np.abs(exact[s, s, s]).max())


@pytest.mark.parametrize("r", [1, 2, 3])
def test_operator_convergence_slope(oracle_mod, r):
    # relative error of L on sin(k x) (periodic) falls like h^{2r} with constant c_r
    L = 1.0
    errs, hs = [], []
    for n in (16, 32, 64):
        h = L / n
        x = np.arange(n) * h
        k = 2 * math.pi / L
        u = np.sin(k * x)
        lap = oracle_mod.laplacian(u, r, h, periodic=True)
        err = np.abs(lap + k * k * u).max() / (k * k)
        errs.append(err)
        hs.append(h)
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(np.abs(slopes - 2 * r) < 0.15), slopes
    c_r = 2 * math.factorial(r) ** 2 / math.factorial(2 * r + 2)
    kh = 2 * math.pi / 64
    assert abs(errs[-1] / kh ** (2 * r) - c_r) / c_r < 0.05


def test_zero_boundary_is_zero_padding(oracle_mod):
    # Dirichlet reading: the zero-ghost result equals the periodic result on a box padded
    # with >= r zero cells on each side, restricted to the original grid.
    rng = np.random.default_rng(5)
    r = 4
    u = rng.standard_normal((7, 9, 11))
    lap = oracle_mod.laplacian(u, r, 1.3)
    big = np.zeros((7 + 2 * r, 9 + 2 * r, 11 + 2 * r))
    big[r:-r, r:-r, r:-r] = u
    lap_big = oracle_mod.laplacian(big, r, 1.3, periodic=True)
    assert np.allclose(lap, lap_big[r:-r, r:-r, r:-r], rtol=0, atol=1e-12)
