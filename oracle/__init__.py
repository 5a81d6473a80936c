"""Plain FP64 CPU oracle for explicit leapfrog acoustic finite differences.

TEST INFRASTRUCTURE ONLY.  This package is imported, called or executed only by
``tests/``, by ``__graft_entry__.smoke()`` (to check one GPU result) and by the
``cpu_baseline`` leg of ``bench.py``.  The GPU library never loads it and shares
no code, header, table or helper with it; the two meet only at the seeded input
generators in ``workloads.py``, which hold none of the method's arithmetic.

What is computed, and where the paper (Medina, St-Cyr, Warburton, "High-Order
Finite-differences on multi-threaded architectures using OCCA") defines it:

* ``weights``   -- the symmetric xy stencil of Sec. 1 (R+1 weights w0..wR, the
  centre weight taken per axis), with the weights fixed as the exact central
  approximation of the second derivative: the unique symmetric stencil that is
  exact on every polynomial of degree <= 2r+1 (Taylor conditions), solved in
  rational arithmetic.  The paper prints the form, not the values.
* ``ricker``    -- the Ricker forcing of Sec. 1, s = (1 - 2 pi^2 f^2 t^2) exp(-pi^2 f^2 t^2),
  evaluated at t = n dt - t0 (the time shift t0 is this build's reading; the
  paper prints none).
* ``dt_max``    -- the von Neumann limit of the centred time scheme of Sec. 1 for
  this stencil: dt^2 v^2 kappa_max^2 <= 4, with kappa_max^2 the largest
  eigenvalue of -L.
* ``laplacian``, ``forward`` -- the time scheme u^{n+1} - 2u^n + u^{n-1} = dt^2 F(u^n)
  of Sec. 1 with the isotropic reduction F = v^2 L u + s(t) delta (Sec. 1, eq. (p)
  with p = q), zero values for r points outside the domain (Sec. 1, last
  paragraph), or a periodic box for closed-form tests.  Implemented in
  ``fd_oracle.c`` as plain loops.
* ``z_weights``, ``vti_dt_max``, ``vti_forward`` -- the two-field VTI propagator
  of Sec. 1 (eqs. (p) and (q)): p and q advanced together by the centred time
  scheme, the symmetric radius-Rxy xy stencil acting on p, and a per-plane
  2Rz+1-point z stencil acting on q whose weights absorb a variable spacing
  dz_k (Sec. 1).  ``vti_oracle.c`` holds the loops.
* ``cerjan``, ``damping_field`` -- the absorbing sponge the paper embeds the domain in
  (Sec. 1, after Cerjan et al., whose profile and constants the paper does not print):
  ``forward(..., damping=...)`` scales both time levels by G every step.
* ``gradient``  -- the discrete adjoint (Lagrange multiplier recursion of the
  forward scheme) of J = 1/2 sum (traces - observed)^2 with respect to v.
  Not in the paper; its statement of the problem names full waveform inversion
  as the application (Sec. 1).

Every pin of this oracle lives in ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fd_oracle.c"), os.path.join(_HERE, "vti_oracle.c")]
_LIB = os.path.join(_HERE, "libfd_oracle.so")

__all__ = [
    "build",
    "weights",
    "weights_f64",
    "ricker",
    "dt_max",
    "laplacian",
    "forward",
    "gradient",
    "misfit",
    "linear_index",
    "z_weights_exact",
    "z_weights",
    "vti_dt_max",
    "vti_forward",
    "cerjan",
    "damping_field",
]


# --------------------------------------------------------------------------- build / load


def build(force: bool = True) -> str:
    """Compile the C sources with gcc (IEEE FP64: no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and all(os.path.getmtime(_LIB) >= os.path.getmtime(f) for f in _SRCS):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = [
        "gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        *_SRCS, "-o", tmp, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.fdo_laplacian.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, P, P]
        lib.fdo_forward.argtypes = [
            ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int,
            I64, I64, P, P, I64, P, P, P, P, P, P,
        ]
        lib.fdo_adjoint.argtypes = [
            ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int,
            I64, I64, P, P, P, P,
        ]
        lib.fdo_adjoint_range.argtypes = [
            ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int,
            I64, I64, I64, P, P, P, P, P, P,
        ]
        lib.fdo_vti_forward.argtypes = [
            P, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int,
            ctypes.c_int, I64, I64, P, P, P, I64, P, P, P, P, P, P, P,
        ]
        for f in (lib.fdo_laplacian, lib.fdo_forward, lib.fdo_adjoint, lib.fdo_adjoint_range,
                  lib.fdo_vti_forward):
            f.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(status: int, what: str):
    if status != 0:
        raise ValueError(f"oracle {what} failed with status {status}")


# --------------------------------------------------------------------------- stencil weights


@lru_cache(maxsize=None)
def weights(r: int) -> tuple[Fraction, ...]:
    """Exact weights (w0, w1, ..., wr) of the symmetric radius-r stencil
    h^2 u'' ~ w0 u_i + sum_l w_l (u_{i+l} + u_{i-l}) that is exact for every
    polynomial of degree <= 2r+1 (Sec. 1 stencil form; weight values fixed by
    the Taylor conditions, this build's reading).

    Odd powers vanish by symmetry; the even powers x^{2k}, k = 0..r, give r+1
    linear equations in r+1 unknowns (unit spacing, evaluated at 0):
        k = 0:  w0 + 2 sum_l w_l = 0
        k = 1:  2 sum_l w_l l^2 = 2
        k >= 2: 2 sum_l w_l l^{2k} = 0
    solved by Gaussian elimination over the rationals.
    """
    if not (1 <= r <= 16):
        raise ValueError("r must be in [1, 16]")
    rows = []
    for k in range(r + 1):
        row = [Fraction(1 if k == 0 else 0)]  # coefficient of w0: 0^{2k}
        row += [Fraction(2 * l ** (2 * k)) for l in range(1, r + 1)]
        rhs = Fraction(2) if k == 1 else Fraction(0)
        rows.append(row + [rhs])
    return tuple(_solve_exact(rows))


def _solve_exact(rows):
    """Solution of the square system given as augmented rows [a_0 .. a_{n-1} | b],
    by Gauss-Jordan elimination over the rationals (exact pivots)."""
    rows = [list(r) for r in rows]
    nunk = len(rows)
    for col in range(nunk):
        piv = next(i for i in range(col, nunk) if rows[i][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [x / p for x in rows[col]]
        for i in range(nunk):
            if i != col and rows[i][col] != 0:
                f = rows[i][col]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[col])]
    return [rows[i][nunk] for i in range(nunk)]


def weights_f64(r: int) -> np.ndarray:
    """The exact weights rounded to the nearest double."""
    return np.array([float(x) for x in weights(r)], dtype=np.float64)


# --------------------------------------------------------------------------- source, CFL


def ricker(nsamp: int, dt: float, f0: float = 15.0, t0: float | None = None) -> np.ndarray:
    """Ricker samples s[n] = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = n dt - t0
    (Sec. 1 forcing, f = 15 Hz).  The default shift t0 = 1.5 / f starts the wavelet
    from ~1e-8 instead of from its peak (this build's reading)."""
    if t0 is None:
        t0 = 1.5 / f0
    tau = np.arange(nsamp, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * tau) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def symbol_max(r: int) -> float:
    """Largest value over theta of the 1-D stencil symbol -(w0 + 2 sum_l w_l cos(l theta)),
    taken at theta = pi, where every term adds: -w0 - 2 sum_l w_l (-1)^l."""
    w = weights(r)
    s = -w[0] - 2 * sum(w[l] * (-1) ** l for l in range(1, r + 1))
    return float(s)


def dt_max(ndim: int, r: int, h: float, vmax: float) -> float:
    """Stability limit of the leapfrog scheme: a Fourier mode with eigenvalue -kappa^2 of L
    stays bounded iff dt^2 v^2 kappa^2 <= 4, and kappa_max^2 = ndim * symbol_max(r) / h^2."""
    return 2.0 * h / (vmax * math.sqrt(ndim * symbol_max(r)))


# --------------------------------------------------------------------------- grids


def _dims(shape) -> tuple[int, np.ndarray]:
    """Dense array shape (nz, ny, nx) / (ny, nx) / (nx,) -> ndim and n = [nx, ny, nz]."""
    ndim = len(shape)
    if ndim not in (1, 2, 3):
        raise ValueError("ndim must be 1, 2 or 3")
    rev = list(shape[::-1]) + [1] * (3 - ndim)
    return ndim, np.array(rev, dtype=np.int64)


def linear_index(shape, pos) -> np.ndarray:
    """Linear indices of positions given as (x, y, z) tuples (x fastest)."""
    ndim, n = _dims(shape)
    pos = np.atleast_2d(np.asarray(pos, dtype=np.int64))
    if pos.shape[1] != ndim:
        raise ValueError(f"positions must have {ndim} coordinates")
    idx = np.zeros(pos.shape[0], dtype=np.int64)
    stride = 1
    for a in range(ndim):
        if np.any(pos[:, a] < 0) or np.any(pos[:, a] >= n[a]):
            raise ValueError("position outside the grid")
        idx += pos[:, a] * stride
        stride *= int(n[a])
    return idx


def laplacian(u: np.ndarray, r: int, h: float, periodic: bool = False) -> np.ndarray:
    """L u = h^-2 [ndim w0 u + sum_axes sum_l w_l (u_{+l} + u_{-l})] (Sec. 1 stencil form)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    ndim, n = _dims(u.shape)
    w = weights_f64(r)
    out = np.empty_like(u)
    _check(_lib().fdo_laplacian(ndim, _ptr(n), r, _ptr(w), h, int(periodic), _ptr(u), _ptr(out)), "laplacian")
    return out


def _source_arrays(shape, sources, nsteps):
    nsrc = len(sources)
    idx = np.zeros(nsrc, dtype=np.int64)
    samples = np.zeros((nsteps, nsrc), dtype=np.float64)
    for s, (pos, wav) in enumerate(sources):
        idx[s] = linear_index(shape, [pos])[0]
        wav = np.asarray(wav, dtype=np.float64)
        k = min(nsteps, wav.shape[0])
        samples[:k, s] = wav[:k]
    return idx, np.ascontiguousarray(samples)


def cerjan(n: int, width: int, alpha: float, lo: bool = True, hi: bool = True) -> np.ndarray:
    """Cerjan et al. (Geophysics 50, 1985) sponge factor along one axis of n points: in a
    strip of `width` points at a damped face, the point at distance i from the face
    (i = 0 outermost) gets exp(-(alpha (width - i))^2); 1 elsewhere (factors of two
    overlapping strips multiply)."""
    g = np.ones(n)
    for i in range(min(width, n)):
        f = math.exp(-(alpha * (width - i)) ** 2)
        if lo:
            g[i] *= f
        if hi:
            g[n - 1 - i] *= f
    return g


def damping_field(shape, width: int, alpha: float, faces=(True,) * 6) -> np.ndarray:
    """Point-wise sponge factor G of a dense (nz, ny, nx) / (ny, nx) grid: the product of
    the per-axis Cerjan profiles; faces = (x-, x+, y-, y+[, z-, z+])."""
    ndim = len(shape)
    G = np.ones(shape)
    for a in range(ndim):           # a = 0: x (last array axis)
        n = shape[ndim - 1 - a]
        prof = cerjan(n, width, alpha, faces[2 * a], faces[2 * a + 1])
        sh = [1] * ndim
        sh[ndim - 1 - a] = n
        G = G * prof.reshape(sh)
    return G


def forward(v, h, dt, r, nsteps, sources=(), receivers=None, periodic=False, u0=None, um1=None,
            store_states=False, damping=None):
    """Run ``nsteps`` leapfrog steps of u_tt = v^2 L u + sum_s s_s(t) delta_s.

    v          velocity, dense (nz, ny, nx) / (ny, nx) / (nx,), m/s
    sources    sequence of ((x[, y[, z]]), samples) -- sample n enters the step that
               produces u^{n+1}, scaled by dt^2 / h^ndim (discrete delta)
    receivers  int array [nrec, ndim] of (x, y, z) positions; traces[n][j] = u^{n+1}(x_j)
    u0, um1    initial u^0 and u^{-1} (default zero)
    damping    optional (width, alpha[, faces]): a Cerjan sponge (see damping_field); both
               time levels are scaled by G every step: u^{n+1} = G (2u^n - G u^{n-1} + ...)

    Returns dict(u=u^T, u_prev=u^{T-1}, traces=[T, nrec], states=[T+1, ...] or None).
    """
    v = np.ascontiguousarray(v, dtype=np.float64)
    shape = v.shape
    ndim, n = _dims(shape)
    m = np.ascontiguousarray(v * v)
    w = weights_f64(r)
    u = np.zeros(shape) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    up = np.zeros(shape) if um1 is None else np.array(um1, dtype=np.float64, copy=True)
    src_idx, src = _source_arrays(shape, list(sources), nsteps)
    if receivers is None or len(receivers) == 0:
        rec_idx = np.zeros(0, dtype=np.int64)
    else:
        rec_idx = linear_index(shape, receivers)
    traces = np.zeros((nsteps, rec_idx.shape[0]), dtype=np.float64)
    states = np.zeros((nsteps + 1,) + shape, dtype=np.float64) if store_states else None
    G = None
    if damping is not None:
        G = np.ascontiguousarray(damping_field(shape, *damping))
    st = _lib().fdo_forward(
        ndim, _ptr(n), r, _ptr(w), float(h), float(dt), _ptr(m), int(periodic), int(nsteps),
        int(src_idx.shape[0]), _ptr(src_idx), _ptr(src), int(rec_idx.shape[0]), _ptr(rec_idx),
        _ptr(traces), _ptr(u), _ptr(up), _ptr(states), _ptr(G),
    )
    _check(st, "forward")
    return {"u": u, "u_prev": up, "traces": traces, "states": states}


def misfit(traces, observed) -> float:
    """J = 1/2 sum_n sum_j (traces - observed)^2."""
    d = np.asarray(traces, dtype=np.float64) - np.asarray(observed, dtype=np.float64)
    return 0.5 * float(np.sum(d * d))


def gradient(v, h, dt, r, nsteps, sources, receivers, observed, periodic=False, checkpoint=None, progress=None):
    """J and dJ/dv for J = 1/2 sum (traces - observed)^2 by the discrete adjoint.

    Runs the Lagrange multiplier recursion in fd_oracle.c for dJ/dm (m = v^2) and returns
    dJ/dv = 2 v dJ/dm.  The recursion at step k needs the forward state u^{k-1}:
    checkpoint=None stores every state u^0..u^{T-1} (small grids only); checkpoint=K keeps
    (u^{jK}, u^{jK-1}) for j = 0, 1, .. and, segment by segment from the last one,
    recomputes u^{jK}..u^{jK+K-1} from its checkpoint before running the recursion over
    that segment, so the memory is about T/K + K fields.  Both give the same numbers bit
    for bit (the recomputed states are the stored ones).  Returns dict(J, grad_v, grad_m,
    traces).
    """
    v = np.ascontiguousarray(v, dtype=np.float64)
    shape = v.shape
    ndim, n = _dims(shape)
    rec_idx = linear_index(shape, receivers)
    m = np.ascontiguousarray(v * v)
    w = weights_f64(r)
    obs = np.asarray(observed, dtype=np.float64)
    grad_m = np.zeros(shape, dtype=np.float64)
    if checkpoint is None:
        fw = forward(v, h, dt, r, nsteps, sources, receivers, periodic=periodic, store_states=True)
        traces = fw["traces"]
        resid = np.ascontiguousarray(traces - obs)
        states = np.ascontiguousarray(fw["states"][:nsteps])
        st = _lib().fdo_adjoint(
            ndim, _ptr(n), r, _ptr(w), float(h), float(dt), _ptr(m), int(periodic), int(nsteps),
            int(rec_idx.shape[0]), _ptr(rec_idx), _ptr(resid), _ptr(states), _ptr(grad_m),
        )
        _check(st, "adjoint")
    else:
        K = int(checkpoint)
        if K < 1:
            raise ValueError("checkpoint interval must be >= 1")
        sources = [(pos, np.asarray(wav, dtype=np.float64)) for pos, wav in sources]

        def segment(k0, nst, u0, um1, store):
            # the forward scheme from (u^{k0}, u^{k0-1}) for nst steps; source sample k0 + i
            # enters step i
            return forward(v, h, dt, r, nst, [(pos, wav[k0:]) for pos, wav in sources], receivers,
                           periodic=periodic, u0=u0, um1=um1, store_states=store)

        bounds = [(k, min(k + K, nsteps)) for k in range(0, nsteps, K)]
        ckpts = []
        traces = np.zeros((nsteps, rec_idx.shape[0]))
        u, up = np.zeros(shape), np.zeros(shape)
        for k_lo, k_hi in bounds:
            ckpts.append((u, up))
            fw = segment(k_lo, k_hi - k_lo, u, up, False)
            traces[k_lo:k_hi] = fw["traces"]
            u, up = fw["u"], fw["u_prev"]
            if progress is not None:
                progress(f"oracle gradient: forward to step {k_hi} of {nsteps}")
        resid = np.ascontiguousarray(traces - obs)
        lam1, lam2 = np.zeros(shape), np.zeros(shape)  # lambda^{T+1} = lambda^{T+2} = 0
        for (k_lo, k_hi), (u0, um1) in zip(reversed(bounds), reversed(ckpts)):
            # u^{k_lo} .. u^{k_hi-1}: the checkpoint and k_hi - k_lo - 1 recomputed steps
            states = np.ascontiguousarray(segment(k_lo, k_hi - k_lo - 1, u0, um1, True)["states"])
            st = _lib().fdo_adjoint_range(
                ndim, _ptr(n), r, _ptr(w), float(h), float(dt), _ptr(m), int(periodic), int(k_hi), int(k_lo),
                int(rec_idx.shape[0]), _ptr(rec_idx), _ptr(resid), _ptr(states), _ptr(lam1), _ptr(lam2),
                _ptr(grad_m),
            )
            _check(st, "adjoint_range")
            del states
            if progress is not None:
                progress(f"oracle gradient: adjoint down to step {k_lo}")
    return {
        "J": misfit(traces, obs),
        "grad_m": grad_m,
        "grad_v": 2.0 * v * grad_m,
        "traces": traces,
    }


# --------------------------------------------------------------------------- VTI propagator


@lru_cache(maxsize=None)
def _z_weights_cached(zc: tuple, rz: int) -> tuple:
    nz = len(zc) - 2 * rz
    table = []
    for k in range(nz):
        zk = zc[k + rz]
        d = [zc[k + rz + l] - zk for l in range(-rz, rz + 1)]
        # moments: sum_l w_l d_l^m = (d^2/dz^2) (z - z_k)^m at z_k = 2 if m == 2 else 0
        rows = [[di ** m for di in d] + [Fraction(2 if m == 2 else 0)] for m in range(2 * rz + 1)]
        table.append(tuple(_solve_exact(rows)))
    return tuple(table)


def z_weights_exact(zc, rz: int) -> tuple:
    """Per-plane second-derivative weights of the z stencil of Sec. 1: for plane k the
    2rz+1 weights w_{k,l} (l = -rz..rz) of the unique stencil on the planes k-rz..k+rz
    that differentiates every polynomial of degree <= 2rz exactly at z_k, as exact
    fractions.  zc holds the coordinates of planes -rz .. nz+rz-1 (the rz ghost planes
    on each side included), strictly increasing; each double is taken exactly."""
    zc = tuple(Fraction(float(z)) for z in zc)
    if len(zc) < 2 * rz + 1 or any(b <= a for a, b in zip(zc, zc[1:])):
        raise ValueError("z coordinates must be strictly increasing, nz >= 1")
    return _z_weights_cached(zc, int(rz))


def z_weights(zc, rz: int) -> np.ndarray:
    """z_weights_exact rounded to doubles, as an [nz][2rz+1] array."""
    return np.array([[float(w) for w in row] for row in z_weights_exact(zc, rz)], dtype=np.float64)


def uniform_z(nz: int, rz: int, dz: float) -> np.ndarray:
    """Coordinates of planes -rz .. nz+rz-1 of a uniform z grid (plane 0 at z = 0)."""
    return np.arange(-rz, nz + rz, dtype=np.float64) * dz


def _cell_dz(zc, rz: int) -> np.ndarray:
    """z extent of the cell of plane k: half the distance between its two neighbours
    (the spacing itself on a uniform grid)."""
    zc = np.asarray(zc, dtype=np.float64)
    nz = zc.shape[0] - 2 * rz
    k = np.arange(nz) + rz
    return 0.5 * (zc[k + 1] - zc[k - 1])


def vti_dt_max(rxy: int, rz: int, h: float, wz: np.ndarray, vz, eps, delta) -> float:
    """Largest stable time step.  For constant coefficients a Fourier mode on which
    -(Dxx + Dyy) and -Dzz act as the numbers a_xy and a_z obeys the 2x2 recursion with
        M = [[nux2 a_xy, nuz2 a_z], [nun2 a_xy, nuz2 a_z]],
    stable iff every eigenvalue of M lies in [0, 4/dt^2].  M has non-negative entries, so
    its largest eigenvalue grows with each entry: it is largest at a_xy = 2 S_xy / h^2
    (both axes at the Nyquist point) and the largest a_z, bounded by the largest row sum
    of |wz| (exact on a uniform grid).  The smaller eigenvalue is negative when
    nun2 > nux2 (delta > eps); no time step is stable then and 0.0 is returned."""
    w = weights(rxy)
    sxy = float(-w[0] - 2 * sum(w[l] * (-1) ** l for l in range(1, rxy + 1)))
    axy = 2.0 * sxy / (h * h)
    az = float(np.max(np.sum(np.abs(np.asarray(wz, dtype=np.float64)), axis=1)))
    vz = np.asarray(vz, dtype=np.float64)
    nuz2 = vz * vz
    nux2 = nuz2 * (1.0 + 2.0 * np.asarray(eps, dtype=np.float64))
    nun2 = nuz2 * (1.0 + 2.0 * np.asarray(delta, dtype=np.float64))
    if np.any(nun2 > nux2):
        return 0.0
    a, b, c = nux2 * axy, nuz2 * az, nun2 * axy
    lam = 0.5 * ((a + b) + np.sqrt((a - b) ** 2 + 4.0 * b * c))
    return float(2.0 / math.sqrt(float(np.max(lam))))


def vti_forward(vz, eps, delta, h, dt, rxy, rz, nsteps, zc=None, sources=(), receivers=None,
                periodic_xy=False, periodic_z=False, state=None):
    """Run ``nsteps`` steps of the VTI scheme (Sec. 1, eqs. (p), (q)).

    vz, eps, delta  dense (nz, ny, nx) models: vertical velocity (m/s) and the two
                    anisotropy parameters
    zc              coordinates of planes -rz .. nz+rz-1 (default: uniform, spacing h)
    sources         sequence of ((x, y, z), samples, amp_p, amp_q): sample n enters the
                    step producing level n+1, scaled by dt^2 / (h^2 dz_k)
    receivers       int array [nrec, 3] of (x, y, z); traces[n][j] = field^{n+1}(x_j)
    state           optional (p0, pm1, q0, qm1), default zero

    Returns dict(p, p_prev, q, q_prev, traces_p, traces_q).
    """
    vz = np.ascontiguousarray(vz, dtype=np.float64)
    shape = vz.shape
    if len(shape) != 3:
        raise ValueError("the VTI propagator is three-dimensional")
    nz = shape[0]
    _, n = _dims(shape)
    eps = np.ascontiguousarray(np.broadcast_to(eps, shape), dtype=np.float64)
    delta = np.ascontiguousarray(np.broadcast_to(delta, shape), dtype=np.float64)
    if zc is None:
        zc = uniform_z(nz, rz, h)
    zc = np.asarray(zc, dtype=np.float64)
    if zc.shape[0] != nz + 2 * rz:
        raise ValueError("zc must hold nz + 2 rz plane coordinates")
    wz = np.ascontiguousarray(z_weights(zc, rz))
    dzc = np.ascontiguousarray(_cell_dz(zc, rz))
    wxy = weights_f64(rxy)
    if state is None:
        p, pm, q, qm = (np.zeros(shape) for _ in range(4))
    else:
        p, pm, q, qm = (np.array(a, dtype=np.float64, copy=True) for a in state)
    sources = list(sources)
    nsrc = len(sources)
    src_idx = np.zeros(nsrc, dtype=np.int64)
    src = np.zeros((nsteps, nsrc), dtype=np.float64)
    amp = np.zeros((nsrc, 2), dtype=np.float64)
    for e, (pos, wav, ap, aq) in enumerate(sources):
        src_idx[e] = linear_index(shape, [pos])[0]
        wav = np.asarray(wav, dtype=np.float64)
        k = min(nsteps, wav.shape[0])
        src[:k, e] = wav[:k]
        amp[e] = (ap, aq)
    rec_idx = np.zeros(0, dtype=np.int64) if receivers is None or len(receivers) == 0 else \
        linear_index(shape, receivers)
    trp = np.zeros((nsteps, rec_idx.shape[0]))
    trq = np.zeros((nsteps, rec_idx.shape[0]))
    st = _lib().fdo_vti_forward(
        _ptr(n), int(rxy), int(rz), _ptr(wxy), _ptr(wz), _ptr(dzc), float(h), float(dt), _ptr(vz), _ptr(eps),
        _ptr(delta), int(periodic_xy), int(periodic_z), int(nsteps), nsrc, _ptr(src_idx),
        _ptr(np.ascontiguousarray(src)), _ptr(amp), int(rec_idx.shape[0]), _ptr(rec_idx), _ptr(trp), _ptr(trq),
        _ptr(p), _ptr(pm), _ptr(q), _ptr(qm),
    )
    _check(st, "vti_forward")
    return {"p": p, "p_prev": pm, "q": q, "q_prev": qm, "traces_p": trp, "traces_q": trq}
