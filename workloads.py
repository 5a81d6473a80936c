"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module draws velocity models, shot geometry and request arrival times from
seeds.  It holds none of the method's arithmetic: no stencil weights, no time
step, no Ricker wavelet, no update.  Each side computes those itself (the GPU
library through its C ABI, the oracle through ``oracle``) from the Courant
factor and frequency stated here.

The paper benchmarks "a representative synthetic test case" whose grid, model
and source it does not state; the five workloads below stand in for it.  All
randomness comes from ``numpy.random.SeedSequence(seed).spawn`` so that each
purpose (model, anomalies, FD cells, arrivals, per-request models) has its own
stream.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# ----------------------------------------------------------------------------- velocity models


def layered_profile(nd: int, nlayers: int = 8, vmin: float = 1500.0, vmax: float = 4500.0,
                    seed: int = 0) -> np.ndarray:
    """Velocity per depth index of ``nlayers`` horizontal layers of equal thickness, drawn
    top to bottom from U[vmin, vmax] (unsorted)."""
    rng = np.random.default_rng(seed)
    vel = rng.uniform(vmin, vmax, size=nlayers)
    layer = np.minimum((np.arange(nd) * nlayers) // nd, nlayers - 1)
    return vel[layer]


def layered_velocity(shape, nlayers: int = 8, vmin: float = 1500.0, vmax: float = 4500.0,
                     seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Horizontal layers of equal thickness along the slowest (depth) axis, velocities
    drawn top to bottom from U[vmin, vmax] (unsorted).  shape is (nz, ny, nx) or (ny, nx)."""
    nd = shape[0]
    prof = layered_profile(nd, nlayers, vmin, vmax, seed)
    v = np.broadcast_to(prof.reshape((nd,) + (1,) * (len(shape) - 1)), shape)
    return np.ascontiguousarray(v, dtype=dtype)


def gaussian_smooth_periodic(f: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian filter of standard deviation ``sigma`` cells, applied with FFTs on a
    periodic box (a model generator, not part of the method)."""
    F = np.fft.rfftn(f)
    mult = np.ones(F.shape)
    for ax, n in enumerate(f.shape):
        freq = np.fft.rfftfreq(n) if ax == f.ndim - 1 else np.fft.fftfreq(n)
        g = np.exp(-0.5 * (2 * np.pi * freq * sigma) ** 2)
        shp = [1] * f.ndim
        shp[ax] = g.shape[0]
        mult = mult * g.reshape(shp)
    return np.fft.irfftn(F * mult, s=f.shape, axes=tuple(range(f.ndim)))


def smoothed_noise_velocity(shape, mean: float = 2500.0, std: float = 300.0, sigma: float = 8.0,
                            seed: int = 1, dtype=np.float64) -> np.ndarray:
    """White N(0,1) noise, Gaussian-smoothed (sigma cells, periodic), rescaled to exactly
    ``std`` and shifted to ``mean``."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(shape)
    s = gaussian_smooth_periodic(f, sigma)
    s = (s - s.mean()) / s.std() * std + mean
    return np.ascontiguousarray(s, dtype=dtype)


def gaussian_anomalies(shape, n: int = 3, amplitude: float = 200.0, sigma: float = 12.0,
                       zmin: int = 0, seed: int = 0) -> np.ndarray:
    """Sum of ``n`` Gaussian blobs (sigma cells), centres uniform in [N/4, 3N/4] along
    each axis and below depth ``zmin``, amplitudes +-``amplitude`` with random sign."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    out = np.zeros(shape)
    for _ in range(n):
        c = [rng.uniform(s / 4, 3 * s / 4) for s in shape]
        c[0] = max(c[0], zmin + 2 * sigma) if shape[0] > zmin + 2 * sigma else c[0]
        sign = 1.0 if rng.random() < 0.5 else -1.0
        d2 = sum((g - ci) ** 2 for g, ci in zip(grids, c))
        out += sign * amplitude * np.exp(-0.5 * d2 / sigma ** 2)
    return out


# ----------------------------------------------------------------------------- geometry, arrivals


def surface_receivers(nx: int, ny: int, z: int, every: int) -> np.ndarray:
    """(x, y, z) positions on the plane z, every ``every``-th point in x and y, x fastest."""
    xs = np.arange(0, nx, every)
    ys = np.arange(0, ny, every)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), np.full(xx.size, z)], axis=1).astype(np.int64)


def line_receivers(nx: int, y: int) -> np.ndarray:
    """(x, y) positions along the row y of a 2-D grid."""
    return np.stack([np.arange(nx), np.full(nx, y)], axis=1).astype(np.int64)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of ``rate`` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def spawn_seeds(seed: int, n: int) -> list[int]:
    return [int(s.generate_state(1)[0]) for s in np.random.SeedSequence(seed).spawn(n)]


# ----------------------------------------------------------------------------- the five workloads


@dataclasses.dataclass
class Shot:
    """One forward shot: everything either side needs to run it, except the time step,
    which each side derives from ``courant`` and its own stability limit."""

    name: str
    ndim: int
    shape: tuple            # dense array shape (nz, ny, nx) or (ny, nx)
    h: float
    r: int
    dtype: str              # "f32" or "f64"
    courant: float          # dt = courant * dt_max(ndim, r, h, max(v))
    nsteps: int
    source: tuple           # (x, y[, z])
    f0: float = 15.0
    receivers: Optional[np.ndarray] = None
    velocity_kind: str = "constant"
    velocity_args: dict = dataclasses.field(default_factory=dict)

    def velocity(self) -> np.ndarray:
        if self.velocity_kind == "constant":
            return np.full(self.shape, float(self.velocity_args.get("v", 2000.0)))
        if self.velocity_kind == "layered":
            return layered_velocity(self.shape, **self.velocity_args)
        if self.velocity_kind == "smoothed_noise":
            return smoothed_noise_velocity(self.shape, **self.velocity_args)
        raise ValueError(self.velocity_kind)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))


def c1_2d_fp64() -> Shot:
    """2-D, 256x256, h = 10 m, r = 4, FP64, constant 2000 m/s, dt = 0.5 CFL, Ricker 15 Hz
    at the centre, zero boundaries, 500 steps, one receiver line at row 32."""
    return Shot("2d_256_r4_fp64", 2, (256, 256), 10.0, 4, "f64", 0.5, 500, (128, 128),
                receivers=line_receivers(256, 32), velocity_kind="constant", velocity_args={"v": 2000.0})


def c2_3d_layered(n: int = 512, nsteps: int = 1000, seed: int = 0) -> Shot:
    """3-D, 512^3, h = 10 m, r = 4 (25-point star), FP32, 8 layers with v ~ U[1500, 4500],
    Ricker 15 Hz at (256, 256, 16), 1000 steps, surface receivers every 4th point."""
    zs = round(16 * n / 512)
    return Shot(f"3d_{n}_r4_layered_fp32", 3, (n, n, n), 10.0, 4, "f32", 0.5, nsteps,
                (n // 2, n // 2, zs), receivers=surface_receivers(n, n, zs, 4),
                velocity_kind="layered", velocity_args={"seed": seed})


def c3_3d_noise(n: int = 384, nsteps: int = 2000, seed: int = 1) -> Shot:
    """3-D, 384^3, r = 8 (49-point star), FP32, v = 2500 + smoothed noise (sigma 8 cells,
    std 300), 2000 steps, dt = 0.4 CFL."""
    zs = round(16 * n / 512)
    return Shot(f"3d_{n}_r8_noise_fp32", 3, (n, n, n), 10.0, 8, "f32", 0.4, nsteps,
                (n // 2, n // 2, zs), receivers=surface_receivers(n, n, zs, 4),
                velocity_kind="smoothed_noise", velocity_args={"seed": seed})


@dataclasses.dataclass
class GradientCase:
    """Forward + adjoint gradient: true model = layered + 3 Gaussian anomalies, start model
    = layered only, one shot, surface receivers, L2 misfit, checkpoints every ``ckpt``."""

    n: int = 256
    r: int = 4
    nsteps: int = 2000
    ckpt: int = 50
    rec_every: int = 2
    seed: int = 2
    fd_cells: int = 16
    h: float = 10.0
    courant: float = 0.5
    f0: float = 15.0

    def models(self):
        s_layer, s_anom, s_cells = spawn_seeds(self.seed, 3)
        shape = (self.n,) * 3
        base = layered_velocity(shape, seed=s_layer)
        zs = self.source[2]
        true = base + gaussian_anomalies(shape, 3, 200.0, 12.0 * self.n / 256, zmin=zs, seed=s_anom)
        return true, base

    @property
    def source(self):
        return (self.n // 2, self.n // 2, max(1, round(8 * self.n / 256)))

    def receivers(self):
        return surface_receivers(self.n, self.n, self.source[2], self.rec_every)

    def fd_cells_idx(self):
        """Cells for the finite-difference check: uniform over points at least r from every wall."""
        _, _, s_cells = spawn_seeds(self.seed, 3)
        rng = np.random.default_rng(s_cells)
        lo, hi = self.r, self.n - self.r
        return rng.integers(lo, hi, size=(self.fd_cells, 3))  # (z, y, x) array indices


def stretched_z(nz: int, rz: int, h: float, stretch: float = 1.5) -> np.ndarray:
    """Coordinates of planes -rz .. nz+rz-1 of a z grid whose spacing grows linearly with
    depth from h (top) to stretch * h (bottom), rounded to multiples of 1/64 m.  The rz
    ghost planes above and below continue the end spacings."""
    k = np.arange(-rz, nz + rz - 1, dtype=np.float64)
    frac = np.clip(k, 0, max(nz - 1, 1)) / max(nz - 1, 1)
    dz = h * (1.0 + (stretch - 1.0) * frac)
    z = np.concatenate([[-rz * h], -rz * h + np.cumsum(dz)])
    return np.round(z * 64.0) / 64.0


@dataclasses.dataclass
class VtiShot:
    """One shot of the two-field VTI propagator: layered vertical velocity with layered
    anisotropy (eps ~ U[0.05, 0.25] per layer, delta = eps * U[0.2, 0.8], so delta <= eps),
    a z grid stretched with depth, Ricker source forcing p only (the form of eq. (p))."""

    n: int = 512
    rxy: int = 12
    rz: int = 8
    dtype: str = "f32"
    nsteps: int = 1000
    h: float = 10.0
    stretch: float = 1.5
    courant: float = 0.5
    f0: float = 15.0
    seed: int = 5

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    def models(self, dtype=np.float64):
        s_v, s_e, s_d = spawn_seeds(self.seed, 3)
        nl = 8
        vz = layered_velocity(self.shape, nl, seed=s_v, dtype=dtype)
        e = np.random.default_rng(s_e).uniform(0.05, 0.25, size=nl)
        d = e * np.random.default_rng(s_d).uniform(0.2, 0.8, size=nl)
        layer = np.minimum((np.arange(self.n) * nl) // self.n, nl - 1)
        eps = np.ascontiguousarray(np.broadcast_to(e[layer][:, None, None], self.shape), dtype=dtype)
        delta = np.ascontiguousarray(np.broadcast_to(d[layer][:, None, None], self.shape), dtype=dtype)
        return vz, eps, delta

    def zc(self) -> np.ndarray:
        return stretched_z(self.n, self.rz, self.h, self.stretch)

    @property
    def source(self):
        return (self.n // 2, self.n // 2, max(1, round(16 * self.n / 512)))

    def receivers(self):
        return surface_receivers(self.n, self.n, self.source[2], 4)

    @property
    def npoints(self) -> int:
        return self.n ** 3


@dataclasses.dataclass
class ServeRequest:
    rid: int
    arrival: float          # seconds after the trace starts
    n: int                  # cubic grid side
    nsteps: int
    seed: int               # per-request velocity seed

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    @property
    def source(self):
        return (self.n // 2, self.n // 2, max(1, round(16 * self.n / 512)))

    def receivers(self):
        return surface_receivers(self.n, self.n, self.source[2], 4)

    def velocity(self, dtype=np.float32):
        return layered_velocity(self.shape, seed=self.seed, dtype=dtype)

    def profile(self) -> np.ndarray:
        """Velocity per depth index of this request's layered model."""
        return layered_profile(self.n, seed=self.seed)

    @property
    def points(self) -> int:
        return self.n ** 3 * self.nsteps


def serving_trace(nreq: int = 256, rate: float = 20.0, sides=(128, 192, 256, 320, 400),
                  steps=(500, 2000), seed: int = 4) -> list[ServeRequest]:
    """Poisson arrivals at ``rate`` req/s, cubic sides uniform over ``sides``, step counts
    uniform integers in [steps[0], steps[1]], per-request layered-model seeds."""
    s_arr, s_side, s_steps, s_models = spawn_seeds(seed, 4)
    t = poisson_arrivals(nreq, rate, s_arr)
    side = np.random.default_rng(s_side).choice(np.asarray(sides), size=nreq)
    ns = np.random.default_rng(s_steps).integers(steps[0], steps[1] + 1, size=nreq)
    seeds = spawn_seeds(s_models, nreq)
    return [ServeRequest(i, float(t[i]), int(side[i]), int(ns[i]), seeds[i]) for i in range(nreq)]
