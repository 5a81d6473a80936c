"""Propagator: one forward shot on the GPU, with torch owning all device memory.

A thin object over the C ABI: it allocates the workspace, wavelet and trace tensors
with torch on the current device, passes their addresses to libfdwave.so and keeps
them alive for as long as the context borrows them.  All arithmetic happens in the
library's HIP kernels.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import fdwave as F

_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64}


class Propagator:
    """Leapfrog propagator for u_tt = v^2 lap(u) + sources on a 2-D or 3-D grid.

    v         dense velocity tensor (nz, ny, nx) or (ny, nx), on a GPU, dtype float32
              (dtype "f32") or float64 ("f64")
    r         stencil radius (1..8)
    h, dt     grid spacing (m) and time step (s); dt must satisfy fd_dt_max
    bc        "zero" (Dirichlet ghost cells) or "periodic"
    """

    def __init__(self, v: torch.Tensor, r: int, h: float, dt: float, dtype: str = "f32", bc: str = "zero",
                 max_sources: int = 4, max_receivers: int = 0, stream: Optional[torch.cuda.Stream] = None):
        if not v.is_cuda:
            raise ValueError("velocity must be a GPU tensor")
        self.dtype = dtype
        self.tdtype = _TORCH_DTYPE[dtype]
        self.shape = tuple(v.shape)
        self.ndim = len(self.shape)
        self.r, self.h, self.dt, self.bc = r, float(h), float(dt), bc
        self.device = v.device
        self._stream = stream
        v = v.to(self.tdtype).contiguous()
        nbytes = F.fd_workspace_bytes(self.shape, r, dtype, max_sources, max_receivers)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.field_bytes = F.fd_field_bytes(self.shape, r, dtype)
        self._wavelets = []
        self.traces: Optional[torch.Tensor] = None
        self.ctx = F.fd_create(self.shape, r, h, dt, v, dtype, bc, self.workspace, max_sources, max_receivers,
                               self.stream_handle())

    # -------------------------------------------------------------- plumbing

    def stream_handle(self):
        return F.stream_ptr(self._stream)

    @property
    def kernel_config(self) -> str:
        return F.fd_kernel_config(self.ctx)

    @property
    def adjoint_config(self) -> str:
        """Tile shape, z-chunk and launch size of this context's adjoint kernel."""
        return F.fd_adjoint_config(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            F.fd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- sources and receivers

    def ricker(self, nsamp: int, f0: float = 15.0, t0: Optional[float] = None) -> torch.Tensor:
        """Ricker samples at t = n dt - t0 computed on the device (t0 defaults to 1.5 / f0)."""
        t0 = 1.5 / f0 if t0 is None else t0
        out = torch.empty(nsamp, dtype=self.tdtype, device=self.device)
        F.fd_ricker(out, self.dt, f0, t0, self.stream_handle())
        return out

    def inject(self, wavelet: torch.Tensor, pos: Sequence[int], amp: float = 1.0):
        """Add a point source at (x, y[, z]); sample n enters u^{n+1} scaled by amp dt^2 / h^ndim."""
        wavelet = wavelet.to(device=self.device, dtype=self.tdtype).contiguous()
        self._wavelets.append(wavelet)
        F.fd_inject(self.ctx, wavelet, pos, amp)

    def set_damping(self, width: int = 20, alpha: float = 0.015, faces: int = 63):
        """Absorbing sponge of `width` points at the faces in the bit mask `faces` (bit 0 x-,
        1 x+, 2 y-, 3 y+, 4 z-, 5 z+); width = 0 switches it off."""
        F.fd_set_damping(self.ctx, width, alpha, faces)

    def enable_time_blocking(self, config: int = 0):
        """Run fd_step two time steps per launch (bitwise the same result); allocates the
        two extra padded fields the two-step kernel writes into."""
        self.aux = torch.empty(2 * self.field_bytes, dtype=torch.uint8, device=self.device)
        F.fd_set_time_blocking(self.ctx, self.aux, config)

    def disable_time_blocking(self):
        F.fd_set_time_blocking(self.ctx, None)
        self.aux = None

    def clear_sources(self):
        F.fd_clear_sources(self.ctx)
        self._wavelets = []

    def record(self, positions, cap: int) -> torch.Tensor:
        """Record u^{n+1} at positions [(x, y[, z]), ...] for the next ``cap`` steps."""
        positions = np.asarray(positions, dtype=np.int64).reshape(-1, self.ndim)
        nrec = positions.shape[0]
        self.traces = torch.zeros((max(cap, 0), nrec), dtype=self.tdtype, device=self.device)
        F.fd_record(self.ctx, positions, self.traces, cap)
        return self.traces

    # -------------------------------------------------------------- stepping and state

    def step(self, nsteps: int):
        F.fd_step(self.ctx, nsteps)

    def sync(self):
        F.fd_sync(self.ctx)

    def check_finite(self) -> bool:
        """True if the current state (u^n, u^{n-1}) holds no NaN or infinity (synchronises)."""
        return F.fd_check_finite(self.ctx)

    @property
    def step_count(self) -> int:
        return F.fd_get_step(self.ctx)

    def state(self):
        """(u^n, u^{n-1}, n) as dense tensors."""
        u = torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        up = torch.empty(self.shape, dtype=self.tdtype, device=self.device)
        n = F.fd_get_state(self.ctx, u, up, F.FD_DENSE)
        return u, up, n

    def set_state(self, u: torch.Tensor, u_prev: torch.Tensor, step: int):
        F.fd_set_state(self.ctx, u.to(self.tdtype).contiguous(), u_prev.to(self.tdtype).contiguous(), step,
                       F.FD_DENSE)

    def new_field(self) -> torch.Tensor:
        """A zeroed padded field (checkpoint / ring slot) of this grid."""
        n = self.field_bytes // torch.tensor([], dtype=self.tdtype).element_size()
        return torch.zeros(n, dtype=self.tdtype, device=self.device)

    def save_padded(self, cur: torch.Tensor, prev: torch.Tensor) -> int:
        return F.fd_get_state(self.ctx, cur, prev, F.FD_PADDED)

    def load_padded(self, cur: torch.Tensor, prev: torch.Tensor, step: int):
        F.fd_set_state(self.ctx, cur, prev, step, F.FD_PADDED)
