"""VtiPropagator: one shot of the two-field VTI propagator on the GPU.

The pseudo-acoustic VTI equations of Sec. 1 of Medina, St-Cyr and Warburton
(eqs. (p) and (q)): p and the auxiliary field q, the symmetric radius-rxy xy stencil
acting on p, a per-plane (2rz+1)-point z stencil acting on q (variable z spacing
absorbed in its weights), stepped with the centred second-order time scheme.  A thin
object over the C ABI: torch owns the device memory, libfdwave.so does the arithmetic.
"""

from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import fdwave as F

_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64}


class VtiPropagator:
    """vz, eps, delta  dense (nz, ny, nx) GPU tensors (or eps/delta as floats)
    rxy, rz          xy and z stencil radii (rxy in {2,4,8,12}, rz in {1,2,4,8}, rz <= rxy)
    h                xy spacing (m); zc: plane coordinates -rz .. nz+rz-1 (default: spacing h)
    dt               time step (s); must satisfy the limit checked by fd_vti_create
    """

    def __init__(self, vz: torch.Tensor, eps, delta, rxy: int, rz: int, h: float, dt: float,
                 zc: Optional[Sequence[float]] = None, dtype: str = "f32", max_sources: int = 1,
                 max_receivers: int = 0, stream: Optional[torch.cuda.Stream] = None):
        if not vz.is_cuda:
            raise ValueError("vz must be a GPU tensor")
        self.dtype = dtype
        self.tdtype = _TORCH_DTYPE[dtype]
        self.shape = tuple(vz.shape)
        self.rxy, self.rz, self.h, self.dt = int(rxy), int(rz), float(h), float(dt)
        self.zc = None if zc is None else np.asarray(zc, dtype=np.float64)
        self.device = vz.device
        self._stream = stream
        vz = vz.to(self.tdtype).contiguous()

        def field(a):
            if isinstance(a, torch.Tensor):
                return a.to(device=self.device, dtype=self.tdtype).contiguous()
            return torch.full(self.shape, float(a), dtype=self.tdtype, device=self.device)

        eps, delta = field(eps), field(delta)
        nbytes = F.fd_vti_workspace_bytes(self.shape, rxy, rz, dtype, max_sources, max_receivers)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._wavelets = []
        self.traces_p: Optional[torch.Tensor] = None
        self.traces_q: Optional[torch.Tensor] = None
        self.ctx = F.fd_vti_create(self.shape, rxy, rz, h, self.zc, dt, vz, eps, delta, dtype, self.workspace,
                                   max_sources, max_receivers, self.stream_handle())

    @staticmethod
    def dt_max(rxy: int, rz: int, h: float, nz: int, vz_max: float, eps_max: float, delta_max: float,
               zc=None) -> float:
        return F.fd_vti_dt_max(rxy, rz, h, zc, nz, vz_max, eps_max, delta_max)

    def stream_handle(self):
        return F.stream_ptr(self._stream)

    @property
    def kernel_config(self) -> str:
        return F.fd_vti_kernel_config(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            F.fd_vti_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ricker(self, nsamp: int, f0: float = 15.0, t0: Optional[float] = None) -> torch.Tensor:
        """Ricker samples at t = n dt - t0 computed on the device (t0 defaults to 1.5 / f0)."""
        t0 = 1.5 / f0 if t0 is None else t0
        out = torch.empty(nsamp, dtype=self.tdtype, device=self.device)
        F.fd_ricker(out, self.dt, f0, t0, self.stream_handle())
        return out

    def inject(self, wavelet: torch.Tensor, pos: Sequence[int], amp_p: float = 1.0, amp_q: float = 0.0):
        """Point source at (x, y, z); eq. (p) of Sec. 1 forces p only (amp_q = 0)."""
        w = wavelet.to(device=self.device, dtype=self.tdtype).contiguous()
        self._wavelets.append(w)
        F.fd_vti_inject(self.ctx, w, pos, amp_p, amp_q)

    def record(self, positions, nsteps: int, record_q: bool = False):
        """Receivers at (x, y, z) rows of `positions`; returns the [nsteps, nrec] trace tensor
        of p (and of q when record_q), filled as the steps run."""
        n = len(positions)
        self.traces_p = torch.zeros((nsteps, n), dtype=self.tdtype, device=self.device)
        self.traces_q = torch.zeros((nsteps, n), dtype=self.tdtype, device=self.device) if record_q else None
        F.fd_vti_record(self.ctx, positions, self.traces_p, self.traces_q, nsteps)
        return (self.traces_p, self.traces_q) if record_q else self.traces_p

    def step(self, nsteps: int):
        F.fd_vti_step(self.ctx, nsteps)

    def sync(self):
        F.fd_vti_sync(self.ctx)

    @property
    def step_index(self) -> int:
        return F.fd_vti_get_step(self.ctx)

    def state(self):
        """(p^n, p^{n-1}, q^n, q^{n-1}) as new dense tensors."""
        out = [torch.empty(self.shape, dtype=self.tdtype, device=self.device) for _ in range(4)]
        F.fd_vti_get_state(self.ctx, *out)
        self.sync()
        return tuple(out)

    def set_state(self, p, p_prev, q, q_prev, step: int = 0):
        args = [a.to(device=self.device, dtype=self.tdtype).contiguous() for a in (p, p_prev, q, q_prev)]
        F.fd_vti_set_state(self.ctx, *args, step)
        self.sync()
