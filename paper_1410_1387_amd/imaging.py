"""Multi-shot imaging and inversion on top of the adjoint: reverse time migration and
full waveform inversion, the applications Sec. 1 of Medina, St-Cyr and Warburton names
for high-order propagators.

* ``Survey``: shots (source position, receivers) sharing one grid, radius, time step,
  wavelet and checkpoint interval.
* ``forward_traces``: one shot's traces, with the same arithmetic as the forward of
  ``WaveProp`` (same power-of-two source scaling) but no checkpoints.
* ``misfit_and_gradient``: J = sum over shots of 1/2 |traces - observed|^2 and its
  gradient in v, the sum of the per-shot discrete-adjoint gradients.
* ``rtm_image``: the migration of recorded data, I = sum over shots of J_s^T d_s, the
  adjoint of the linearised modelling applied to the data (the back-propagated
  receiver field correlated, at every step, with the Laplacian of the source field,
  i.e. with its second time derivative; the adjoint kernel's imaging condition).
* ``fwi``: steepest descent on J with a backtracking line search, box bounds and an
  optional gradient mask.

Every wave-equation step runs in the library's HIP kernels (through ``WaveProp`` and
``Propagator``); this module only orders calls and sums tensors.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from .autograd import GradientProblem, WaveProp, misfit
from .propagator import Propagator


@dataclasses.dataclass
class Survey:
    r: int
    h: float
    dt: float
    nsteps: int
    shots: List[Tuple[tuple, np.ndarray]]   # (source (x, y[, z]), receivers [nrec, ndim])
    f0: float = 15.0
    t0: Optional[float] = None
    ckpt: int = 50
    dtype: str = "f32"

    def problem(self, i: int) -> GradientProblem:
        src, rec = self.shots[i]
        return GradientProblem(r=self.r, h=self.h, dt=self.dt, nsteps=self.nsteps, source=tuple(src),
                               receivers=np.asarray(rec), f0=self.f0, t0=self.t0, ckpt=self.ckpt, dtype=self.dtype)


def forward_traces(v: torch.Tensor, pb: GradientProblem) -> torch.Tensor:
    """Traces [nsteps, nrec] of one shot (no checkpoints; the arithmetic of WaveProp's forward)."""
    tdt = torch.float32 if pb.dtype == "f32" else torch.float64
    v = v.detach().to(tdt).contiguous()
    T = int(pb.nsteps)
    prop = Propagator(v, pb.r, pb.h, pb.dt, pb.dtype, max_sources=1, max_receivers=len(pb.receivers))
    A = pb.source_amp(v.dim())
    prop.inject(prop.ricker(T, pb.f0, pb.t0), pb.source, amp=A)
    traces = prop.record(pb.receivers, T)
    prop.step(T)
    prop.sync()
    out = traces / A
    prop.close()
    return out


def modelled_data(v: torch.Tensor, survey: Survey) -> List[torch.Tensor]:
    return [forward_traces(v, survey.problem(i)) for i in range(len(survey.shots))]


def misfit_only(v: torch.Tensor, survey: Survey, observed: Sequence[torch.Tensor]) -> float:
    return float(sum(float(misfit(forward_traces(v, survey.problem(i)), observed[i]))
                     for i in range(len(survey.shots))))


def misfit_and_gradient(v: torch.Tensor, survey: Survey, observed: Sequence[torch.Tensor]):
    """(J, dJ/dv) summed over the survey's shots."""
    J = 0.0
    g = None
    for i in range(len(survey.shots)):
        vv = v.detach().clone().requires_grad_(True)
        traces = WaveProp.apply(vv, survey.problem(i))
        Ji = misfit(traces, observed[i])
        Ji.backward()
        J += float(Ji.detach())
        g = vv.grad if g is None else g + vv.grad
    return J, g


def rtm_image(v: torch.Tensor, survey: Survey, data: Sequence[torch.Tensor]) -> torch.Tensor:
    """Migration of the recorded data: sum over shots of J_s^T d_s in the velocity model v
    (d_s without the direct arrival -- e.g. the data minus the data modelled in a smooth
    background -- images the reflectors)."""
    img = None
    for i in range(len(survey.shots)):
        vv = v.detach().clone().requires_grad_(True)
        traces = WaveProp.apply(vv, survey.problem(i))
        (gi,) = torch.autograd.grad(traces, vv, data[i].to(traces.dtype))
        img = gi if img is None else img + gi
    return img


def fwi(v0: torch.Tensor, survey: Survey, observed: Sequence[torch.Tensor], iters: int = 5,
        step: Optional[float] = None, vmin: float = 1000.0, vmax: float = 6000.0, max_halvings: int = 6,
        mask: Optional[torch.Tensor] = None,
        callback: Optional[Callable[[int, float, torch.Tensor], None]] = None):
    """Steepest descent on the multi-shot misfit: direction -(mask g) / max|mask g|, a step
    of `step` m/s (default 1 % of the mean velocity) halved until the misfit decreases and
    grown by 1.5 after a success, velocities clipped to [vmin, vmax].  `mask` (same shape
    as v) weights the gradient, e.g. zero near the sources and receivers, where the
    gradient is largest but least informative (the acquisition footprint).  Returns
    (v, misfit history); stops early when no halving decreases the misfit."""
    v = v0.detach().clone()
    alpha = float(step) if step is not None else 0.01 * float(v.mean())
    J, g = misfit_and_gradient(v, survey, observed)
    hist = [J]
    for it in range(iters):
        if mask is not None:
            g = g * mask.to(g.dtype)
        gmax = float(g.abs().max())
        if not (gmax > 0):
            break
        d = -g / gmax
        accepted = False
        for _ in range(max_halvings + 1):
            trial = torch.clamp(v + alpha * d, vmin, vmax)
            Jt = misfit_only(trial, survey, observed)
            if Jt < J:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            break
        v = trial
        J, g = misfit_and_gradient(v, survey, observed)
        hist.append(J)
        alpha *= 1.5
        if callback is not None:
            callback(it, J, v)
    return v, hist
