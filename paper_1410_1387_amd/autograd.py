"""Velocity gradient of a shot's receiver traces as a torch.autograd.Function.

Two ways to have the forward states at hand for the adjoint, with bitwise the same
gradient:
  * keep every state (``states="all"``): the forward pass steps with
    ``fd_step_record`` into a new padded field each step (T + 1 fields, e.g. 178 GB for
    256^3 x 2000 steps in FP32 -- HBM that one GPU has), and the backward pass runs the
    adjoint over them with ``fd_adjoint_stored``, without recomputation;
  * checkpoints (``states="checkpoint"``): the forward pass (Propagator) saves the state
    (u^{jK}, u^{jK-1}) in the padded layout every K steps, and for each checkpoint
    segment from the last to the first ``fd_adjoint_segment`` recomputes the segment's
    states into a ring of K - 1 padded fields before the adjoint runs over them.
``states="auto"`` (the default) keeps every state when they take at most three quarters
of the device memory that is free.  The adjoint kernel advances mu = c * lambda (the
discrete adjoint of the leapfrog scheme, discretise-then-differentiate) and accumulates
the imaging term g += mu^k * Lh u^{k-1} in the working precision (FP32 for "f32"), with
``blocked`` summed per segment of K steps and then across segments.  Finally
dJ/dv = 2 g / v.  Every step runs in the library's HIP kernels; this module only
allocates tensors and orders the calls.

Scaling: the forward source is injected with a power-of-two amplitude A (so the
internal wavefield is O(1) instead of O(dt^2 / h^3)) and the residual with a
power-of-two 2^m (so the adjoint field is O(1)); traces are returned divided by A
and the gradient multiplied by 1 / (A 2^m).  All three scalings are exact.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

from . import fdwave as F
from .propagator import Propagator


@dataclasses.dataclass
class GradientProblem:
    """One shot: grid spacing h, time step dt, radius r, nsteps, a Ricker source
    (f0 Hz, shifted by t0 s) at ``source`` = (x, y, z), receivers [nrec, 3] (x, y, z),
    segment length ``ckpt`` (the checkpoint interval, and the blocking of the imaging
    sum), how the forward states are kept (``states``: "auto", "all" or "checkpoint")
    and working dtype."""

    r: int
    h: float
    dt: float
    nsteps: int
    source: tuple
    receivers: np.ndarray
    f0: float = 15.0
    t0: Optional[float] = None
    ckpt: int = 50
    dtype: str = "f32"
    amp_scaling: bool = True
    blocked: bool = False   # sum the imaging term per checkpoint segment, then into g
    states: str = "auto"    # "all": keep every forward state; "checkpoint": recompute segments

    def source_amp(self, ndim: int) -> float:
        """Power of two nearest to h^ndim / dt^2 (makes the injected term O(wavelet))."""
        if not self.amp_scaling:
            return 1.0
        return 2.0 ** round(math.log2(self.h ** ndim / self.dt ** 2))


def _pow2_scale(t: torch.Tensor) -> float:
    """Power of two that brings max|t| to about 1 (1.0 for an all-zero tensor)."""
    m = float(t.abs().max())
    if not (m > 0) or not math.isfinite(m):
        return 1.0
    return 2.0 ** (-math.floor(math.log2(m)))


STATES_MEMORY_SHARE = 0.75


def _available_bytes(device) -> int:
    """Device memory free for new tensors: the driver's free bytes plus what torch's
    allocator holds unused."""
    free, _ = torch.cuda.mem_get_info(device)
    return int(free + torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device))


def keeps_all_states(problem: "GradientProblem", field_bytes: int, device) -> bool:
    """Whether WaveProp keeps every forward state for this problem (T + 1 padded fields)."""
    if problem.states not in ("auto", "all", "checkpoint"):
        raise ValueError(f"states must be 'auto', 'all' or 'checkpoint', not {problem.states!r}")
    if problem.states != "auto":
        return problem.states == "all"
    return (int(problem.nsteps) + 1) * field_bytes <= STATES_MEMORY_SHARE * _available_bytes(device)


class WaveProp(torch.autograd.Function):
    """traces = WaveProp.apply(v, problem): receiver traces [nsteps, nrec] of the shot
    in velocity model v (dense (nz, ny, nx) GPU tensor); differentiable in v."""

    @staticmethod
    def forward(ctx, v: torch.Tensor, problem: GradientProblem):
        pb = problem
        tdt = torch.float32 if pb.dtype == "f32" else torch.float64
        v = v.detach().to(tdt).contiguous()
        ndim = v.dim()
        T, K = int(pb.nsteps), int(pb.ckpt)
        if K < 1:
            raise ValueError("checkpoint interval must be >= 1")
        nrec = len(pb.receivers)
        prop = Propagator(v, pb.r, pb.h, pb.dt, pb.dtype, max_sources=1, max_receivers=nrec)
        A = pb.source_amp(ndim)
        wav = prop.ricker(T, pb.f0, pb.t0)
        prop.inject(wav, pb.source, amp=A)
        traces = prop.record(pb.receivers, T)
        ckpts, fields = [], None
        if keeps_all_states(pb, prop.field_bytes, prop.device):
            # fields[k] = u^k (k < T); fields[T] holds u^{-1} = 0, then takes u^T.  The
            # kernels write every interior point of fields[1 .. T-1] before it is read,
            # so those need only their ghost and padding cells cleared
            n = prop.field_bytes // torch.tensor([], dtype=prop.tdtype).element_size()
            fields = torch.empty((T + 1, n), dtype=prop.tdtype, device=prop.device)
            F.fd_clear_ghosts(prop.ctx, fields, T + 1)  # on the context's stream, the current one
            fields[0].zero_()
            fields[T].zero_()
            prev, cur = fields[T], fields[0]
            for k in range(T):
                out = fields[k + 1] if k + 1 < T else fields[T]
                F.fd_step_record(prop.ctx, cur, prev, out, k)
                prev, cur = cur, out
        else:
            for k0 in range(0, T, K):
                cur, prv = prop.new_field(), prop.new_field()
                prop.save_padded(cur, prv)
                ckpts.append((k0, cur, prv))
                prop.step(min(K, T - k0))
        ctx.prop, ctx.ckpts, ctx.fields, ctx.amp, ctx.T, ctx.K, ctx.blocked = prop, ckpts, fields, A, T, K, pb.blocked
        ctx.save_for_backward(v)
        return traces / A

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        (v,) = ctx.saved_tensors
        prop: Propagator = ctx.prop
        T, K = ctx.T, ctx.K
        resid = grad_traces.detach().to(prop.tdtype).contiguous()
        s = _pow2_scale(resid)
        mu = torch.zeros(2 * prop.new_field().numel(), dtype=prop.tdtype, device=prop.device)
        g = prop.new_field()
        gseg = prop.new_field() if ctx.blocked else None
        if ctx.fields is not None:
            for k0 in reversed(range(0, T, K)):
                F.fd_adjoint_stored(prop.ctx, ctx.fields[k0], k0, min(k0 + K, T), mu, resid, s, g, gseg)
        else:
            ring = None
            if K > 1:
                ring = torch.zeros((K - 1) * prop.new_field().numel(), dtype=prop.tdtype, device=prop.device)
            for k0, cur, prv in reversed(ctx.ckpts):
                k1 = min(k0 + K, T)
                F.fd_adjoint_segment(prop.ctx, cur, prv, k0, k1, ring if k1 - k0 > 1 else None, mu, resid, s, g,
                                     gseg)
        grad_v = torch.empty_like(v)
        F.fd_gradient_finish(prop.ctx, g, v, grad_v, 1.0 / (ctx.amp * s))
        prop.sync()
        ctx.prop = None
        ctx.ckpts = None
        ctx.fields = None
        return grad_v, None


def misfit(traces: torch.Tensor, observed: torch.Tensor) -> torch.Tensor:
    """J = 1/2 sum (traces - observed)^2 (accumulated in FP64)."""
    d = traces.double() - observed.double()
    return 0.5 * (d * d).sum()


def gradient(v: torch.Tensor, problem: GradientProblem, observed: torch.Tensor):
    """(J, dJ/dv) for the L2 trace misfit of one shot."""
    v = v.detach().clone().requires_grad_(True)
    traces = WaveProp.apply(v, problem)
    J = misfit(traces, observed)
    J.backward()
    return float(J.detach()), v.grad
