"""Continuous batching of forward shots on one GPU.

``ShotServer`` runs a persistent request loop in a worker thread:

* requests are submitted at any time (``submit`` returns a Future);
* the loop admits queued requests in arrival order while their HBM footprint
  (workspace + traces + wavelet, plus the dense velocity model that is on the device
  only while the shot is set up) fits the budget and a batch slot is free; a shot's
  context is created on a separate setup stream, so admission overlaps with the
  batched work already on the GPU;
* the admitted shots -- different grid sizes, same radius and dtype -- that make up
  the stepping window advance together in one stencil launch per time step
  (``fd_batch_step``): every workgroup finds its (shot, tile) in a prefix table and
  every shot keeps its step counter in device memory, so a chunk of an even number
  of steps is a captured HIP graph that is replayed while shots come and go;
* the window is the oldest admitted shots, taken in admission order until their grid
  points per step reach ``fill_points``: enough work to fill the GPU (a small shot
  alone leaves most compute units idle), but no more, so that shots finish in
  roughly arrival order instead of all sharing the GPU at once (which would stretch
  every shot's latency without raising throughput).  The default, 16 M points, is
  about 190 MiB of FP32 fields (u^n, u^(n-1), c): a window of small shots then stays
  within the GPU's 256 MB last-level cache, and a shot of 256^3 or more, which fills
  the GPU by itself, steps alone;
* after each chunk the loop retires shots whose counters reached their step count,
  frees their memory and admits new ones at the next chunk boundary;
* a request whose Future is cancelled before admission is dropped (once admitted it runs
  to completion: its Future is then running and cannot be cancelled).

Each shot's wavefields stay resident in HBM from admission to completion.  Results
are the receiver traces; latency is completion minus arrival.  ``run_sequential``
serves the same requests one at a time (one shot on the GPU at once) for comparison.
"""

from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import math
import queue
import threading
import time
from typing import Any, Callable, Optional

import numpy as np
import torch

from . import fdwave as F


@dataclasses.dataclass
class ShotRequest:
    """One shot: velocity (dense (nz, ny, nx) array, or a callable returning one), step count,
    Ricker source (f0, shift t0 = 1.5/f0 by default) at ``source`` (x, y, z), receivers
    [nrec, 3].  ``arrival`` (s, relative to the start of a trace) is used by ``serve_trace``."""

    rid: int
    velocity: Any
    nsteps: int
    source: tuple
    receivers: np.ndarray
    h: float = 10.0
    courant: float = 0.5
    f0: float = 15.0
    t0: Optional[float] = None
    arrival: float = 0.0
    dt: Optional[float] = None   # explicit time step; default courant * fd_dt_max(max v)
    shape: Optional[tuple] = None  # grid shape; required when velocity is a callable

    def grid_shape(self) -> tuple:
        if int(self.nsteps) < 0:
            raise ValueError(f"nsteps must be >= 0, not {self.nsteps}")
        if self.shape is not None:
            return tuple(self.shape)
        if callable(self.velocity):
            raise ValueError("shape is required when velocity is a callable")
        return tuple(np.shape(self.velocity))


@dataclasses.dataclass
class ShotResult:
    rid: int
    status: str                      # "ok" or "failed"
    traces: Optional[torch.Tensor]   # [nsteps, nrec] on the GPU
    arrival: float
    admitted: float
    completed: float
    points: int                      # grid points x steps
    error: str = ""

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class _Live:
    """A shot resident on the GPU."""

    def __init__(self, req: ShotRequest, ctx: int, tensors: list, traces: torch.Tensor, footprint: int,
                 npoints: int, arrival: float, admitted: float, future: cf.Future, kernel: str = ""):
        self.req, self.ctx, self.tensors, self.traces = req, ctx, tensors, traces
        self.footprint, self.npoints = footprint, npoints
        self.arrival, self.admitted, self.future = arrival, admitted, future
        self.kernel = kernel  # shots batch only with shots of the same stencil kernel


def kernel_of(ctx: int) -> str:
    """The stencil kernel (tile shape) a context steps with: its configuration name without
    the per-shot z chunking and grid size."""
    return F.fd_kernel_config(ctx).split(", zchunk")[0]


def shot_footprint(shape, nsteps: int, nrec: int, r: int, dtype: str) -> int:
    """HBM bytes a shot holds while resident: context workspace (2 wavefields, c, tables),
    traces and wavelet."""
    es = 4 if dtype == "f32" else 8
    return F.fd_workspace_bytes(shape, r, dtype, 1, nrec) + (nsteps * nrec + nsteps) * es


def staging_bytes(shape, dtype: str) -> int:
    """HBM bytes a shot holds only while it is being set up: the dense velocity model on the
    device (read by fd_create into c, then freed).  A velocity callable that returns a device
    tensor in another dtype briefly holds its own copy as well."""
    return int(np.prod(shape)) * (4 if dtype == "f32" else 8)


class _ShotFactory:
    """Creates one shot's context and device buffers on a given stream."""

    def __init__(self, r: int, dtype: str, device):
        self.r, self.dtype, self.device = r, dtype, device
        self.tdt = torch.float32 if dtype == "f32" else torch.float64
        self.npdt = np.float32 if dtype == "f32" else np.float64

    def create(self, req: ShotRequest, stream: torch.cuda.Stream):
        nrec = len(req.receivers)
        sp = F.stream_ptr(stream)
        with torch.cuda.stream(stream):
            vin = req.velocity() if callable(req.velocity) else req.velocity
            if isinstance(vin, torch.Tensor):  # already a device tensor (e.g. built on the GPU)
                v = vin.to(device=self.device, dtype=self.tdt).contiguous()
            else:
                v = torch.from_numpy(np.ascontiguousarray(vin, dtype=self.npdt)).to(self.device)
            shape = tuple(v.shape)
            ws = torch.empty(F.fd_workspace_bytes(shape, self.r, self.dtype, 1, nrec), dtype=torch.uint8,
                             device=self.device)
            wav = torch.empty(req.nsteps, dtype=self.tdt, device=self.device)
            traces = torch.zeros((req.nsteps, nrec), dtype=self.tdt, device=self.device)
        dt = req.dt if req.dt is not None else req.courant * F.fd_dt_max(len(shape), self.r, req.h,
                                                                             float(v.max()))
        ctx = F.fd_create(shape, self.r, req.h, dt, v, self.dtype, "zero", ws, 1, nrec, sp)
        try:
            if req.nsteps > 0:  # a shot of zero steps has no samples and records nothing
                F.fd_ricker(wav, dt, req.f0, 1.5 / req.f0 if req.t0 is None else req.t0, sp)
                F.fd_inject(ctx, wav, req.source, 1.0)
                F.fd_record(ctx, req.receivers, traces, req.nsteps)
            F.fd_sync(ctx)
        except Exception:
            F.fd_destroy(ctx)
            raise
        del v
        footprint = ws.numel() + (wav.numel() + traces.numel()) * traces.element_size()
        return ctx, [ws, wav], traces, footprint, int(np.prod(shape)) * req.nsteps


class ShotServer:
    """Persistent continuous-batching server for same-radius, same-dtype shots.

    budget_bytes  HBM the resident shots may hold together
    max_shots     resident shots (and batch slots)
    chunk         time steps per batched launch sequence (even: replayed as a graph)
    fill_points   grid points per step the stepping window aims for (None: every
                  resident shot steps)
    """

    def __init__(self, r: int = 4, dtype: str = "f32", budget_bytes: int = 64 << 30, max_shots: int = 64,
                 chunk: int = 16, device: str = "cuda", fill_points: Optional[int] = 16_000_000):
        self.r, self.dtype = r, dtype
        self.budget, self.max_shots, self.chunk = int(budget_bytes), int(max_shots), int(chunk)
        self.fill_points = None if fill_points is None else int(fill_points)
        self.device = torch.device(device)
        if self.device.index is None:  # the worker thread needs an explicit device index
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self._factory = _ShotFactory(r, dtype, self.device)
        self._outstanding: set = set()   # futures the loop has taken from the inbox
        self._inbox: "queue.Queue" = queue.Queue()
        self._thread: Optional[threading.Thread] = None
        self._stop = threading.Event()
        self.t0 = time.perf_counter()
        self.stats = {"chunks": 0, "membership_changes": 0, "max_resident_bytes": 0, "max_resident_shots": 0,
                      "max_stepping_shots": 0, "gpu_points": 0, "gpu_busy_s": 0.0, "chunk_points": 0,
                      "admit_s": 0.0, "max_admission_bytes": 0}
        self._error: Optional[BaseException] = None

    # ------------------------------------------------------------------ public API

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def start(self):
        if self._thread is None:
            self.t0 = time.perf_counter()
            self._thread = threading.Thread(target=self._loop_guarded, name="shot-server", daemon=True)
            self._thread.start()
        return self

    def submit(self, req: ShotRequest, arrival: Optional[float] = None) -> cf.Future:
        fut: cf.Future = cf.Future()
        self._inbox.put((req, self.now() if arrival is None else arrival, fut))
        return fut

    def stop(self):
        self._stop.set()
        if self._thread is not None:
            self._thread.join()
            self._thread = None
        if self._error is not None:
            raise self._error

    def serve_trace(self, requests: list, realtime: bool = True) -> list:
        """Submit each request at its arrival time (seconds after start) and wait for all."""
        self.start()
        futs = []
        for req in sorted(requests, key=lambda q: q.arrival):
            if realtime:
                delay = req.arrival - self.now()
                if delay > 0:
                    time.sleep(delay)
            futs.append(self.submit(req, req.arrival if realtime else self.now()))
        for f in futs:
            while not f.done():
                if self._thread is None or not self._thread.is_alive():
                    break
                try:
                    f.result(timeout=0.5)
                except cf.TimeoutError:
                    pass
        self.stop()  # raises the worker's exception, if it died
        return [f.result() for f in futs]

    # ------------------------------------------------------------------ the loop

    def _loop_guarded(self):
        try:
            self._loop()
        except BaseException as e:  # surface to stop(); fail every waiting future
            self._error = e
            pending = list(self._outstanding)
            while True:
                try:
                    pending.append(self._inbox.get_nowait()[2])
                except queue.Empty:
                    break
            for fut in pending:
                try:
                    fut.set_exception(e)
                except cf.InvalidStateError:  # done or cancelled
                    pass

    def _fail(self, req, arrival, fut, err: str):
        now = self.now()
        try:
            fut.set_result(ShotResult(req.rid, "failed", None, arrival, now, now, 0, err))
        except cf.InvalidStateError:  # the caller cancelled it meanwhile
            pass
        self._outstanding.discard(fut)

    def _loop(self):
        torch.cuda.set_device(self.device)
        bstream = torch.cuda.Stream(device=self.device)   # batched chunks
        sstream = torch.cuda.Stream(device=self.device)   # shot setup
        bws = torch.empty(F.fd_batch_workspace_bytes(self.max_shots), dtype=torch.uint8, device=self.device)
        batch = F.fd_batch_create(self.max_shots, bws, F.stream_ptr(bstream))
        pending: collections.deque = collections.deque()
        active: list = []      # resident shots, in admission order
        stepping: list = []    # the window the batch advances
        used = 0
        dirty = False
        inflight: collections.deque = collections.deque()   # (event, [shots finishing in that chunk])
        try:
            while True:
                # drain the inbox; block only when there is nothing else to do
                block = not active and not pending
                while True:
                    try:
                        item = self._inbox.get(timeout=0.005) if block else self._inbox.get_nowait()
                    except queue.Empty:
                        break
                    pending.append(item)
                    self._outstanding.add(item[2])
                    block = False
                if not active and not pending and not inflight:
                    if self._stop.is_set():
                        break
                    continue
                # admit in arrival order while the head fits
                while pending and len(active) < self.max_shots:
                    req, arrival, fut = pending[0]
                    if fut.cancelled():  # cancelled while queued: drop it
                        pending.popleft()
                        self._outstanding.discard(fut)
                        continue
                    try:
                        shape = req.grid_shape()
                        need = shot_footprint(shape, req.nsteps, len(req.receivers), self.r, self.dtype)
                        peak = need + staging_bytes(shape, self.dtype)  # while the model is staged
                    except Exception as e:  # malformed request
                        pending.popleft()
                        self._fail(req, arrival, fut, f"bad request: {e}")
                        continue
                    if peak > self.budget:
                        pending.popleft()
                        self._fail(req, arrival, fut, f"footprint {need} B + {peak - need} B of staged model "
                                                      f"exceeds the budget {self.budget} B")
                        continue
                    if used + peak > self.budget:
                        break  # wait for memory: head-of-line order is kept
                    pending.popleft()
                    if not fut.set_running_or_notify_cancel():  # cancelled just now
                        self._outstanding.discard(fut)
                        continue
                    t_adm = time.perf_counter()
                    try:
                        ctx, tensors, traces, fp, npts = self._factory.create(req, sstream)
                    except Exception as e:  # a bad request fails alone; the others go on
                        self._fail(req, arrival, fut, str(e) if isinstance(e, F.FdError) else
                                   f"{type(e).__name__}: {e}")
                        continue
                    for t in tensors + [traces]:  # written by batched kernels on bstream
                        t.record_stream(bstream)
                    # set-up has finished on sstream (create synchronises it); from now on the
                    # shot runs on the batch stream, so batched steps need no cross-stream
                    # ordering and later set-ups on sstream never wait for a running chunk
                    F.fd_set_stream(ctx, F.stream_ptr(bstream))
                    self.stats["admit_s"] += time.perf_counter() - t_adm
                    self.stats["max_admission_bytes"] = max(self.stats["max_admission_bytes"], used + peak)
                    active.append(_Live(req, ctx, tensors, traces, fp, npts, arrival, self.now(), fut,
                                        kernel_of(ctx)))
                    used += fp
                    dirty = True
                self.stats["max_resident_bytes"] = max(self.stats["max_resident_bytes"], used)
                self.stats["max_resident_shots"] = max(self.stats["max_resident_shots"], len(active))
                if not active and not inflight:
                    continue
                if dirty:
                    want = self._window(active)
                    if [id(s) for s in want] != [id(s) for s in stepping] or any(s.future.done() for s in active):
                        # fd_batch_set waits for the in-flight chunks before rewriting the table
                        self._retire_done(inflight, wait_all=True)
                        keep = [s for s in active if not s.future.done()]
                        for s in active:
                            if s.future.done():
                                used -= s.footprint
                                F.fd_destroy(s.ctx)
                                s.tensors = None
                        active = keep
                        stepping = self._window(active)
                        F.fd_batch_set(batch, [s.ctx for s in stepping], [s.req.nsteps for s in stepping])
                        self.stats["membership_changes"] += 1
                        self.stats["max_stepping_shots"] = max(self.stats["max_stepping_shots"], len(stepping))
                    dirty = False
                    if not stepping:
                        continue
                before = {id(s): F.fd_get_step(s.ctx) for s in stepping}
                ev0 = torch.cuda.Event(enable_timing=True)
                ev0.record(bstream)
                F.fd_batch_step(batch, self.chunk)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(bstream)
                pts = sum((F.fd_get_step(s.ctx) - before[id(s)]) * (s.npoints // max(1, s.req.nsteps))
                          for s in stepping)
                finishing = [s for s in stepping if F.fd_get_step(s.ctx) >= s.req.nsteps and not s.future.done()
                             and not getattr(s, "_queued_done", False)]
                for s in finishing:
                    s._queued_done = True
                    self.stats["gpu_points"] += s.npoints
                inflight.append((ev, finishing, ev0, pts))
                self.stats["chunks"] += 1
                if len(inflight) > 1:
                    if self._retire_done(inflight, wait_all=False):
                        dirty = True
        finally:
            self._retire_done(inflight, wait_all=True)
            for s in active:
                try:
                    s.future.set_exception(RuntimeError("server stopped"))
                except cf.InvalidStateError:  # already completed
                    pass
                F.fd_destroy(s.ctx)
            F.fd_batch_destroy(batch)

    def _window(self, active: list) -> list:
        """The oldest unfinished resident shots, in admission order, that use the oldest
        one's stencil kernel (one launch runs one kernel; the library picks a shot's tile
        shape from its grid), until their grid points per step reach fill_points (at least
        one shot).  The oldest shot always steps, so no shot waits for ever."""
        live = [s for s in active if not s.future.done() and not getattr(s, "_queued_done", False)]
        if not live:
            return []
        live = [s for s in live if s.kernel == live[0].kernel]
        if self.fill_points is None:
            return live
        out, pts = [], 0
        for s in live:
            if out and pts >= self.fill_points:
                break
            out.append(s)
            pts += s.npoints // max(1, s.req.nsteps)
        return out

    def _retire_done(self, inflight, wait_all: bool) -> bool:
        """Complete the shots of finished chunks (all in-flight chunks when wait_all, else all
        but the newest).  Returns True if any shot completed."""
        any_done = False
        while inflight and (wait_all or len(inflight) > 1):
            ev, finishing, ev0, pts = inflight.popleft()
            ev.synchronize()
            now = self.now()
            self.stats["gpu_busy_s"] += ev0.elapsed_time(ev) / 1e3
            self.stats["chunk_points"] += pts
            for s in finishing:
                s.future.set_result(ShotResult(s.req.rid, "ok", s.traces, s.arrival, s.admitted, now, s.npoints))
                self._outstanding.discard(s.future)
                any_done = True
        return any_done


def run_sequential(requests: list, r: int = 4, dtype: str = "f32", realtime: bool = True,
                   device: str = "cuda") -> list:
    """Serve the requests one at a time in arrival order (one shot on the GPU at once,
    fd_step with one launch per step): the baseline the batched server is compared with."""
    dev = torch.device(device)
    factory = _ShotFactory(r, dtype, dev)
    stream = torch.cuda.Stream(device=dev)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    out = []
    for req in sorted(requests, key=lambda q: q.arrival):
        if realtime and req.arrival > now():
            time.sleep(req.arrival - now())
        arrival = req.arrival if realtime else now()
        start = now()
        try:
            req.grid_shape()  # validates the request
            ctx, tensors, traces, fp, npts = factory.create(req, stream)
        except Exception as e:
            msg = str(e) if isinstance(e, F.FdError) else f"{type(e).__name__}: {e}"
            out.append(ShotResult(req.rid, "failed", None, arrival, start, now(), 0, msg))
            continue
        F.fd_set_stream(ctx, F.stream_ptr(stream))
        F.fd_step(ctx, req.nsteps)
        F.fd_sync(ctx)
        out.append(ShotResult(req.rid, "ok", traces, arrival, start, now(), npts))
        F.fd_destroy(ctx)
    return out


def summarize(results: list, makespan: Optional[float] = None) -> dict:
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    pts = sum(r.points for r in ok)
    if makespan is None:
        makespan = max(r.completed for r in ok) - min(r.arrival for r in ok) if ok else 0.0
    return {
        "requests": len(results), "completed": len(ok), "failed": len(results) - len(ok),
        "makespan_s": makespan, "gpts_per_s": pts / makespan / 1e9 if makespan > 0 else 0.0,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()), "point_updates": pts,
    }
