"""Benchmark: grid-point updates per second of the leapfrog acoustic propagator on
one MI355X, with the stencil kernel's HBM roofline fraction, and the FP64 oracle
timed on the host cores beside it.

One bench step is one whole shot of the 3-D workload: 512^3 grid, h = 10 m,
radius 4 (25-point star), FP32, 8 random layers in [1500, 4500] m/s (seed 0),
Ricker 15 Hz at (256, 256, 16), 1000 time steps, 128 x 128 surface receivers.
A shot runs every row of the forward path on the GPU: model preparation
(c = (v dt / h)^2), Ricker samples, source and receiver registration, and 1000
stencil launches with the source and receivers fused in.  The velocity model is
resident in HBM before the timed region starts.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--no-vti] [--no-gradient] [--no-serving]
                    [--serving-pairs P] [--copy-probe]
    python bench.py --workload 3d_384_r8_noise_fp32      # the other forward workloads (also
    python bench.py --workload 3d_512_r4_layered_fp64    # 3d_512_r4_layered_fp32, the default)
    python bench.py --summarize-prof DIR [--workload W]  # rocprofv3 CSVs -> profiles/ summary

The JSON line also carries the paper's own benchmark kernel, the two-field VTI
propagator (R_xy = 12, R_z = 8) on a 512^3 FP32 grid, under "vti"; the 256^3 velocity
gradient (every forward state kept in HBM, and from checkpoints with recompute) under
"gradient"; and the two
serving traces under "serving", each served three times with continuous batching and
three times one shot at a time, interleaved, with p50/p99 shot latency of the main
trace (sides 128-400) on the top level.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "fwd_r4_512_traffic.json")
KERNEL_SOURCES = ["paper_1410_1387_amd/csrc/fd_stencil.h", "paper_1410_1387_amd/csrc/fd_fwd_f32.hip",
                  "paper_1410_1387_amd/csrc/fd_types.h"]
VTI_PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "vti_r12_8_512_traffic.json")
ADJ_PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "adj_r4_256_traffic.json")
ADJ_KERNEL_SOURCES = ["paper_1410_1387_amd/csrc/fd_stencil.h", "paper_1410_1387_amd/csrc/fd_adj_f32.hip",
                      "paper_1410_1387_amd/csrc/fd_types.h"]
VTI_KERNEL_SOURCES = ["paper_1410_1387_amd/csrc/fd_stencil.h", "paper_1410_1387_amd/csrc/fd_vti.h",
                      "paper_1410_1387_amd/csrc/fd_vti_f32.hip", "paper_1410_1387_amd/csrc/fd_types.h"]
KERNEL_SOURCES_F64 = ["paper_1410_1387_amd/csrc/fd_stencil.h", "paper_1410_1387_amd/csrc/fd_fwd_f64.hip",
                      "paper_1410_1387_amd/csrc/fd_types.h"]
# forward workloads bench.py can time (--workload): name -> (traffic summary, kernel sources);
# the first is the default and the only one the VTI, gradient and serving sections join
FORWARD_WORKLOADS = {
    "3d_512_r4_layered_fp32": (PROFILE_TRAFFIC, KERNEL_SOURCES),
    "3d_384_r8_noise_fp32": (os.path.join(ROOT, "profiles", "fwd_r8_384_traffic.json"), KERNEL_SOURCES),
    "3d_512_r4_layered_fp64": (os.path.join(ROOT, "profiles", "fwd_r4_512_fp64_traffic.json"), KERNEL_SOURCES_F64),
}
DEFAULT_WORKLOAD = "3d_512_r4_layered_fp32"
# the paper's best VTI rates (Mpts/s, FP32, R_xy = 12, R_z = 8), quoted as context only
PAPER_VTI_MPTS = {"K20x, OCCA:OpenCL, 2 pts/thread": 2525.0, "K10 (one chip), OCCA:CUDA, 2 pts/thread": 1579.0,
                  "2x Xeon (16 threads), OCCA:OpenMP": 1548.0}


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path=PROFILE_TRAFFIC, sources=KERNEL_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was taken on
    the kernel source that is built now; otherwise None."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash(sources):
        return None
    return d.get("hbm_bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------- forward shot


def forward_shot(name: str):
    """The forward workload called `name` (see FORWARD_WORKLOADS)."""
    import dataclasses

    import workloads

    if name == "3d_512_r4_layered_fp32":
        return workloads.c2_3d_layered()
    if name == "3d_384_r8_noise_fp32":
        return workloads.c3_3d_noise()
    if name == "3d_512_r4_layered_fp64":
        return dataclasses.replace(workloads.c2_3d_layered(), name=name, dtype="f64")
    raise ValueError(f"unknown workload {name}")


def run_forward(args):
    import numpy as np
    import torch

    from paper_1410_1387_amd import fdwave as F

    shot = forward_shot(args.workload)
    traffic_json, sources = FORWARD_WORKLOADS[args.workload]
    dtype = shot.dtype
    tdt = torch.float32 if dtype == "f32" else torch.float64
    esize = 4 if dtype == "f32" else 8
    nz, ny, nx = shot.shape
    T = shot.nsteps
    v = torch.tensor(shot.velocity(), dtype=tdt, device="cuda")
    vmax = float(v.max())
    dt = shot.courant * F.fd_dt_max(3, shot.r, shot.h, vmax)
    nrec = len(shot.receivers)
    ws = torch.empty(F.fd_workspace_bytes(shot.shape, shot.r, dtype, 1, nrec), dtype=torch.uint8, device="cuda")
    wav = torch.empty(T, dtype=tdt, device="cuda")
    traces = torch.empty((T, nrec), dtype=tdt, device="cuda")
    stream = torch.cuda.current_stream()
    sp = F.stream_ptr(stream)

    def one_shot(ev=None):
        ctx = F.fd_create(shot.shape, shot.r, shot.h, dt, v, dtype, "zero", ws, 1, nrec, sp)
        F.fd_ricker(wav, dt, shot.f0, 1.5 / shot.f0, sp)
        F.fd_inject(ctx, wav, shot.source, 1.0)
        F.fd_record(ctx, shot.receivers, traces, T)
        if ev is not None:
            ev[0].record(stream)
        F.fd_step(ctx, T)
        if ev is not None:
            ev[1].record(stream)
        F.fd_sync(ctx)
        cfg = F.fd_kernel_config(ctx)
        F.fd_destroy(ctx)
        return cfg

    for _ in range(args.warmup):
        one_shot()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        cfg = one_shot(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in events]
    launch_ms = sum(step_ms) / (args.steps * T)  # average stencil launch duration
    pts = nx * ny * nz
    value = pts * T * args.steps / wall / 1e9
    algo_bytes = 4.0 * esize * pts  # read u^n, u^{n-1}, c and write u^{n+1}
    achieved = algo_bytes / (launch_ms * 1e-3) / 1e9
    tr = measured_traffic(traffic_json, sources)
    finite = bool(torch.isfinite(traces).all().item())
    log(f"forward: {value:.1f} Gpts/s per shot incl. setup; stencil {launch_ms * 1e3:.1f} us/launch, "
        f"{achieved:.0f} GB/s algorithmic ({cfg}); traces finite={finite}")
    return {
        "value": value,
        "dtype": dtype,
        "ms_per_step": wall / args.steps * 1e3,
        "config": {
            "workload": shot.name, "grid": [nx, ny, nz], "radius": shot.r, "h_m": shot.h, "dt_s": dt,
            "time_steps_per_shot": T, "velocity": velocity_label(shot),
            "source": list(shot.source), "receivers": nrec, "shots_per_step": 1, "kernel": cfg,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if tr is None else round(tr / (launch_ms * 1e-3) / 1e9, 1),
            "traffic_bytes_per_launch": tr,
            "algorithmic_bytes_per_launch": algo_bytes, "launch_us": round(launch_ms * 1e3, 2),
            "stencil_gpts_per_s": round(pts / (launch_ms * 1e-3) / 1e9, 2),
        },
    }


def velocity_label(shot) -> str:
    a = shot.velocity_args
    if shot.velocity_kind == "layered":
        return f"8 layers U[1500,4500] m/s seed {a.get('seed', 0)}"
    if shot.velocity_kind == "smoothed_noise":
        return f"2500 m/s + smoothed noise (sigma 8 cells, std 300) seed {a.get('seed', 1)}"
    return shot.velocity_kind


def run_vti(args):
    """The paper's own benchmark kernel: the two-field VTI propagator with R_xy = 12 and
    R_z = 8 (Sec. 1), here on a 512^3 FP32 grid with a z spacing stretched from 10 m to
    15 m with depth, layered vz / eps / delta (delta <= eps), Ricker 15 Hz forcing p at
    (256, 256, 16), 1000 steps, 128 x 128 receivers recording p.  The model is resident
    in HBM before the timed region."""
    import numpy as np
    import torch

    import workloads
    from paper_1410_1387_amd import fdwave as F

    shot = workloads.VtiShot()
    T, pts = shot.nsteps, shot.npoints
    vz, eps, delta = (torch.from_numpy(a).cuda() for a in shot.models(np.float32))
    zc = shot.zc()
    dt = shot.courant * F.fd_vti_dt_max(shot.rxy, shot.rz, shot.h, zc, shot.n, float(vz.max()), float(eps.max()),
                                        float(delta.max()))
    rec = shot.receivers()
    ws = torch.empty(F.fd_vti_workspace_bytes(shot.shape, shot.rxy, shot.rz, "f32", 1, len(rec)), dtype=torch.uint8,
                     device="cuda")
    wav = torch.empty(T, dtype=torch.float32, device="cuda")
    traces = torch.empty((T, len(rec)), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    sp = F.stream_ptr(stream)

    def one_shot(ev=None):
        ctx = F.fd_vti_create(shot.shape, shot.rxy, shot.rz, shot.h, zc, dt, vz, eps, delta, "f32", ws, 1, len(rec),
                              sp)
        F.fd_ricker(wav, dt, shot.f0, 1.5 / shot.f0, sp)
        F.fd_vti_inject(ctx, wav, shot.source, 1.0, 0.0)
        F.fd_vti_record(ctx, rec, traces, None, T)
        if ev is not None:
            ev[0].record(stream)
        F.fd_vti_step(ctx, T)
        if ev is not None:
            ev[1].record(stream)
        F.fd_vti_sync(ctx)
        cfg = F.fd_vti_kernel_config(ctx)
        F.fd_vti_destroy(ctx)
        return cfg

    one_shot()
    torch.cuda.synchronize()
    nshots = max(1, min(args.steps, 2))
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nshots)]
    t0 = time.perf_counter()
    for k in range(nshots):
        cfg = one_shot(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = sum(a.elapsed_time(b) for a, b in events) / (nshots * T)
    algo = 36.0 * pts  # read p, q at n and n-1 and ax, an, az; write p, q at n+1 (FP32)
    achieved = algo / (launch_ms * 1e-3) / 1e9
    rate = pts / (launch_ms * 1e-3) / 1e9
    tr = measured_traffic(VTI_PROFILE_TRAFFIC, VTI_KERNEL_SOURCES)
    log(f"vti: stencil {launch_ms * 1e3:.1f} us/launch = {rate:.1f} Gpts/s, {achieved:.0f} GB/s algorithmic ({cfg})")
    return {
        "workload": "vti_512_rxy12_rz8_stretched_z_fp32", "gpts_per_s_per_shot": round(pts * T * nshots / wall / 1e9, 2),
        "stencil_gpts_per_s": round(rate, 2), "launch_us": round(launch_ms * 1e3, 2),
        "grid": list(shot.shape[::-1]), "rxy": shot.rxy, "rz": shot.rz, "time_steps_per_shot": T,
        "z_spacing_m": [10.0, 15.0], "kernel": cfg,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if tr is None else round(tr / (launch_ms * 1e-3) / 1e9, 1),
                     "algorithmic_bytes_per_launch": algo},
        "paper_context_mpts": PAPER_VTI_MPTS,
        "ratio_to_paper_best_gpu": round(rate * 1e3 / PAPER_VTI_MPTS["K20x, OCCA:OpenCL, 2 pts/thread"], 1),
    }


def run_copy_probe(nbytes=1 << 30, reps=3):
    """A plain device copy of known size: the reference that hardware byte counters are
    scaled by (what FETCH_SIZE / WRITE_SIZE report for exactly nbytes read and written)."""
    import torch

    from paper_1410_1387_amd import fdwave as F

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        F.fd_copy_probe(b, a, nbytes, F.stream_ptr())
    torch.cuda.synchronize()
    del a, b


def run_stream_probe(nbytes=512 << 20, reps=20, blocks=(512, 768, 1024)):
    """What HBM delivers for the forward update's stream mix (three reads and one in-place
    write of nbytes each, 16-byte vectors, grid-stride) with no halo and no arithmetic:
    the best of a few launch sizes, in GB/s, from HIP events on the launch stream."""
    import torch

    from paper_1410_1387_amd import fdwave as F

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    stream = torch.cuda.current_stream()
    sp = F.stream_ptr(stream)
    best = 0.0
    for nb in blocks:
        for _ in range(3):
            F.fd_stream_probe(a, b, c, nbytes, nb, sp)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            F.fd_stream_probe(a, b, c, nbytes, nb, sp)
        e1.record(stream)
        e1.synchronize()
        best = max(best, 4.0 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9)
    del a, b, c
    log(f"stream probe (3 reads + 1 in-place write, {nbytes >> 20} MiB each): {best:.0f} GB/s")
    return best


def summarize_prof(d: str, workload: str = DEFAULT_WORKLOAD):
    """Reduce a rocprofv3 directory (trace/, fetch/, write/ subdirectories of CSV output) to
    per-launch HBM bytes of the stencil kernels, scaled by the copy-probe factors.  For the
    default workload: the forward, VTI and adjoint kernels; otherwise that workload's
    forward kernel."""
    import csv
    import glob

    import numpy as np

    def rows(pattern):
        out = []
        for f in glob.glob(os.path.join(d, pattern)):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    first_dispatch = {}

    def counter(pattern, name):
        """Counter value per kernel name, per dispatch (in dispatch order)."""
        vals = {}
        for r in rows(pattern):
            if r["Counter_Name"] == name:
                vals.setdefault(r["Kernel_Name"], []).append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        for k, v in vals.items():
            first_dispatch[k] = min(first_dispatch.get(k, 1 << 62), min(d for d, _ in v))
        return {k: [x for _, x in sorted(v)] for k, v in vals.items()}

    durations = {}
    for r in rows("trace/*kernel_trace.csv"):
        durations.setdefault(r["Kernel_Name"], []).append(
            (int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durations = {k: [x for _, x in sorted(v)] for k, v in durations.items()}

    def mean(xs):
        return sum(xs) / len(xs)

    fetch = counter("fetch/*counter_collection.csv", "FETCH_SIZE")
    write = counter("write/*counter_collection.csv", "WRITE_SIZE")
    copy = [k for k in fetch if "copy_probe" in k][0]
    probe_bytes = 1 << 30
    f_scale = probe_bytes / (mean(fetch[copy]) * 1024.0)
    w_scale = probe_bytes / (mean(write[copy]) * 1024.0)
    bench_args = ("--steps 1 --warmup 0 --no-cpu --no-serving --copy-probe" if workload == DEFAULT_WORKLOAD else
                  f"--workload {workload} --steps 1 --warmup 0 --no-cpu --no-vti --copy-probe")
    cmds = [
        f"rocprofv3 --kernel-trace --stats -d DIR/trace -o trace --output-format csv -- python3 bench.py {bench_args}",
        f"rocprofv3 --pmc FETCH_SIZE -d DIR/fetch -o fetch --output-format csv -- python3 bench.py {bench_args}",
        f"rocprofv3 --pmc WRITE_SIZE -d DIR/write -o write --output-format csv -- python3 bench.py {bench_args}",
    ]
    # (kernel, summary file, sources, algorithmic bytes, dispatches that belong to the
    # measurement: the forward shot runs first, so its launches are the forward kernel's
    # first T (the gradient section launches the same kernel at 256^3 afterwards); the
    # isolated adjoint launches that the bench times come last)
    iso = ADJ_ISOLATED_WARMUP + ADJ_ISOLATED_REPS
    shot = forward_shot(workload)
    fwd_json, fwd_sources = FORWARD_WORKLOADS[workload]
    esize = 4 if shot.dtype == "f32" else 8
    sections = [("fwd_kernel", fwd_json, fwd_sources, 4.0 * esize * int(np.prod(shot.shape)), slice(0, shot.nsteps),
                 "first")]
    if workload == DEFAULT_WORKLOAD:
        sections += [("vti_kernel", VTI_PROFILE_TRAFFIC, VTI_KERNEL_SOURCES, 36.0 * 512 ** 3, slice(0, None), "most"),
                     ("adj_kernel", ADJ_PROFILE_TRAFFIC, ADJ_KERNEL_SOURCES, 28.0 * 256 ** 3, slice(-iso, None),
                      "most")]
    for tag, out_path, sources, algo, sel, pick in sections:
        cands = [k for k in fetch if tag in k]
        if not cands:
            continue
        # the forward shot runs first: its kernel is the first forward kernel dispatched
        # (the gradient section may step its 256^3 grid with another build of the tile);
        # the other sections take the kernel with the most dispatches
        kern = (min(cands, key=lambda k: first_dispatch[k]) if pick == "first"
                else max(cands, key=lambda k: len(fetch[k])))
        avg_ns = mean(durations[kern][sel]) if kern in durations else None
        fb, wb = mean(fetch[kern][sel]) * 1024.0 * f_scale, mean(write[kern][sel]) * 1024.0 * w_scale
        res = {
            "kernel": kern, "kernel_hash": kernel_hash(sources), "dispatches": len(fetch[kern][sel]),
            "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb,
            "algorithmic_bytes_per_launch": algo,
            "fetch_scale": f_scale, "write_scale": w_scale, "copy_probe_bytes": probe_bytes,
            "trace_avg_launch_ns": avg_ns, "commands": cmds,
        }
        with open(out_path, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res, indent=1))


# --------------------------------------------------------------------------- CPU baseline


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# the oracle in a child process with its own OpenMP thread count (the oracle reads
# OMP_NUM_THREADS when its library loads): a 1-step and a (1 + nsteps)-step call, whose
# difference is the cost of nsteps steps without the per-call set-up; prints
# {"pts_per_s": ..., "steps": nsteps, "s": seconds of those steps}
_ORACLE_CHILD = """
import json, sys, time
import numpy as np
sys.path.insert(0, {root!r})
import bench, oracle
shot = bench.forward_shot({workload!r})
v = shot.velocity()
dt = shot.courant * oracle.dt_max(3, shot.r, shot.h, v.max())
u0 = np.random.default_rng(0).standard_normal(shot.shape)
el = []
for n in (1, 1 + {nsteps}):
    t = time.perf_counter()
    oracle.forward(v, shot.h, dt, shot.r, n, [(shot.source, oracle.ricker(n, dt))], shot.receivers, u0=u0, um1=u0)
    el.append(time.perf_counter() - t)
per = (el[1] - el[0]) / {nsteps}
print(json.dumps({{"pts_per_s": float(np.prod(shot.shape)) / per, "steps": {nsteps}, "s": el[1] - el[0]}}))
"""


def _oracle_one_thread(workload: str, nsteps: int):
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = _ORACLE_CHILD.format(root=ROOT, workload=workload, nsteps=nsteps)
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if res.returncode != 0:
        log(f"cpu baseline (1 thread) failed: {res.stderr[-400:]}")
        return None
    return json.loads(res.stdout.strip().splitlines()[-1])


def run_cpu_baseline(workload: str = DEFAULT_WORKLOAD, budget_s: float = 12.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload: the
    full grid and velocity model, a few time steps (throughput per step is constant);
    then the same on one thread (one step), in a child process."""
    import numpy as np

    import oracle

    oracle._lib()
    shot = forward_shot(workload)
    v = shot.velocity()
    dt = shot.courant * oracle.dt_max(3, shot.r, shot.h, v.max())
    # OpenMP threads the oracle runs with: OMP_NUM_THREADS if set, else one per usable core
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(shot.shape)
    # per-step cost from a 1-step and a 3-step call (each call also pays a fixed set-up)
    tk = []
    for k in (1, 3):
        t = time.perf_counter()
        oracle.forward(v, shot.h, dt, shot.r, k, [(shot.source, oracle.ricker(k, dt))], u0=u0, um1=u0)
        tk.append(time.perf_counter() - t)
    per = max((tk[1] - tk[0]) / 2, 1e-3)
    nsteps = max(2, min(400, int((budget_s - max(tk[0] - per, 0.0)) / per)))
    t = time.perf_counter()
    oracle.forward(v, shot.h, dt, shot.r, nsteps, [(shot.source, oracle.ricker(nsteps, dt))], shot.receivers,
                   u0=u0, um1=u0)
    el = time.perf_counter() - t
    pts = int(np.prod(shot.shape))
    val = pts * nsteps / el / 1e9
    grid = "x".join(str(n) for n in shot.shape[::-1])
    model = cpu_model()
    log(f"cpu baseline: {val:.3f} Gpts/s ({nsteps} steps of {grid} FP64 in {el:.1f} s, {cores} threads, {model})")
    one = _oracle_one_thread(workload, 1)
    if one is not None:
        log(f"cpu baseline, 1 thread: {one['pts_per_s'] / 1e9:.4f} Gpts/s ({one['steps']} step in {one['s']:.1f} s)")
    return {"value": round(val, 4), "unit": "Gpts/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_cpus_visible": os.cpu_count(),
            "one_thread": None if one is None else {"value": round(one["pts_per_s"] / 1e9, 5), "unit": "Gpts/s",
                                                    "steps": one["steps"], "wall_s": round(one["s"], 2)},
            "sample": f"FP64 oracle, full {grid} grid of the same workload ({velocity_label(shot)}), r={shot.r}, "
                      f"{nsteps} time steps ({el:.1f} s wall) on {cores} threads; the one-thread figure is the "
                      f"difference of a 2-step and a 1-step run of the same grid in a child process with "
                      f"OMP_NUM_THREADS=1"}


def run_gradient():
    """The velocity-gradient workload: 256^3, r = 4, FP32, 2000 steps, true model = layers +
    3 Gaussian anomalies, start model = layers, 128 x 128 surface receivers, L2 misfit.
    Times one FP32 gradient after a warm-up, twice: keeping every forward state in HBM
    (when they fit: 2001 padded fields, 178 GB; the adjoint then needs no recompute) and
    from checkpoints every 50 steps with recomputed segments (bitwise the same gradient);
    observed data from an FP32 forward in the true model."""
    import torch

    import workloads
    from paper_1410_1387_amd import Propagator
    from paper_1410_1387_amd import fdwave as F
    from paper_1410_1387_amd.autograd import GradientProblem, WaveProp, keeps_all_states, misfit

    case = workloads.GradientCase()
    v_true, v0 = case.models()
    dt = case.courant * F.fd_dt_max(3, case.r, case.h, float(max(v_true.max(), v0.max())))
    rec = case.receivers()
    p = Propagator(torch.tensor(v_true, dtype=torch.float32, device="cuda"), case.r, case.h, dt, "f32",
                   max_sources=1, max_receivers=len(rec))
    p.inject(p.ricker(case.nsteps, case.f0), case.source)
    obs = p.record(rec, case.nsteps)
    p.step(case.nsteps)
    p.sync()
    obs = obs.clone()
    p.close()
    pb = GradientProblem(r=case.r, h=case.h, dt=dt, nsteps=case.nsteps, source=case.source, receivers=rec,
                         f0=case.f0, ckpt=case.ckpt, dtype="f32", states="auto")
    v0t = torch.tensor(v0, dtype=torch.float32, device="cuda")

    def once():
        v = v0t.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = WaveProp.apply(v, pb)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J = misfit(tr, obs)
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, float(J.detach()), v.grad

    # keep every forward state when they fit (decided once, then fixed for both runs)
    fb = F.fd_field_bytes((case.n,) * 3, case.r, "f32")
    kept = keeps_all_states(pb, fb, v0t.device)
    pb.states = "all" if kept else "checkpoint"
    once()
    tf, tb, J, g = once()
    n3 = case.n ** 3
    finite = bool(torch.isfinite(g).all().item())
    log(f"gradient ({'every state kept' if kept else 'checkpoints'}): forward {tf:.3f} s, backward {tb:.3f} s, "
        f"J {J:.4e}, finite={finite}")
    del g
    pb.states = "checkpoint"
    once()
    tfc, tbc, Jc, gc = once()
    log(f"gradient (checkpoints every {case.ckpt} steps): forward {tfc:.3f} s, backward {tbc:.3f} s, "
        f"J {Jc:.4e}, same misfit: {Jc == J}")
    del gc
    torch.cuda.empty_cache()
    adj_ms = time_adjoint_kernel(v0t, case, dt, rec)
    algo = 28.0 * n3
    achieved = algo / (adj_ms * 1e-3) / 1e9
    tr = measured_traffic(ADJ_PROFILE_TRAFFIC, ADJ_KERNEL_SOURCES)
    log(f"adjoint kernel: {adj_ms * 1e3:.1f} us/launch, {achieved:.0f} GB/s algorithmic")
    return {
        "workload": f"gradient_{case.n}_r{case.r}_fp32_{case.nsteps}steps",
        "states": ("every forward state kept in HBM (no recompute)" if kept
                   else f"checkpoints every {case.ckpt} steps (recompute)"),
        "states_gb": round((case.nsteps + 1) * fb / 1e9, 1) if kept else None,
        "gradient_s": round(tf + tb, 4), "forward_s": round(tf, 4), "backward_s": round(tb, 4),
        "gpts_per_s": round(n3 * case.nsteps / (tf + tb) / 1e9, 2),
        "unit": "grid points x time steps per second of a full gradient (forward + adjoint)",
        "backward_step_us": round(tb / case.nsteps * 1e6, 1), "misfit": J, "finite": finite,
        "receivers": len(rec),
        "checkpointed": {"ckpt": case.ckpt, "gradient_s": round(tfc + tbc, 4), "forward_s": round(tfc, 4),
                         "backward_s": round(tbc, 4), "backward_step_us": round(tbc / case.nsteps * 1e6, 1),
                         "same_misfit": Jc == J},
        "adjoint_kernel_roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if tr is None else round(tr / (adj_ms * 1e-3) / 1e9, 1),
            "algorithmic_bytes_per_launch": algo, "launch_us": round(adj_ms * 1e3, 2),
        },
    }


ADJ_ISOLATED_WARMUP, ADJ_ISOLATED_REPS = 5, 200


def time_adjoint_kernel(v, case, dt, rec, reps=ADJ_ISOLATED_REPS, nrot=8):
    """Average duration of one adjoint-kernel launch at the gradient workload's size (read
    mu^{k+1}, mu^{k+2}, c, u^{k-1}, g; write mu^k, g: 28 B/pt): one-step segments need no
    recompute, so each fd_adjoint_segment call is exactly one adjoint launch.  u^{k-1}
    comes from `nrot` different fields in turn, as in the backward pass (where it is a new
    ring slot every step): one field read again and again would be served by the
    last-level cache and time the kernel faster than it runs in a gradient."""
    import torch

    from paper_1410_1387_amd import Propagator
    from paper_1410_1387_amd import fdwave as F

    p = Propagator(v, case.r, case.h, dt, "f32", max_sources=1, max_receivers=len(rec))
    p.inject(p.ricker(case.nsteps, case.f0), case.source)
    p.record(rec, case.nsteps)
    fb = p.field_bytes
    z = lambda nbytes: torch.zeros(nbytes // 4, dtype=torch.float32, device=v.device)  # noqa: E731
    u_curs, u_prev, mu, g = [z(fb) for _ in range(nrot)], z(fb), z(2 * fb), z(fb)
    resid = torch.zeros((case.nsteps, len(rec)), dtype=torch.float32, device=v.device)
    stream = torch.cuda.current_stream()
    for k in range(ADJ_ISOLATED_WARMUP):
        F.fd_adjoint_segment(p.ctx, u_curs[k % nrot], u_prev, k, k + 1, None, mu, resid, 1.0, g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(reps):
        F.fd_adjoint_segment(p.ctx, u_curs[k % nrot], u_prev, k + 1, k + 2, None, mu, resid, 1.0, g)
    e1.record(stream)
    p.sync()
    ms = e0.elapsed_time(e1) / reps
    p.close()
    return ms


SERVING_SIDES = (128, 192, 256, 320, 400)
SMALL_SIDES = (64, 96, 128, 160)


def serving_requests(nreq=256, rate=20.0, sides=SERVING_SIDES):
    """A serving trace: Poisson arrivals at ``rate`` req/s (20 for the main trace), cubic
    sides uniform over ``sides`` ({128, 192, 256, 320, 400}), 500-2000 steps, r = 4, FP32,
    layered velocity per request seed.  The layered model is expanded on the GPU from its
    depth profile."""
    import torch

    import workloads
    from paper_1410_1387_amd import fdwave as F
    from paper_1410_1387_amd.serving import ShotRequest

    reqs = []
    for q in workloads.serving_trace(nreq, rate=rate, sides=sides):
        prof = q.profile().astype("float32")
        dt = 0.5 * F.fd_dt_max(3, 4, 10.0, float(prof.max()))

        def make(prof=prof, n=q.n):
            col = torch.tensor(prof, device="cuda").view(n, 1, 1)
            return col.expand(n, n, n).contiguous()

        reqs.append(ShotRequest(rid=q.rid, velocity=make, shape=q.shape, nsteps=q.nsteps, source=q.source,
                                receivers=q.receivers(), arrival=q.arrival, dt=dt))
    return reqs


def _serving_stats(srv, res, wall, budget_gib):
    from paper_1410_1387_amd.serving import summarize

    st = summarize(res)
    st.update({"wall_s": round(wall, 2), "budget_gib": budget_gib, "chunk_steps": 16,
               "max_resident_shots": srv.stats["max_resident_shots"], "fill_points": srv.fill_points,
               "max_stepping_shots": srv.stats["max_stepping_shots"],
               "max_resident_gib": round(srv.stats["max_resident_bytes"] / 2 ** 30, 2),
               "batched_chunks": srv.stats["chunks"], "membership_changes": srv.stats["membership_changes"],
               "gpu_busy_s": round(srv.stats["gpu_busy_s"], 2), "host_admission_s": round(srv.stats["admit_s"], 2),
               "gpts_per_s_while_busy": round(srv.stats["chunk_points"] / max(srv.stats["gpu_busy_s"], 1e-9) / 1e9, 1)})
    return st


def _median(xs):
    ys = sorted(xs)
    n = len(ys)
    return ys[n // 2] if n % 2 else 0.5 * (ys[n // 2 - 1] + ys[n // 2])


def serve_both(reqs, budget_gib, label, pairs=3):
    """One trace served `pairs` times with continuous batching (A) and `pairs` times one shot
    at a time (B) on the same GPU, interleaved A B B A A B ... so that drift of the box's
    clocks and temperature falls on both modes alike.  Reports every run, the median of each
    mode and the per-pair throughput ratios A / B (median, min, max)."""
    from paper_1410_1387_amd.serving import ShotServer, run_sequential, summarize

    runs = {"batched": [], "one_at_a_time": []}
    order = []
    for k in range(pairs):
        order += ["batched", "one_at_a_time"] if k % 2 == 0 else ["one_at_a_time", "batched"]
    for mode in order:
        if mode == "batched":
            srv = ShotServer(r=4, dtype="f32", budget_bytes=budget_gib << 30, max_shots=64, chunk=16)
            t0 = time.perf_counter()
            res = srv.serve_trace(reqs)
            st = _serving_stats(srv, res, time.perf_counter() - t0, budget_gib)
        else:
            st = summarize(run_sequential(reqs))
        runs[mode].append(st)
        log(f"serving {label} ({mode.replace('_', ' ')}, run {len(runs[mode])}): {st['gpts_per_s']:.1f} Gpts/s, "
            f"makespan {st['makespan_s']:.2f} s, p50 {st['p50_latency_s']:.2f} s, p99 {st['p99_latency_s']:.2f} s")
    ratios = [a["gpts_per_s"] / b["gpts_per_s"] for a, b in zip(runs["batched"], runs["one_at_a_time"])
              if b["gpts_per_s"] > 0]
    out = {"pairs": pairs, "order": order, "runs": runs}
    for mode, rs in runs.items():
        out[mode] = {key: round(_median([r[key] for r in rs]), 4)
                     for key in ("gpts_per_s", "p50_latency_s", "p99_latency_s", "makespan_s")}
        out[mode]["completed"] = min(r["completed"] for r in rs)
        out[mode]["requests"] = rs[0]["requests"]
    out["throughput_ratio"] = {"median": round(_median(ratios), 4), "min": round(min(ratios), 4),
                               "max": round(max(ratios), 4), "per_pair": [round(x, 4) for x in ratios]}
    log(f"serving {label}: batched / one at a time = {out['throughput_ratio']['median']:.3f} "
        f"(pairs {', '.join(f'{x:.3f}' for x in ratios)})")
    return out


def run_serving(nreq=256, budget_gib=96, pairs=3):
    """The serving trace (sides 128-400 at 20 req/s), and a trace of small shots (sides
    64-160, arriving at 400 req/s so that the GPU, not the arrivals, sets the pace), each
    served with continuous batching and one shot at a time in interleaved pairs."""
    out = {"workload": f"serving_{nreq}req_poisson20_sides128-400_r4_fp32"}
    out.update(serve_both(serving_requests(nreq), budget_gib, "sides 128-400", pairs))
    small = {"workload": f"serving_{nreq}req_poisson400_sides64-160_r4_fp32"}
    small.update(serve_both(serving_requests(nreq, rate=400.0, sides=SMALL_SIDES), budget_gib, "sides 64-160",
                            pairs))
    out["small_shots"] = small
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed shots (each a whole shot of the workload)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-gradient", action="store_true", help="skip the adjoint gradient workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the shot-serving workload")
    ap.add_argument("--serving-pairs", type=int, default=3,
                    help="interleaved (batched, one-at-a-time) runs of each serving trace")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB copy (counter scaling reference)")
    ap.add_argument("--no-vti", action="store_true", help="skip the VTI propagator section")
    ap.add_argument("--summarize-prof", metavar="DIR", help="summarize rocprofv3 CSV output and exit")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(FORWARD_WORKLOADS),
                    help="forward workload to time (the VTI, gradient and serving sections run only with "
                         "the default)")
    args = ap.parse_args()
    if args.summarize_prof:
        summarize_prof(args.summarize_prof, args.workload)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described but not built)"}))
        sys.exit(2)

    import torch

    from paper_1410_1387_amd import fdwave as F

    F.lib()  # the HIP library must be present: no fallback
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_probe:
        run_copy_probe()
    fw = run_forward(args)
    stream_gbs = run_stream_probe()
    fw["roofline"]["stream_probe_gbs"] = round(stream_gbs, 1)
    fw["roofline"]["frac_of_stream_probe"] = round(fw["roofline"]["achieved"] / stream_gbs, 4)
    out = {
        "metric": "grid-point updates/s (Gpts/s), % of HBM roofline; p50/p99 shot latency",
        "value": round(fw["value"], 2),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fw["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": fw["dtype"],
        "data": "synthetic",
        "config": fw["config"],
        "roofline": fw["roofline"],
    }
    default = args.workload == DEFAULT_WORKLOAD
    if default and not args.no_vti:
        out["vti"] = run_vti(args)
    if default and not args.no_gradient:
        out["gradient"] = run_gradient()
    if default and not args.no_serving:
        sv = run_serving(pairs=max(1, args.serving_pairs))
        out["serving"] = sv
        # the metric's latency half: the main serving trace, continuous batching, median run
        out["p50_latency_s"] = sv["batched"]["p50_latency_s"]
        out["p99_latency_s"] = sv["batched"]["p99_latency_s"]
        out["serving_vs_one_at_a_time"] = sv["throughput_ratio"]["median"]
    out["cpu_baseline"] = None if args.no_cpu else run_cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
