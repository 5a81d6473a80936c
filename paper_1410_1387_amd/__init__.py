"""MI355X (gfx950) library for explicit high-order finite-difference time stepping of
the acoustic wave equation u_tt = v^2 lap(u) + s(t) delta(x - x_s).

The problem statement (time scheme, star stencil, zero ghost cells, point source,
Ricker forcing) follows Sec. 1 of Medina, St-Cyr and Warburton, "High-Order
Finite-differences on multi-threaded architectures using OCCA".  The computation
runs in hand-written HIP kernels in ``libfdwave.so`` behind the C ABI of
``include/fdwave.h``; this package is a thin ctypes binding plus three small host
layers: ``Propagator`` (one shot), ``WaveProp`` (a torch.autograd.Function for
the velocity gradient) and ``ShotServer`` (continuous batching of shots).
"""

from .fdwave import FdError  # noqa: F401


def __getattr__(name):
    # lazy imports keep ``import paper_1410_1387_amd`` free of torch/GPU work
    if name == "Propagator":
        from .propagator import Propagator

        return Propagator
    if name in ("WaveProp", "GradientProblem"):
        from . import autograd as _ag

        return getattr(_ag, name)
    if name in ("ShotServer", "ShotRequest"):
        from . import serving as _sv

        return getattr(_sv, name)
    raise AttributeError(name)
