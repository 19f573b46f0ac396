"""MI355X-native hyper-power preconditioned Stokes solver (arXiv 2311.06926).

The compute path is ``libhyperpower.so`` (hand-written gfx950 HIP kernels
behind a C ABI, ``include/hyperpower.h``); ``Solver`` is its thin Python
binding and ``autograd`` wraps the solve as a differentiable function.
"""
__all__ = ["Solver", "HyperPowerSolve", "MassMatrix"]


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    if name in ("HyperPowerSolve", "MassMatrix"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
