"""MI355X (gfx950) implementation of one population-dynamics time step of the real-time,
sign-problem-suppressed QMC of Shen & Lidar, arXiv:2502.18929.

``binding`` wraps the C ABI of ``include/qmc.h`` (libqmc.so, HIP kernels in ``csrc/``);
``workloads`` describes the synthetic circuits.  Importing this package loads nothing; the
library is loaded on first use and its absence is an error (there is no CPU fallback).
"""

__all__ = ["binding", "workloads", "build"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
