"""MI355X (gfx950) isoAdvector advection step: HIP kernels behind a C interface.

The package holds the kernels and host plan (csrc/), their build (build.py) and a
thin ctypes binding (binding.py).  Input generation lives in the separate
``wavegen`` package and the CPU reference in ``oracle``.
"""
from .binding import (Batch, IsoError, IsoOptions, IsoStepStats, Mesh, Plan, default_options, header_functions, lib)

__all__ = ["Batch", "IsoError", "IsoOptions", "IsoStepStats", "Mesh", "Plan", "default_options", "header_functions", "lib"]
