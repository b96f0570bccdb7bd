"""Plain FP64 CPU oracle of the isoAdvector step — test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU baseline may use
this package.  It shares no code with the GPU library.
"""
from .oracle import OracleMesh, build, default_opts, tri_integral, tri_wet_fraction

__all__ = ["OracleMesh", "build", "default_opts", "tri_integral", "tri_wet_fraction"]
