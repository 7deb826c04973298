"""FP64 CPU reference implementation of AccAltProj (test infrastructure).

This package is a checker, not part of the product: only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it. It shares
no code with the GPU library; the two meet only through the seeded inputs.
"""
from .accaltproj import *  # noqa: F401,F403
