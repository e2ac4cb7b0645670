"""FP64 CPU reference for motion-blur rasterization (test infrastructure only).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU path never does.
"""
from .oracle import COUNTER_NAMES, render, keyframes, fast_coeffs, closest_point, schedule, Decisions  # noqa: F401
