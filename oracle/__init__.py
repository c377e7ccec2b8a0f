"""Plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the GPU library.
"""
from .oracle import Oracle, load_library, build_oracle  # noqa: F401
