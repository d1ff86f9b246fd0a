"""CPU FP64 oracle (test infrastructure).

Plain, slow, obviously correct reference implementations of what the GPU
path computes.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU
path: the only module both sides use is the seeded input generator
(paper_2401_16113_amd.workloads), which holds none of the method's
arithmetic.
"""
from . import cn_oracle  # noqa: F401
