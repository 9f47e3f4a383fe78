"""Plain, slow FP64 CPU oracle of the RPA Lanczos-quadrature hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (no kernels, headers, tables or helpers) and does not import it.
"""
from .rpa_oracle import *  # noqa: F401,F403
