"""FP64 CPU oracle of the beta-CROWN bound (test infrastructure only).

Imported only by the tests, the smoke check and the benchmark's CPU-baseline
leg.  It shares no code with the GPU library.
"""
from . import batch, beta_crown  # noqa: F401
