"""Float64 CPU oracle for the GFC solve. Test infrastructure only: imported by tests,
the smoke check and the benchmark's CPU-baseline leg, never by the product path."""
from .gfc_oracle import *  # noqa: F401,F403
