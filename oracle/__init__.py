"""FP64 CPU oracle of the field-window estimator.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library.  It shares no code with
the HIP path; the two meet only through the seeded input generators.
"""
from .hermes_oracle import *  # noqa: F401,F403
