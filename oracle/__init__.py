"""FP64 CPU oracle for FFT beamforming -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never calls it and shares no code
with it.  See ``oracle.fftbf_oracle`` for the definitions and citations.
"""
from .fftbf_oracle import *  # noqa: F401,F403
