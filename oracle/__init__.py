"""FP64 CPU oracle (test infrastructure only; see oracle/synth.py)."""
from .synth import *  # noqa: F401,F403
