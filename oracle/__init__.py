"""FP64 CPU oracle (test infrastructure only; see h2_oracle.py)."""
from .h2_oracle import *  # noqa: F401,F403
