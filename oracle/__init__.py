"""FP64 CPU oracle for HyGT (test infrastructure; see hygt_oracle.py)."""
from .hygt_oracle import *  # noqa: F401,F403
