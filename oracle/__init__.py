"""FP64 CPU oracle (test infrastructure only; see sfft_oracle)."""
from .sfft_oracle import *  # noqa: F401,F403
from .sfft_oracle import SolveInfo  # noqa: F401
