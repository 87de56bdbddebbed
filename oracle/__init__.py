"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from .cholesky_oracle import *  # noqa: F401,F403
