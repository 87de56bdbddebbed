"""MI355X-native blocked Cholesky factorisation and derivative propagation (Murray 2016).

Public calls (torch tensors as device memory, work on the current stream):
  chol_factor(A)     Sigma -> L               (Sec. 4.2 chol_blocked)
  chol_rev(L, A)     L-bar -> Sigma-bar       (Sec. 4.2 chol_blocked_rev)
  chol_fwd(L, A)     Sigma-dot -> L-dot       (Sec. 4.2 chol_blocked_fwd)
"""
from ._binding import (CholError, LIB_PATH, chol_factor, chol_fwd, chol_rev, load_library,
                       profile_begin, profile_end, workspace_bytes)

__all__ = ["CholError", "LIB_PATH", "chol_factor", "chol_fwd", "chol_rev", "load_library",
           "profile_begin", "profile_end", "workspace_bytes"]
