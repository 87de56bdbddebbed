"""MI355X-native blocked Cholesky factorisation and derivative propagation (Murray 2016).

Public calls (torch tensors as device memory, work on the current stream):
  chol_factor(A)     Sigma -> L               (Sec. 4.2 chol_blocked)
  chol_rev(L, A)     L-bar -> Sigma-bar       (Sec. 4.2 chol_blocked_rev)
  chol_fwd(L, A)     Sigma-dot -> L-dot       (Sec. 4.2 chol_blocked_fwd)
  chol_factor_fwd(A, D)  both in one sweep (Sigma -> L and Sigma-dot -> L-dot)
  chol_rev_noalloc(L, A) chol_rev on the library's static device scratch (n <= 4096)
(single-matrix options: diag='auto' | 'symbolic' | 'level2' for the diagonal-block variant of
chol_rev / chol_fwd, layout='row' | 'col' for row- or column-major storage, precision for the
reduced-precision trailing modes) and their batched forms (many matrices, n <= 512, one
call each: step-synchronous grouped launches, or one persistent launch for the forward sweep),
including a fused
factor + reverse sweep (chol_factor_rev_batched) and a fused Gaussian-process loss
(chol_gp_nll_batched: Sigma -> L -> f -> Sigma-bar per matrix).  `autograd` wraps them as
torch.autograd Functions; `serve` runs a continuous-batching request loop on top of them.
"""
from ._binding import (Batch, CholError, LIB_PATH, batched_workspace_bytes, chol_factor,
                       chol_factor_batched, chol_factor_fwd, chol_factor_rev_batched, chol_fwd,
                       chol_fwd_batched, chol_gp_nll_batched, chol_rev, chol_rev_batched, chol_rev_noalloc,
                       load_library, profile_begin, profile_end, Vecs, workspace_bytes)

__all__ = ["Batch", "CholError", "LIB_PATH", "batched_workspace_bytes", "chol_factor",
           "chol_factor_batched", "chol_factor_fwd", "chol_factor_rev_batched", "chol_fwd",
           "chol_fwd_batched", "chol_gp_nll_batched", "chol_rev", "chol_rev_batched", "chol_rev_noalloc",
           "load_library",
           "profile_begin", "profile_end", "Vecs", "workspace_bytes"]
