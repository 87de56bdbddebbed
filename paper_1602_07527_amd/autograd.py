"""torch.autograd wrappers: the x -> Sigma -> L -> f chain of Sec. 2, with the library's blocked
sweeps as the Cholesky node's forward and backward.

cholesky_ex(Sigma)         (L, info): L = chol(Sigma) by chol_factor; backward
                           Sigma-bar = chol_rev(L, L-bar).
cholesky_batched(Sigmas)   the same for a list of matrices (n <= 512), one launch each way.
gp_neg_log_lik(Sigmas, ys) f_b = sum log L_ii + |L^-1 y_b|^2 / 2 per matrix; the forward is one
                           launch of chol_gp_nll_batched, which also yields df_b/dSigma_b.

Only tril(Sigma) is read.  The gradient handed back for Sigma is the symmetric form (S + S^T)/2 of
eqn (symrev): its inner product with any symmetric perturbation is the first-order change of the
loss, which is the convention torch.linalg.cholesky follows as well.  recompute=True keeps only
the inputs for backward and recomputes what backward needs (L, or the GP gradient) with one more
launch: memory traded for work.  A failed factorisation is reported through the returned device
`info` tensors (0, or the 1-based first non-positive pivot), never by a host synchronisation.
"""
import torch

from . import _binding as B


def _factor_copy(Sigma, nb):
    L = Sigma.detach().clone(memory_format=torch.contiguous_format)
    _, info = B.chol_factor(L, nb=nb)
    return L, info


class _Cholesky(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Sigma, recompute, nb):
        L, info = _factor_copy(Sigma, nb)
        ctx.recompute, ctx.nb = recompute, nb
        ctx.save_for_backward(Sigma if recompute else L)
        ctx.mark_non_differentiable(info)
        return L, info

    @staticmethod
    def backward(ctx, Lbar, _info_grad):
        (saved,) = ctx.saved_tensors
        L = _factor_copy(saved, ctx.nb)[0] if ctx.recompute else saved
        Sbar = Lbar.detach().clone(memory_format=torch.contiguous_format)
        B.chol_rev(L, Sbar, form="sym", nb=ctx.nb)
        return Sbar, None, None


def cholesky_ex(Sigma, recompute=False, nb=0):
    """(L, info): L = chol(Sigma) (lower, positive diagonal, strict upper 0), differentiable with
    the blocked reverse sweep as its backward; info is the device int32 pivot code."""
    return _Cholesky.apply(Sigma, recompute, nb)


def cholesky(Sigma, recompute=False, nb=0):
    """L = chol(Sigma); see cholesky_ex."""
    return cholesky_ex(Sigma, recompute, nb)[0]


def _factor_copies(Sigmas):
    Ls = [S.detach().clone(memory_format=torch.contiguous_format) for S in Sigmas]
    return Ls, B.chol_factor_batched(Ls)


class _BatchedCholesky(torch.autograd.Function):
    @staticmethod
    def forward(ctx, recompute, *Sigmas):
        Ls, info = _factor_copies(Sigmas)
        ctx.recompute = recompute
        ctx.save_for_backward(*(Sigmas if recompute else Ls))
        ctx.mark_non_differentiable(info)
        return (info, *Ls)

    @staticmethod
    def backward(ctx, _info_grad, *Lbars):
        saved = ctx.saved_tensors
        Ls = _factor_copies(saved)[0] if ctx.recompute else list(saved)
        Sbars = [torch.zeros_like(L) if g is None else g.detach().clone(memory_format=torch.contiguous_format)
                 for L, g in zip(Ls, Lbars)]
        B.chol_rev_batched(Ls, Sbars, form="sym")
        return (None, *Sbars)


def cholesky_batched(Sigmas, recompute=False):
    """([chol(S) for S in Sigmas], info) in one launch, differentiable (one launch of the batched
    reverse sweep as backward)."""
    info, *Ls = _BatchedCholesky.apply(recompute, *Sigmas)
    return Ls, info


def _gp_forward(Sigmas, ys):
    work = [S.detach().clone(memory_format=torch.contiguous_format) for S in Sigmas]
    grads = [torch.empty_like(w) for w in work]
    f, info = B.chol_gp_nll_batched(work, [y.detach().contiguous() for y in ys], grads)
    return f, info, grads


class _GPNegLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, recompute, n_mats, *args):
        Sigmas, ys = args[:n_mats], args[n_mats:]
        f, info, grads = _gp_forward(Sigmas, ys)
        ctx.recompute, ctx.n_mats = recompute, n_mats
        ctx.save_for_backward(*(Sigmas if recompute else grads), *ys)
        ctx.mark_non_differentiable(info)
        return f, info

    @staticmethod
    def backward(ctx, gf, _info_grad):
        n = ctx.n_mats
        if any(ctx.needs_input_grad[2 + n:]):
            raise NotImplementedError("gp_neg_log_lik differentiates with respect to the Sigmas only")
        saved = ctx.saved_tensors
        ys = saved[n:]
        grads = _gp_forward(saved[:n], ys)[2] if ctx.recompute else saved[:n]
        return (None, None, *[gf[b] * grads[b] for b in range(n)], *[None] * len(ys))


def gp_neg_log_lik(Sigmas, ys, recompute=False):
    """(f, info): f_b = sum_i log L_ii + |L^-1 y_b|^2 / 2 for every (Sigma_b, y_b), differentiable
    with respect to the Sigmas; the forward is one launch that also produces df_b/dSigma_b."""
    return _GPNegLogLik.apply(recompute, len(Sigmas), *Sigmas, *ys)
