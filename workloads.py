"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and assembles SPD test matrices; it contains none of the
factorisation or derivative arithmetic.  Every generator is NumPy float64 on the host and is
deterministic for a given seed.  No public dataset is involved: the paper's experiments use random
covariance matrices, and the larger workloads here use squared-exponential kernel matrices of the
kind met in Gaussian-process models (the x -> Sigma -> L -> f chain of Sec. 2).

Recipes (the draw order is part of the recipe):
  dense_spd(N, seed):      A ~ N(0,1) (N x N);  Sigma = A A^T / N + shift*I
  se_kernel(X, ell, nug):  Sigma_ij = exp(-|x_i - x_j|^2 / (2 ell^2)) + nug*delta_ij, with
                           |x_i - x_j|^2 = |x_i|^2 + |x_j|^2 - 2 x_i.x_j clamped at 0
  lower_normal(N, rng):    tril of an N(0,1) matrix (an L-bar)
  sym_normal(N, rng):      N(0,1) lower triangle mirrored (a symmetric Sigma-dot whose every
                           independent entry is N(0,1))
"""
from __future__ import annotations

import numpy as np

# Seeds of the named workloads.
SEED_SMALL = 1001      # dense N = 256 random-covariance case
SEED_MEDIUM = 1002     # N = 4096 squared-exponential kernel, 3-D inputs, lengthscale 0.3
SEED_LARGE = 1003      # N = 16384 squared-exponential kernel, 3-D inputs, lengthscale 0.2
SEED_BATCH = 1004      # 2048 matrices, N log-uniform in [16, 512]
SEED_SERVE = 1005      # serving stream: Poisson arrivals, N log-uniform in [64, 4096]


def lower_normal(N, rng):
    """tril of an N x N standard-normal draw (an L-bar input)."""
    return np.tril(rng.standard_normal((N, N)))


def sym_normal(N, rng):
    """Symmetric matrix whose lower triangle (diagonal included) is N(0,1), mirrored upward."""
    lo = np.tril(rng.standard_normal((N, N)))
    return lo + np.tril(lo, -1).T


def dense_spd(N, seed, shift=1.0):
    """Sigma = A A^T / N + shift * I with A ~ N(0,1); returns (Sigma, rng) so later draws continue
    the same stream."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, N))
    S = A @ A.T / max(N, 1)
    S[np.diag_indices(N)] += shift
    return S, rng


def se_kernel(X, lengthscale, nugget, variance=1.0, out=None, row_block=2048):
    """Squared-exponential kernel matrix of the rows of X plus nugget * I, built in row blocks so
    that N = 16384 needs no N x N temporaries beyond the output."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    if out is None:
        out = np.empty((N, N))
    sq = np.einsum("ij,ij->i", X, X)
    inv2l2 = 1.0 / (2.0 * lengthscale * lengthscale)
    for r0 in range(0, N, row_block):
        r1 = min(N, r0 + row_block)
        d2 = sq[r0:r1, None] + sq[None, :] - 2.0 * (X[r0:r1] @ X.T)
        np.maximum(d2, 0.0, out=d2)
        np.multiply(d2, -inv2l2, out=d2)
        np.exp(d2, out=d2)
        if variance != 1.0:
            d2 *= variance
        out[r0:r1] = d2
    out[np.diag_indices(N)] += nugget
    return out


def small_case(N=256, seed=SEED_SMALL):
    """The N = 256 dense case: Sigma = A A^T/N + I (eigenvalues roughly in [1, 5]),
    L-bar = tril(N(0,1)), Sigma-dot = mirrored N(0,1)."""
    S, rng = dense_spd(N, seed, shift=1.0)
    Lbar = lower_normal(N, rng)
    Sdot = sym_normal(N, rng)
    return {"Sigma": S, "Lbar": Lbar, "Sdot": Sdot}


def se_case(N, seed, lengthscale, nugget, dim=3, with_sdot=True):
    """Squared-exponential case: X ~ U[0,1]^dim, Sigma = SE(X; lengthscale) + nugget*I,
    L-bar = tril(N(0,1)), Sigma-dot = mirrored N(0,1) (drawn after L-bar)."""
    rng = np.random.default_rng(seed)
    X = rng.random((N, dim))
    S = se_kernel(X, lengthscale, nugget)
    Lbar = lower_normal(N, rng)
    out = {"Sigma": S, "Lbar": Lbar, "X": X}
    if with_sdot:
        out["Sdot"] = sym_normal(N, rng)
    return out


def medium_case(N=4096, seed=SEED_MEDIUM):
    """N = 4096 squared-exponential kernel on U[0,1]^3, lengthscale 0.3, nugget 1e-4."""
    return se_case(N, seed, 0.3, 1e-4)


def large_case(N=16384, seed=SEED_LARGE, with_sdot=True):
    """N = 16384 squared-exponential kernel on U[0,1]^3, lengthscale 0.2, nugget 1e-2."""
    return se_case(N, seed, 0.2, 1e-2, with_sdot=with_sdot)


def batch_sizes(batch=2048, lo=16, hi=512, seed=SEED_BATCH):
    """N_i = round(exp(U(ln lo, ln hi))) clipped to [lo, hi]; returns (sizes, rng)."""
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=batch))).astype(np.int64)
    return np.clip(n, lo, hi), rng


def batch_case(batch=2048, lo=16, hi=512, seed=SEED_BATCH, shift=0.1):
    """List of dense SPD matrices Sigma_i = A_i A_i^T / N_i + shift*I with log-uniform sizes, plus
    y_i ~ N(0,1) right-hand sides (drawn matrix by matrix: A_i then y_i)."""
    sizes, rng = batch_sizes(batch, lo, hi, seed)
    Sig, ys = [], []
    for n in sizes:
        A = rng.standard_normal((n, n))
        S = A @ A.T / n
        S[np.diag_indices(n)] += shift
        Sig.append(S)
        ys.append(rng.standard_normal(n))
    return {"sizes": sizes, "Sigma": Sig, "y": ys}


def se_case_device(N, seed, lengthscale, nugget, device, dim=3, with_sdot=True):
    """Device-resident squared-exponential case for timing runs at large N (building a
    16384 x 16384 kernel on the host takes minutes).  X comes from the same NumPy stream as
    se_case; the kernel matrix is assembled on the device in float64 with the same formula;
    L-bar (lower) and Sigma-dot (lower triangle; symmetric by convention) are N(0,1) draws from a
    torch generator on the device seeded with `seed`.  Values equal se_case's only up to the
    rounding of the device's exp, and the normal draws differ: use it for timing and for
    property checks, not for element-wise comparison with se_case."""
    import torch

    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.random((N, dim))).to(device)
    sq = (X * X).sum(dim=1)
    S = torch.empty((N, N), dtype=torch.float64, device=device)
    inv2l2 = 1.0 / (2.0 * lengthscale * lengthscale)
    for r0 in range(0, N, 4096):
        r1 = min(N, r0 + 4096)
        d2 = sq[r0:r1, None] + sq[None, :] - 2.0 * (X[r0:r1] @ X.T)
        S[r0:r1] = torch.exp(d2.clamp_(min=0.0).mul_(-inv2l2))
    S.diagonal().add_(nugget)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Lbar = torch.randn((N, N), dtype=torch.float64, device=device, generator=g).tril_()
    out = {"Sigma": S, "Lbar": Lbar}
    if with_sdot:
        out["Sdot"] = torch.randn((N, N), dtype=torch.float64, device=device, generator=g).tril_()
    return out


def serve_trace(rate=200.0, seconds=60.0, lo=64, hi=4096, seed=SEED_SERVE):
    """Request stream of the serving workload: Poisson arrivals (exponential gaps at `rate` per
    second) during `seconds`; per request n log-uniform in [lo, hi], a lengthscale U[0.1, 0.5]
    and a seed for its inputs (see se_request_device)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * seconds * 1.5) + 64)
    t = np.cumsum(gaps)
    t = t[t < seconds]
    m = len(t)
    n = np.clip(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=m))).astype(np.int64), lo, hi)
    return {"t": t, "n": n, "lengthscale": rng.uniform(0.1, 0.5, size=m),
            "seed": rng.integers(1, 2 ** 31 - 1, size=m)}


def se_request_device(n, lengthscale, seed, device):
    """One serving request's inputs on the device: Sigma = SE kernel on n points uniform in [0,1]^2
    (unit variance) + 1e-3 I, and L-bar = tril(N(0,1)) (float64, the se_case_device recipe)."""
    c = se_case_device(int(n), int(seed), float(lengthscale), 1e-3, device, dim=2, with_sdot=False)
    return c["Sigma"], c["Lbar"]


def large_case_device(device, N=16384, seed=SEED_LARGE, with_sdot=True):
    """N = 16384 squared-exponential kernel (3-D, lengthscale 0.2, nugget 1e-2), built on device."""
    return se_case_device(N, seed, 0.2, 1e-2, device, with_sdot=with_sdot)
