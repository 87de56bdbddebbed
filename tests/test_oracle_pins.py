"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the mathematics) that fixes the expected value.  None
of these calls the HIP library; all run with -m "not gpu".
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from _golden import load

U = np.finfo(np.float64).eps


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def spd(N, seed, shift=1.0):
    S, rng = W.dense_spd(N, seed, shift)
    return S, rng


# ----------------------------------------------------------------------------- Phi and tril

def test_phi_literal():
    # eqn (phi): strict lower kept, diagonal halved, strict upper zero.
    A = np.array([[2.0, 5.0, 7.0], [3.0, 4.0, 9.0], [1.0, -6.0, 8.0]])
    want = np.array([[1.0, 0, 0], [3.0, 2.0, 0], [1.0, -6.0, 4.0]])
    assert np.array_equal(O.Phi(A), want)


# ----------------------------------------------------------------------------- factor

def test_chol_golden_integer():
    g = load("chol_int.txt")
    L, info = O.chol(g["Sigma"])
    assert info == 0
    assert np.abs(L - g["L"]).max() <= 4 * U * np.abs(g["L"]).max()


@pytest.mark.parametrize("N", [1, 2, 3, 7, 33, 100])
def test_chol_reconstruction_and_lapack(N):
    S, _ = spd(N, 10 + N)
    L, info = O.chol(S)
    assert info == 0
    assert np.all(np.diag(L) > 0) and np.all(np.triu(L, 1) == 0)
    assert rel(L @ L.T, S) <= 4 * N * U
    # a library special case: host LAPACK dpotrf, also as the oracle's large-size route
    assert rel(L, sla.cholesky(S, lower=True)) <= 50 * N * U
    Lh = O.chol_host(S + np.triu(np.full((N, N), 7.0), 1))     # reads the lower triangle only
    assert rel(Lh, L) <= 50 * N * U and np.all(np.triu(Lh, 1) == 0)


def test_chol_reads_lower_only():
    S, _ = spd(9, 3)
    junk = S + np.triu(np.full((9, 9), 1e3), 1)
    assert np.array_equal(O.chol(S)[0], O.chol(junk)[0])


def test_chol_info_non_spd():
    S, _ = spd(12, 4)
    S[6, 6] = -1.0       # first non-positive pivot at column 7 (1-based)
    L, info = O.chol(S)
    assert info == 7
    assert np.all(np.isfinite(L[:, :6]))


def test_scalar_case():
    # N = 1: L = sqrt(s), L-dot = s-dot / (2 L), Sigma-bar = L-bar / (2 L).
    s, sd, lb = 2.25, 0.3, -0.7
    L, _ = O.chol(np.array([[s]]))
    assert L[0, 0] == 1.5
    assert O.chol_fwd(L, np.array([[sd]]))[0, 0] == pytest.approx(sd / 3.0, rel=1e-15)
    for form in ("sym", "tril", "indep"):
        assert O.chol_rev(L, np.array([[lb]]), form)[0, 0] == pytest.approx(lb / 3.0, rel=1e-15)


# ----------------------------------------------------------------------------- forward mode

def test_fwd_golden():
    g = load("fwd_closed.txt")
    Ld = O.chol_fwd(g["L"], g["Sdot"])
    assert np.abs(Ld - g["Ldot"]).max() <= 1e-13


@pytest.mark.parametrize("N", [2, 5, 31])
def test_fwd_closed_forms(N):
    S, rng = spd(N, 100 + N)
    L = sla.cholesky(S, lower=True)
    # Sigma-dot = M L^T + L M^T for lower M  =>  L-dot = M  (eqn (dchol) with dL = M)
    M = np.tril(rng.standard_normal((N, N)))
    assert rel(O.chol_fwd(L, M @ L.T + L @ M.T), M) <= 1e-12
    # scaling Sigma by (1+t) scales L by sqrt(1+t): chol_fwd(L, Sigma) = L/2
    assert rel(O.chol_fwd(L, S), 0.5 * L) <= 1e-13


@pytest.mark.parametrize("N", [3, 16, 64])
def test_fwd_central_differences(N):
    # the paper's own check (Appendix code): central differences with a +-h Sigma-dot/2 step,
    # evaluated with host LAPACK so the pin does not reuse the oracle's factorisation.
    S, rng = spd(N, 200 + N)
    Sd = W.sym_normal(N, rng)
    h = 1e-6
    fd = (sla.cholesky(S + h / 2 * Sd, lower=True) - sla.cholesky(S - h / 2 * Sd, lower=True)) / h
    L = sla.cholesky(S, lower=True)
    assert rel(O.chol_fwd(L, Sd), fd) <= 1e-7


# ----------------------------------------------------------------------------- reverse mode

def test_rev_golden():
    g = load("rev_closed.txt")
    Sb = O.chol_rev(g["L"], g["Lbar"], "sym")
    assert np.abs(Sb - g["Sbar_sym"]).max() <= 1e-13


@pytest.mark.parametrize("N", [2, 6, 37])
def test_rev_closed_forms(N):
    S, rng = spd(N, 300 + N)
    L = sla.cholesky(S, lower=True)
    Si = np.linalg.inv(S)
    # f = Tr(C Sigma): L-bar = tril(2 C L) -> Sigma-bar = C
    G = rng.standard_normal((N, N))
    C = G + G.T
    assert rel(O.chol_rev(L, np.tril(2 * C @ L)), C) <= 1e-12
    # f = (1/2) Tr(Sigma) = (1/2)|L|_F^2: L-bar = L -> I/2
    assert rel(O.chol_rev(L, L), 0.5 * np.eye(N)) <= 1e-13
    # f = log det L = (1/2) log det Sigma: L-bar = diag(1/L_ii) -> Sigma^-1 / 2
    assert rel(O.chol_rev(L, np.diag(1 / np.diag(L))), 0.5 * Si) <= 1e-12
    # Gaussian-process loss sum log L_ii + |L^-1 y|^2/2 -> (Sigma^-1 - a a^T)/2, a = Sigma^-1 y
    y = rng.standard_normal(N)
    _, Lbar = O.gp_loss_and_lbar(L, y)
    a = np.linalg.solve(S, y)
    assert rel(O.chol_rev(L, Lbar), 0.5 * (Si - np.outer(a, a))) <= 1e-12


@pytest.mark.parametrize("N", [4, 24])
def test_rev_central_differences(N):
    # f(Sigma) = sum(G * L(Sigma)) with G lower; directional derivative along a symmetric
    # Sigma-dot equals sum_ij Sbar_ij Sdot_ij, with L from host LAPACK.
    S, rng = spd(N, 400 + N)
    G = np.tril(rng.standard_normal((N, N)))
    Sd = W.sym_normal(N, rng)
    h = 1e-6
    f = lambda A: np.sum(G * sla.cholesky(A, lower=True))
    fd = (f(S + h / 2 * Sd) - f(S - h / 2 * Sd)) / h
    L = sla.cholesky(S, lower=True)
    got = np.sum(O.chol_rev(L, G, "sym") * Sd)
    assert got == pytest.approx(fd, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("N", [3, 20, 65])
def test_adjoint_identity_and_forms(N):
    # Tr(L-bar^T L-dot) = sum_ij Sbar_ij Sdot_ij for the symmetric and the lower-triangular forms
    # (the paper's reverse-mode check in the Appendix code), and = sum_{k>=l} for Brewer's form.
    S, rng = spd(N, 500 + N)
    L = sla.cholesky(S, lower=True)
    Lb = W.lower_normal(N, rng)
    Sd = W.sym_normal(N, rng)
    lhs = np.sum(Lb * O.chol_fwd(L, Sd))
    f = O.sbar_forms(O.chol_rev_S(L, Lb))
    assert np.sum(f["sym"] * Sd) == pytest.approx(lhs, rel=1e-11)
    assert np.sum(f["tril"] * Sd) == pytest.approx(lhs, rel=1e-11)
    assert np.sum(np.tril(f["indep"]) * Sd) == pytest.approx(lhs, rel=1e-11)
    assert np.allclose(f["sym"], f["sym"].T, rtol=0, atol=0)


def test_derivative_inputs_read_lower_only():
    N = 11
    S, rng = spd(N, 7)
    L = sla.cholesky(S, lower=True)
    Lb = W.lower_normal(N, rng)
    Sd = W.sym_normal(N, rng)
    junk = np.triu(rng.standard_normal((N, N)), 1)
    assert np.array_equal(O.chol_rev(L, Lb), O.chol_rev(L, Lb + junk))
    assert np.array_equal(O.chol_fwd(L, np.tril(Sd)), O.chol_fwd(L, np.tril(Sd) + junk))


# ----------------------------------------------------------------------------- GP loss value

def test_gp_loss_golden_integer():
    # Sec. 2's chain closed by f = sum log L_ii + |L^-1 y|^2 / 2 on a hand-built case in which
    # z = L^-1 y and w = L^-T z are integers (tests/golden/gp_int.txt): f and L-bar follow by hand.
    g = load("gp_int.txt")
    L, y, z, w = g["L"], g["y"][:, 0], g["z"][:, 0], g["w"][:, 0]
    f, Lbar = O.gp_loss_and_lbar(L, y)
    want_f = np.log(np.prod(np.diag(L))) + 0.5 * float(z @ z)
    assert f == pytest.approx(want_f, rel=4 * U)
    want_Lbar = np.diag(1.0 / np.diag(L)) - np.tril(np.outer(w, z))
    assert np.abs(Lbar - want_Lbar).max() <= 8 * U * np.abs(want_Lbar).max()


@pytest.mark.parametrize("N", [1, 5, 40])
def test_gp_loss_value_is_half_logdet_plus_quadratic(N):
    # f = log det L + |L^-1 y|^2 / 2 = (1/2) log det Sigma + (1/2) y^T Sigma^-1 y, with the right
    # side from host LAPACK routes that share nothing with the oracle's triangular solves.
    S, rng = spd(N, 900 + N)
    y = rng.standard_normal(N)
    f, _ = O.gp_loss_and_lbar(sla.cholesky(S, lower=True), y)
    sign, logdet = np.linalg.slogdet(S)
    assert sign > 0
    want = 0.5 * logdet + 0.5 * float(y @ np.linalg.solve(S, y))
    assert f == pytest.approx(want, rel=1e-13, abs=1e-13)
