"""The oracle's independent routes agree, and the O(N^4) Jacobian of Sec. 3 matches brute force.

Routes (Sec. 3 vs Sec. 4): symbolic formulas (eqns (symfwd), (symrev)); Level-2 column algorithms
(Sec. 4.1); Level-3 block algorithms (Sec. 4.2) for every block size, including sizes that do not
divide N.  Jacobian (N <= 8): eqn (delements) entry by entry, eqn (bletch) with Kronecker products,
central differences of host LAPACK, chol_fwd columns and chol_rev rows.  A final group plants
mistakes in a copy of the oracle and checks that some pin fails.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import oracle.cholesky_oracle as OC
import workloads as W

U = np.finfo(np.float64).eps


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def case(N, seed):
    S, rng = W.dense_spd(N, seed)
    L = sla.cholesky(S, lower=True)
    return S, L, W.lower_normal(N, rng), W.sym_normal(N, rng)


@pytest.mark.parametrize("N", [1, 2, 9, 40])
def test_level2_matches_symbolic(N):
    S, L, Lb, Sd = case(N, 600 + N)
    assert rel(O.chol_unblocked(S), L) <= 100 * N * U
    assert rel(O.chol_unblocked_fwd(L, Sd), O.chol_fwd(L, Sd)) <= 1e-12
    assert rel(O.chol_unblocked_rev(L, Lb), O.chol_rev(L, Lb, "tril")) <= 1e-12


@pytest.mark.parametrize("N,nb", [(1, 1), (7, 1), (7, 3), (16, 4), (33, 8), (40, 16), (40, 64),
                                  (50, 7)])
def test_level3_matches_symbolic(N, nb):
    S, L, Lb, Sd = case(N, 700 + N + nb)
    assert rel(O.chol_blocked(S, nb), L) <= 100 * N * U
    assert rel(O.chol_blocked_fwd(L, Sd, nb), O.chol_fwd(L, Sd)) <= 1e-12
    assert rel(O.chol_blocked_rev(L, Lb, nb), O.chol_rev(L, Lb, "tril")) <= 1e-12


def _fd_jacobian(S):
    N = S.shape[0]
    pairs = [(i, j) for j in range(N) for i in range(j, N)]
    J = np.zeros((len(pairs), len(pairs)))
    h = 1e-6
    for c, (k, l) in enumerate(pairs):
        E = np.zeros((N, N))
        E[k, l] = E[l, k] = 1.0
        dL = (sla.cholesky(S + h / 2 * E, lower=True) - sla.cholesky(S - h / 2 * E, lower=True)) / h
        J[:, c] = O.vech(dL)
    return J


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_jacobian_routes(N):
    S, L, _, _ = case(N, 800 + N)
    Jd = O.jacobian_delements(L)
    Jb = O.jacobian_bletch(L)
    Jf = _fd_jacobian(S)
    assert rel(Jd, Jb) <= 1e-13
    assert rel(Jd, Jf) <= 1e-7
    pairs = [(i, j) for j in range(N) for i in range(j, N)]
    # chol_fwd columns: Sigma-dot = E_kl + E_lk
    for c, (k, l) in enumerate(pairs):
        E = np.zeros((N, N))
        E[k, l] = E[l, k] = 1.0
        assert np.allclose(O.vech(O.chol_fwd(L, E)), Jd[:, c], rtol=1e-11, atol=1e-12)
    # chol_rev rows: L-bar = E_ij; the independent-element form (eqn (symrev)) is the gradient
    # with Sigma_kl and Sigma_lk moving together, i.e. the Jacobian row.
    for r, (i, j) in enumerate(pairs):
        E = np.zeros((N, N))
        E[i, j] = 1.0
        row = O.vech(O.chol_rev(L, E, "indep"))
        assert np.allclose(row, Jd[r], rtol=1e-11, atol=1e-12)


def test_jacobian_two_by_two_by_hand():
    # Sigma = [[a, b], [b, c]]: L11 = sqrt(a), L21 = b/sqrt(a), L22 = sqrt(c - b^2/a).
    a, b, c = 4.0, 1.0, 3.0
    L11, L21 = np.sqrt(a), b / np.sqrt(a)
    L22 = np.sqrt(c - b * b / a)
    want = np.array([
        [1 / (2 * L11), 0.0, 0.0],
        [-b / (2 * a ** 1.5), 1 / np.sqrt(a), 0.0],
        [(b * b / a ** 2) / (2 * L22), -b / (a * L22), 1 / (2 * L22)],
    ])
    L = np.array([[L11, 0], [L21, L22]])
    assert np.allclose(O.jacobian_delements(L), want, rtol=1e-14, atol=0)
    assert np.allclose(O.jacobian_bletch(L), want, rtol=1e-14, atol=0)


# ----------------------------------------------------------------------------- planted mistakes

def _pins_pass(N=6, seed=77):
    """A compact subset of the pins, run against whatever the oracle module currently holds."""
    S, L, Lb, Sd = case(N, seed)
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N))
    C = G + G.T
    M = np.tril(rng.standard_normal((N, N)))
    ok = [
        rel(OC.chol(S)[0] @ OC.chol(S)[0].T, S) <= 1e-13,
        rel(OC.chol_rev(L, np.tril(2 * C @ L)), C) <= 1e-10,
        rel(OC.chol_fwd(L, M @ L.T + L @ M.T), M) <= 1e-10,
        rel(OC.chol_unblocked_rev(L, Lb), OC.chol_rev(L, Lb, "tril")) <= 1e-10,
        rel(OC.chol_unblocked_fwd(L, Sd), OC.chol_fwd(L, Sd)) <= 1e-10,
        rel(OC.chol_blocked_rev(L, Lb, 4), OC.chol_rev(L, Lb, "tril")) <= 1e-10,
        rel(OC.chol_blocked_fwd(L, Sd, 4), OC.chol_fwd(L, Sd)) <= 1e-10,
        rel(OC.chol_blocked(S, 4), L) <= 1e-12,
    ]
    return all(ok)


def test_unmodified_oracle_passes_compact_pins():
    assert _pins_pass()


def _phi_no_halving(A):
    return np.tril(np.asarray(A, dtype=np.float64))


def _phi_strict(A):
    return np.tril(np.asarray(A, dtype=np.float64), -1)


def _level2partition_shifted(A, j):
    return A[j, :j], A[j:j + 1, j], A[j + 1:, :j], A[j + 1:, min(j + 1, A.shape[1] - 1)]


@pytest.mark.parametrize("name,fake", [
    ("Phi", _phi_no_halving),
    ("Phi", _phi_strict),
    ("level2partition", _level2partition_shifted),
])
def test_planted_mistake_is_caught(monkeypatch, name, fake):
    monkeypatch.setattr(OC, name, fake)
    assert not _pins_pass()


def test_planted_sign_error_in_level3_rev_is_caught(monkeypatch):
    orig = OC.chol_unblocked_rev
    monkeypatch.setattr(OC, "chol_unblocked_rev", lambda L, A: -orig(L, A))
    assert not _pins_pass()


def test_planted_transpose_in_symbolic_rev_is_caught(monkeypatch):
    def bad_S(L, Lbar):
        L = np.tril(L)
        P = OC.Phi(np.tril(Lbar) @ L.T)             # operands transposed
        X = sla.solve_triangular(L, P, lower=True, trans=1)
        return sla.solve_triangular(L, X.T, lower=True, trans=1).T
    monkeypatch.setattr(OC, "chol_rev_S", bad_S)
    assert not _pins_pass()


def _gp_pins_pass(fn):
    """The two pins of the GP loss value (the integer golden and the log-det route) applied to fn."""
    from _golden import load
    g = load("gp_int.txt")
    L, y, z, w = g["L"], g["y"][:, 0], g["z"][:, 0], g["w"][:, 0]
    f, Lbar = fn(L, y)
    ok = [abs(f - (np.log(np.prod(np.diag(L))) + 0.5 * float(z @ z))) <= 1e-12 * abs(f),
          np.abs(Lbar - (np.diag(1.0 / np.diag(L)) - np.tril(np.outer(w, z)))).max() <= 1e-12]
    S, L2, _, _ = case(7, 91)
    y2 = np.random.default_rng(91).standard_normal(7)
    f2, _ = fn(L2, y2)
    ok.append(abs(f2 - 0.5 * (np.linalg.slogdet(S)[1] + y2 @ np.linalg.solve(S, y2))) <= 1e-12 * abs(f2))
    return all(ok)


def test_gp_pins_catch_planted_mistakes():
    assert _gp_pins_pass(OC.gp_loss_and_lbar)

    def no_half(L, y):               # the 1/2 on |L^-1 y|^2 dropped
        z = sla.solve_triangular(L, y, lower=True)
        f, Lbar = OC.gp_loss_and_lbar(L, y)
        return f + 0.5 * float(z @ z), Lbar

    def transposed_w(L, y):          # w = L^-1 z instead of L^-T z
        z = sla.solve_triangular(L, y, lower=True)
        w = sla.solve_triangular(L, z, lower=True)
        f, _ = OC.gp_loss_and_lbar(L, y)
        return f, np.diag(1.0 / np.diag(L)) - np.tril(np.outer(w, z))

    def log_of_sum(L, y):            # log of the summed diagonal instead of the summed logs
        z = sla.solve_triangular(L, y, lower=True)
        _, Lbar = OC.gp_loss_and_lbar(L, y)
        return float(np.log(np.sum(np.diag(L))) + 0.5 * z @ z), Lbar

    for bad in (no_half, transposed_w, log_of_sum):
        assert not _gp_pins_pass(bad), bad.__name__
