"""Plain FP64 CPU oracle for the Cholesky factor and its forward/reverse derivative propagation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this module:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
no code, tables or helpers with the HIP library.

Source: I. Murray, "Differentiation of the Cholesky decomposition" (arXiv:1602.07527, 2016).
Every function names the section / equation / algorithm it restates.  Matrices are NumPy float64
arrays; all derivative inputs (L-bar, Sigma-dot) are read from their lower triangle only.

Conventions fixed here (the paper leaves them open):
  * Sigma-dot is symmetric; it is rebuilt from its lower triangle (Sec. 3, below eqn (symfwd)).
  * chol_rev's default output is the symmetric gradient  Sbar_sym = (S + S^T)/2  with
    S = L^-T Phi(L^T Lbar) L^-1 (eqn (symrev)); it satisfies  Tr(Lbar^T Ldot) = sum_ij Sbar_ij Sdot_ij
    for every symmetric Sigma-dot.  The paper's lower-triangular form  T = Phi(S + S^T)
    (eqn (symrevtril)) and Brewer's independent-element form  S + S^T - diag(S) (eqn (symrev))
    are available through ``sbar_forms``.
  * Non-SPD input to ``chol``: LAPACK-style info = 1-based index of the first non-positive pivot.

Pins (tests/test_oracle_*.py, run with -m "not gpu"): LL^T = Sigma reconstruction and agreement with
host LAPACK; closed-form forward and reverse results (f = Tr(C Sigma), (1/2) log det Sigma, a
Gaussian-process loss, L-dot = M for Sigma-dot = M L^T + L M^T, chol_fwd(L, Sigma) = L/2);
central finite differences; the adjoint identity; N = 1 scalars; the O(N^4) Jacobian from
eqns (delements) and (bletch) against finite differences at N <= 8; and agreement of the
symbolic, Level-2 and Level-3 routes for every block size.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

__all__ = [
    "tril", "Phi", "sym_from_lower", "chol", "chol_host", "chol_fwd", "chol_rev", "chol_rev_S", "sbar_forms",
    "level2partition", "chol_unblocked", "chol_unblocked_fwd", "chol_unblocked_rev",
    "level3partition", "chol_blocked", "chol_blocked_fwd", "chol_blocked_rev",
    "vech", "vec", "elimination_matrix", "duplication_matrix",
    "jacobian_delements", "jacobian_bletch", "gp_loss_and_lbar",
]


# --------------------------------------------------------------------------------------------
# Elementary operators
# --------------------------------------------------------------------------------------------

def tril(A):
    """Lower triangle including the diagonal; zero elsewhere (eqn (tril), Sec. 4.1)."""
    return np.tril(np.asarray(A, dtype=np.float64))


def Phi(A):
    """Lower triangle with the diagonal halved (eqn (phi), Sec. 3)."""
    out = np.tril(np.asarray(A, dtype=np.float64)).copy()
    idx = np.arange(out.shape[0])
    out[idx, idx] *= 0.5
    return out


def sym_from_lower(A):
    """The symmetric matrix whose lower triangle is tril(A): Sigma-dot must be symmetric (Sec. 3)."""
    lo = np.tril(np.asarray(A, dtype=np.float64))
    return lo + np.tril(lo, -1).T


# --------------------------------------------------------------------------------------------
# Plain definitions
# --------------------------------------------------------------------------------------------

def chol(Sigma):
    """The unique lower-triangular L with positive diagonal and L L^T = Sigma (Sec. 1).

    Written out column by column from L L^T = Sigma: for column j,
    L_jj = sqrt(Sigma_jj - sum_{m<j} L_jm^2) and L_ij = (Sigma_ij - sum_{m<j} L_im L_jm) / L_jj
    for i > j (the update of Sec. 4.1's chol_unblocked).  Only tril(Sigma) is read.
    Returns (L, info): info = 0 on success, else the 1-based column of the first non-positive
    pivot; columns from that one on are then left as NaN.
    """
    A = np.tril(np.asarray(Sigma, dtype=np.float64))
    N = A.shape[0]
    L = np.zeros((N, N))
    for j in range(N):
        piv = A[j, j] - L[j, :j] @ L[j, :j]
        if not piv > 0.0:
            L[j:, j:] = np.tril(np.full((N - j, N - j), np.nan))
            return L, j + 1
        L[j, j] = np.sqrt(piv)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, 0


def chol_host(Sigma):
    """The same unique factor as ``chol`` (Sec. 1) computed by host LAPACK's dpotrf: the library
    special case of the definition, for sizes where the column-by-column loop is too slow
    (pinned against ``chol`` in the CPU tests).  Only tril(Sigma) is read; raises on a
    non-positive pivot."""
    from scipy.linalg import cholesky
    L = cholesky(np.tril(np.asarray(Sigma, dtype=np.float64)), lower=True, check_finite=False)
    return np.ascontiguousarray(L)


def chol_fwd(L, Sigma_dot):
    """Forward-mode propagation  L-dot = L Phi(L^-1 Sigma-dot L^-T)  (eqn (symfwd), Sec. 3).

    Sigma-dot is taken as symmetric from its lower triangle.  The two triangular solves are host
    LAPACK calls (library primitives).
    """
    L = np.tril(np.asarray(L, dtype=np.float64))
    Sd = sym_from_lower(Sigma_dot)
    X = solve_triangular(L, Sd, lower=True)            # L^-1 Sigma-dot
    Y = solve_triangular(L, X.T, lower=True).T         # (L^-1 (L^-1 Sigma-dot)^T)^T = L^-1 Sd L^-T
    return L @ Phi(Y)


def chol_rev_S(L, Lbar):
    """S = L^-T Phi(L^T Lbar) L^-1 of eqn (symrev) (Sec. 3), with Lbar read from its lower triangle."""
    L = np.tril(np.asarray(L, dtype=np.float64))
    P = Phi(L.T @ np.tril(np.asarray(Lbar, dtype=np.float64)))
    X = solve_triangular(L, P, lower=True, trans=1)          # L^-T P
    return solve_triangular(L, X.T, lower=True, trans=1).T    # (L^-T (L^-T P)^T)^T = L^-T P L^-1


def sbar_forms(S_or_T, *, given="S"):
    """The three readings of the reverse-mode output (Sec. 3, eqns (symrev) and (symrevtril)).

    given="S": input is S of eqn (symrev).  given="T": input is the lower-triangular T.
    Returns a dict with
      'tril'  : T = Phi(S + S^T)                 (eqn (symrevtril); the paper's in-place output)
      'sym'   : (S + S^T)/2 = (T + T^T)/2         (symmetric gradient; the library default)
      'indep' : S + S^T - diag(S) = T + T^T - diag(T)  (eqn (symrev); independent elements)
    """
    M = np.asarray(S_or_T, dtype=np.float64)
    if given == "S":
        T = Phi(M + M.T)
    elif given == "T":
        T = np.tril(M)
    else:
        raise ValueError(given)
    dT = np.diag(np.diag(T))
    return {"tril": T, "sym": 0.5 * (T + T.T), "indep": T + T.T - dT}


def chol_rev(L, Lbar, form="sym"):
    """Reverse-mode propagation Sigma-bar(L, L-bar) from eqn (symrev) (Sec. 3); see sbar_forms."""
    return sbar_forms(chol_rev_S(L, Lbar), given="S")[form]


# --------------------------------------------------------------------------------------------
# Level-2 (unblocked) algorithms of Sec. 4.1, zero-based and half-open
# --------------------------------------------------------------------------------------------

def level2partition(A, j):
    """Views r = A[j, :j], d = A[j, j] (as a 1x1 view), B = A[j+1:, :j], c = A[j+1:, j] (Sec. 4.1)."""
    return A[j, :j], A[j:j + 1, j], A[j + 1:, :j], A[j + 1:, j]


def chol_unblocked(A):
    """Sec. 4.1 chol_unblocked (DPOTF2): for each column, d <- sqrt(d - r r^T), c <- (c - B r^T)/d.

    Works on a copy; returns tril of the result.  No positivity check (a negative pivot gives NaN).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    for j in range(A.shape[0]):
        r, d, B, c = level2partition(A, j)
        d[...] = np.sqrt(d - r @ r)
        c[...] = (c - B @ r) / d
    return np.tril(A)


def chol_unblocked_fwd(L, Adot):
    """Sec. 4.1 chol_unblocked_fwd, from eqns (dub1)-(dub2): in place on tril(Adot), column by column,
    d-dot <- (d-dot/2 - r r-dot^T)/d ;  c-dot <- (c-dot - B-dot r^T - B r-dot^T - c d-dot)/d.
    """
    L = np.asarray(L, dtype=np.float64)
    Ad = np.tril(np.asarray(Adot, dtype=np.float64)).copy()
    for j in range(L.shape[0]):
        r, d, B, c = level2partition(L, j)
        rd, dd, Bd, cd = level2partition(Ad, j)
        dd[...] = (dd / 2 - r @ rd) / d
        cd[...] = (cd - Bd @ r - B @ rd - c * dd) / d
    return np.tril(Ad)


def chol_unblocked_rev(L, Abar):
    """Sec. 4.1 chol_unblocked_rev: the reverse sweep over columns j = N..1 of the Level-2 routine.

    In place on tril(Abar): d-bar <- d-bar - c^T c-bar/d;  [d-bar; c-bar] <- [d-bar; c-bar]/d;
    r-bar <- r-bar - [d-bar c-bar^T][r; B];  B-bar <- B-bar - c-bar r;  d-bar <- d-bar/2.
    Input tril(Abar) = L-bar; output = T = tril(Sigma-bar) of eqn (symrevtril).
    """
    L = np.asarray(L, dtype=np.float64)
    Ab = np.tril(np.asarray(Abar, dtype=np.float64)).copy()
    for j in range(L.shape[0] - 1, -1, -1):
        r, d, B, c = level2partition(L, j)
        rb, db, Bb, cb = level2partition(Ab, j)
        db -= c @ cb / d
        db /= d
        cb /= d
        rb -= db * r + cb @ B
        Bb -= np.outer(cb, r)
        db /= 2
    return np.tril(Ab)


# --------------------------------------------------------------------------------------------
# Level-3 (blocked) algorithms of Sec. 4.2
# --------------------------------------------------------------------------------------------

def level3partition(A, j, k):
    """Views R = A[j:k, :j], D = A[j:k, j:k], B = A[k:, :j], C = A[k:, j:k] (Sec. 4.2, half-open)."""
    return A[j:k, :j], A[j:k, j:k], A[k:, :j], A[k:, j:k]


def _blocks_forward(N, nb):
    """Block columns [j, k) left to right; the short block (if any) is last (Sec. 4.2)."""
    return [(j, min(N, j + nb)) for j in range(0, N, nb)]


def chol_blocked(A, nb):
    """Sec. 4.2 chol_blocked (left-looking DPOTRF):
    D <- D - tril(R R^T); D <- chol_unblocked(D); C <- C - B R^T; C <- C tril(D)^-T.
    """
    A = np.tril(np.asarray(A, dtype=np.float64)).copy()
    for j, k in _blocks_forward(A.shape[0], nb):
        R, D, B, C = level3partition(A, j, k)
        D[...] = D - np.tril(R @ R.T)
        D[...] = chol_unblocked(D)
        C[...] = C - B @ R.T
        C[...] = solve_triangular(np.tril(D), C.T, lower=True).T    # C tril(D)^-T
    return np.tril(A)


def chol_blocked_fwd(L, Adot, nb):
    """Sec. 4.2 chol_blocked_fwd:
    D-dot <- D-dot - tril(R-dot R^T + R R-dot^T); D-dot <- chol_unblocked_fwd(D, D-dot);
    C-dot <- C-dot - B-dot R^T - B R-dot^T;  C-dot <- (C-dot - C D-dot^T) D^-T.
    """
    L = np.asarray(L, dtype=np.float64)
    Ad = np.tril(np.asarray(Adot, dtype=np.float64)).copy()
    for j, k in _blocks_forward(L.shape[0], nb):
        R, D, B, C = level3partition(L, j, k)
        Rd, Dd, Bd, Cd = level3partition(Ad, j, k)
        Dd[...] = Dd - np.tril(Rd @ R.T + R @ Rd.T)
        Dd[...] = chol_unblocked_fwd(D, Dd)
        Cd[...] = Cd - Bd @ R.T - B @ Rd.T
        Cd[...] = solve_triangular(D, (Cd - C @ np.tril(Dd).T).T, lower=True).T
    return np.tril(Ad)


def chol_blocked_rev(L, Abar, nb):
    """Sec. 4.2 chol_blocked_rev (blocks from the bottom-right; the short block is top-left):
    C-bar <- C-bar D^-1; B-bar <- B-bar - C-bar R; D-bar <- D-bar - tril(C-bar^T C);
    D-bar <- chol_unblocked_rev(D, D-bar); R-bar <- R-bar - C-bar^T B - (D-bar + D-bar^T) R.
    Output: T = tril(Sigma-bar) of eqn (symrevtril).
    """
    L = np.asarray(L, dtype=np.float64)
    Ab = np.tril(np.asarray(Abar, dtype=np.float64)).copy()
    N = L.shape[0]
    for k in range(N, 0, -nb):
        j = max(0, k - nb)
        R, D, B, C = level3partition(L, j, k)
        Rb, Db, Bb, Cb = level3partition(Ab, j, k)
        Cb[...] = solve_triangular(D, Cb.T, lower=True, trans=1).T   # C-bar D^-1
        Bb -= Cb @ R
        Db[...] = Db - np.tril(Cb.T @ C)
        Db[...] = chol_unblocked_rev(D, Db)
        Rb -= Cb.T @ B + (Db + Db.T) @ R
    return np.tril(Ab)


# --------------------------------------------------------------------------------------------
# The O(N^4) Jacobian of Sec. 3 (for N <= 8 only)
# --------------------------------------------------------------------------------------------

def vec(A):
    """Stack the columns of A (Sec. 3, before eqn (vec2kron))."""
    return np.asarray(A, dtype=np.float64).reshape(-1, order="F")


def _vech_pairs(N):
    """(row, col) of the lower-triangle entries in column-stacking order (Sec. 2, eqn (chainmat))."""
    return [(i, j) for j in range(N) for i in range(j, N)]


def vech(A):
    """Stack the lower-triangular part of each column of A (Sec. 2)."""
    A = np.asarray(A, dtype=np.float64)
    return np.array([A[i, j] for i, j in _vech_pairs(A.shape[0])])


def elimination_matrix(N):
    """The matrix with vech(A) = Lmat vec(A) for any A (Magnus & Neudecker; Sec. 3 before (bletch))."""
    pairs = _vech_pairs(N)
    E = np.zeros((len(pairs), N * N))
    for r, (i, j) in enumerate(pairs):
        E[r, j * N + i] = 1.0
    return E


def duplication_matrix(N):
    """The matrix with vec(A) = D vech(A) for symmetric A (Magnus & Neudecker; Sec. 3 before (bletch))."""
    pairs = _vech_pairs(N)
    Dm = np.zeros((N * N, len(pairs)))
    for c, (i, j) in enumerate(pairs):
        Dm[j * N + i, c] = 1.0
        Dm[i * N + j, c] = 1.0
    return Dm


def jacobian_delements(L):
    """d vech(L) / d vech(Sigma) entry by entry from eqn (delements) (Sec. 3).

    Row (i, j) with i >= j, column (k, l) with k >= l, both in vech order.  (L^-1)_mk is read as the
    (m, k) entry of the inverse.  Brute force; N <= 8 only.
    """
    L = np.asarray(L, dtype=np.float64)
    N = L.shape[0]
    Li = np.linalg.inv(L)
    pairs = _vech_pairs(N)
    J = np.zeros((len(pairs), len(pairs)))
    for r, (i, j) in enumerate(pairs):
        for c, (k, l) in enumerate(pairs):
            s_k = sum(L[i, m] * Li[m, k] for m in range(j + 1, N)) + 0.5 * L[i, j] * Li[j, k]
            s_l = sum(L[i, m] * Li[m, l] for m in range(j + 1, N)) + 0.5 * L[i, j] * Li[j, l]
            J[r, c] = s_k * Li[j, l] + (0.0 if k == l else 1.0) * s_l * Li[j, k]
    return J


def jacobian_bletch(L):
    """d vech(L) / d vech(Sigma) = Lmat (I kron L) Z (L^-1 kron L^-1) D  (eqn (bletch), Sec. 3).

    Z is the diagonal 0 / 1/2 / 1 selector with Z vec(A) = vec(Phi(A)).  N <= 8 only.
    """
    L = np.asarray(L, dtype=np.float64)
    N = L.shape[0]
    Li = np.linalg.inv(L)
    z = np.zeros(N * N)
    for j in range(N):
        for i in range(N):
            z[j * N + i] = 1.0 if i > j else (0.5 if i == j else 0.0)
    return (elimination_matrix(N) @ np.kron(np.eye(N), L) @ np.diag(z)
            @ np.kron(Li, Li) @ duplication_matrix(N))


# --------------------------------------------------------------------------------------------
# The Gaussian-process style loss used by the batched workload (Sec. 2's x -> Sigma -> L -> f)
# --------------------------------------------------------------------------------------------

def gp_loss_and_lbar(L, y):
    """f = sum_i log L_ii + (1/2)||L^-1 y||^2 and its L-bar = diag(1/L_ii) - tril(w z^T),
    z = L^-1 y, w = L^-T z (the reverse-mode sensitivity of f w.r.t. L, Sec. 2).
    """
    L = np.asarray(L, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = solve_triangular(L, y, lower=True)
    w = solve_triangular(L, z, lower=True, trans=1)
    f = float(np.sum(np.log(np.diag(L))) + 0.5 * z @ z)
    Lbar = np.diag(1.0 / np.diag(L)) - np.tril(np.outer(w, z))
    return f, Lbar
