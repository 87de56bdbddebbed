"""Writes the integer fixtures in this folder.  Inputs are built with exact integer arithmetic from
matrices chosen by hand; the expected values follow from the mathematics (no library computes them):
  chol_int.txt     Sec. 1: L is the unique lower-triangular factor with positive diagonal of L L^T.
  rev_closed.txt   Sec. 2/3: for f = Tr(C Sigma) = Tr(C L L^T), dF/dL = 2 C L, so the reverse-mode
                   input L-bar = tril(2 C L) must give the symmetric gradient Sigma-bar = C.
  fwd_closed.txt   Sec. 3, eqn (symfwd): Sigma-dot = M L^T + L M^T with M lower gives L-dot = M.
  gp_int.txt       Sec. 2's x -> Sigma -> L -> f chain with the Gaussian-process loss
                   f = sum_i log L_ii + |L^-1 y|^2 / 2: y = L L^T w0 with w0 integer makes
                   z = L^-1 y = L^T w0 and w = L^-T z = w0 integers, so f = log(prod_i L_ii) + z.z / 2
                   and L-bar = diag(1 / L_ii) - tril(w z^T) follow by hand.
Run:  python tests/golden/make_golden.py
"""
import os
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
L = np.array([[2, 0, 0, 0, 0], [1, 3, 0, 0, 0], [-1, 2, 1, 0, 0], [3, 0, -2, 4, 0],
              [0, 1, 1, -1, 2]], dtype=np.int64)
C = np.array([[1, 2, 0, -1, 3], [2, -3, 1, 0, 0], [0, 1, 2, 1, -2], [-1, 0, 1, 0, 1],
              [3, 0, -2, 1, 4]], dtype=np.int64)
W0 = np.array([1, -2, 0, 3, -1], dtype=np.int64)
M = np.array([[1, 0, 0, 0, 0], [-2, 3, 0, 0, 0], [0, 1, -1, 0, 0], [2, 2, 0, 1, 0],
              [1, -1, 3, 0, -2]], dtype=np.int64)
assert (C == C.T).all() and (np.triu(L, 1) == 0).all() and (np.triu(M, 1) == 0).all()


def dump(name, header, arrays):
    with open(os.path.join(HERE, name), "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for key, A in arrays:
            f.write(f"{key} {A.shape[0]} {A.shape[1]}\n")
            for row in A:
                f.write(" ".join(str(int(v)) for v in row) + "\n")


dump("chol_int.txt",
     ["Sec. 1 definition: L lower-triangular, positive diagonal, L L^T = Sigma.",
      "Sigma = L L^T in exact integers; chol(Sigma) must return L."],
     [("Sigma", L @ L.T), ("L", L)])
dump("rev_closed.txt",
     ["Sec. 2-3: f = Tr(C Sigma) with C symmetric has dF/dL = 2 C L.",
      "chol_rev(L, tril(2 C L)) must return the symmetric gradient C."],
     [("L", L), ("Lbar", np.tril(2 * C @ L)), ("Sbar_sym", C)])
dump("fwd_closed.txt",
     ["Sec. 3 eqn (symfwd): Sigma-dot = M L^T + L M^T with M lower-triangular gives L-dot = M."],
     [("L", L), ("Sdot", M @ L.T + L @ M.T), ("Ldot", M)])
dump("gp_int.txt",
     ["Sec. 2 chain with f = sum log L_ii + |L^-1 y|^2 / 2; y = L L^T w0 (w0 integer), so",
      "z = L^-1 y = L^T w0 and w = L^-T z = w0 exactly: f = log(prod L_ii) + z.z / 2,",
      "L-bar = diag(1 / L_ii) - tril(w z^T)."],
     [("L", L), ("y", (L @ L.T @ W0)[:, None]), ("z", (L.T @ W0)[:, None]), ("w", W0[:, None])])
