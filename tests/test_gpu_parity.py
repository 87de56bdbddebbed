"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle, element by element.

Tolerance (relative Frobenius, FP64 path): 1e-10 for chol_rev / chol_fwd run on the SAME L as the
oracle, and for chol_factor on L itself.  Both sides are backward-stable FP64 computations of the
same quantity; their difference is rounding amplified by conditioning, measured at <= 3e-14 between
independent CPU routes on these inputs (kappa up to 8e6), so 1e-10 leaves >= 1000x headroom while
any indexing or algebra mistake gives O(1) errors.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from _golden import load

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as pkg
    pkg.load_library()            # fails loudly when the HIP library is missing
    return pkg


@pytest.fixture(scope="module")
def dev(cg):
    import torch
    return torch.device("cuda:0")


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def spd_case(N, seed):
    S, rng = W.dense_spd(N, seed)
    L = sla.cholesky(S, lower=True) if N > 0 else np.zeros((0, 0))
    Lb = W.lower_normal(N, rng)
    Sd = W.sym_normal(N, rng)
    junk = np.triu(rng.standard_normal((N, N)) * 1e3, 1)     # must be ignored
    return S, L, Lb, Sd, junk


SIZES = [1, 2, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256, 257, 383, 513]
NBS = [32, 64, 128]


@pytest.mark.parametrize("diag", ["auto", "level2"])
@pytest.mark.parametrize("nb", NBS)
@pytest.mark.parametrize("N", SIZES)
def test_rev_matches_oracle(cg, dev, N, nb, diag):
    S, L, Lb, Sd, junk = spd_case(N, 1000 + N)
    A = cg.chol_rev(to_dev(L, dev), to_dev(Lb + junk, dev), form="sym", nb=nb, diag=diag).cpu().numpy()
    want = O.chol_rev(L, Lb, "sym")
    assert rel(A, want) <= TOL
    assert np.array_equal(A, A.T)


@pytest.mark.parametrize("nb", [64, 128])
@pytest.mark.parametrize("N", [128, 300, 1000, 2048])
def test_rev_diagonal_variants_agree(cg, dev, N, nb):
    """chol_rev's diagonal-block adjoint variants, the symbolic form (products with the block
    inverse) and the Level-2 form (Sec. 4.1's unblocked sweep), match the oracle and each other to
    rounding, on the squared-exponential kernel (worse conditioned than spd_case)."""
    c = W.se_case(N, 4000 + N, 0.3, 1e-3, with_sdot=False)
    L = O.chol(c["Sigma"])[0]
    Lb = c["Lbar"]
    want = O.chol_rev(L, Lb, "sym")
    sym = cg.chol_rev(to_dev(L, dev), to_dev(Lb, dev), nb=nb, diag="symbolic").cpu().numpy()
    lev2 = cg.chol_rev(to_dev(L, dev), to_dev(Lb, dev), nb=nb, diag="level2").cpu().numpy()
    kappa = np.linalg.cond(c["Sigma"])
    print(f"N={N} kappa={kappa:.1e}: symbolic {rel(sym, want):.2e}  Level-2 {rel(lev2, want):.2e}  "
          f"between {rel(sym, lev2):.2e}")
    # both sides use the same L, so the FP64 gate holds whatever the conditioning of Sigma
    assert rel(sym, want) <= TOL and rel(lev2, want) <= TOL and rel(sym, lev2) <= TOL
    assert np.array_equal(sym, sym.T) and np.array_equal(lev2, lev2.T)


def test_both_variants_large_ragged(cg, dev):
    """Both diagonal-block variants of both sweeps at n = 8300, nb = 128 (ragged last block; the
    Level-2 sweeps' look-ahead splits of the trailing rows; junk in the ignored upper triangles)
    against the oracle."""
    N = 8300
    S, L, Lb, Sd, junk = spd_case(N, 6000)
    Lt = to_dev(L, dev)
    want_rev, want_fwd = O.chol_rev(L, Lb, "sym"), O.chol_fwd(L, Sd)
    for diag in ("symbolic", "level2"):
        A = cg.chol_rev(Lt, to_dev(Lb + junk, dev), nb=128, diag=diag).cpu().numpy()
        assert rel(A, want_rev) <= TOL, diag
        assert np.array_equal(A, A.T)
        D = cg.chol_fwd(Lt, to_dev(np.tril(Sd) + junk, dev), nb=128, diag=diag).cpu().numpy()
        assert rel(D, want_fwd) <= TOL, diag
        assert np.all(np.triu(D, 1) == 0)


@pytest.mark.parametrize("nb", [64, 128])
@pytest.mark.parametrize("N", [128, 300, 1000, 2048])
def test_fwd_diagonal_variants_agree(cg, dev, N, nb):
    """chol_fwd's diagonal-block variants (symbolic and Level-2) match the oracle and each other to
    rounding; the strict upper triangle is zero in both."""
    c = W.se_case(N, 5000 + N, 0.3, 1e-3)
    L = O.chol(c["Sigma"])[0]
    Sd = c["Sdot"]
    want = O.chol_fwd(L, Sd)
    sym = cg.chol_fwd(to_dev(L, dev), to_dev(np.tril(Sd), dev), nb=nb, diag="symbolic").cpu().numpy()
    lev2 = cg.chol_fwd(to_dev(L, dev), to_dev(np.tril(Sd), dev), nb=nb, diag="level2").cpu().numpy()
    kappa = np.linalg.cond(c["Sigma"])
    print(f"N={N} kappa={kappa:.1e}: symbolic {rel(sym, want):.2e}  Level-2 {rel(lev2, want):.2e}  "
          f"between {rel(sym, lev2):.2e}")
    # both sides use the same L, so the FP64 gate holds whatever the conditioning of Sigma
    assert rel(sym, want) <= TOL and rel(lev2, want) <= TOL and rel(sym, lev2) <= TOL
    assert np.all(np.triu(sym, 1) == 0) and np.all(np.triu(lev2, 1) == 0)


@pytest.mark.parametrize("N,nb", [(1, 32), (65, 32), (257, 64), (300, 128)])
def test_rev_tril_form(cg, dev, N, nb):
    S, L, Lb, Sd, junk = spd_case(N, 2000 + N)
    A = cg.chol_rev(to_dev(L, dev), to_dev(Lb + junk, dev), form="tril", nb=nb).cpu().numpy()
    assert rel(A, O.chol_rev(L, Lb, "tril")) <= TOL
    assert np.all(np.triu(A, 1) == 0)


@pytest.mark.parametrize("diag", ["auto", "level2"])
@pytest.mark.parametrize("nb", NBS)
@pytest.mark.parametrize("N", SIZES)
def test_fwd_matches_oracle(cg, dev, N, nb, diag):
    S, L, Lb, Sd, junk = spd_case(N, 3000 + N)
    A = cg.chol_fwd(to_dev(L, dev), to_dev(np.tril(Sd) + junk, dev), nb=nb, diag=diag).cpu().numpy()
    assert rel(A, O.chol_fwd(L, Sd)) <= TOL
    assert np.all(np.triu(A, 1) == 0)


@pytest.mark.parametrize("nb", NBS)
@pytest.mark.parametrize("N", SIZES)
def test_factor_matches_oracle(cg, dev, N, nb):
    S, L, Lb, Sd, junk = spd_case(N, 4000 + N)
    A, info = cg.chol_factor(to_dev(S + junk, dev), nb=nb)
    Lg = A.cpu().numpy()
    Lo, info_o = O.chol(S)
    assert int(info.item()) == 0 == info_o
    assert rel(Lg, Lo) <= TOL
    assert np.all(np.triu(Lg, 1) == 0)


@pytest.mark.parametrize("nb", NBS)
@pytest.mark.parametrize("N", SIZES)
def test_factor_fwd_one_sweep(cg, dev, N, nb):
    """chol_factor_fwd: L against the oracle's factor, L-dot against the oracle's forward propagation
    on the oracle's L (the sweep uses its own L: these matrices have condition number below 5, so
    the 1e-10 gate still holds end to end)."""
    S, L, Lb, Sd, junk = spd_case(N, 6000 + N)
    A, D, info = cg.chol_factor_fwd(to_dev(S + junk, dev), to_dev(np.tril(Sd) + junk, dev), nb=nb)
    assert int(info.item()) == 0
    Lg, Dg = A.cpu().numpy(), D.cpu().numpy()
    Lo = O.chol(S)[0]
    assert rel(Lg, Lo) <= TOL
    assert rel(Dg, O.chol_fwd(Lo, Sd)) <= TOL
    assert np.all(np.triu(Lg, 1) == 0) and np.all(np.triu(Dg, 1) == 0)


def test_factor_fwd_reports_bad_pivot(cg, dev):
    S, L, Lb, Sd, junk = spd_case(300, 6500)
    S[130, 130] = -1.0
    _, _, info = cg.chol_factor_fwd(to_dev(S, dev), to_dev(np.tril(Sd), dev), nb=128)
    assert int(info.item()) == O.chol(S)[1] == 131


@pytest.mark.parametrize("N,bad,nb", [(40, 0, 32), (40, 5, 32), (200, 64, 64), (200, 127, 64),
                                      (300, 299, 128), (300, 130, 128)])
def test_factor_reports_first_bad_pivot(cg, dev, N, bad, nb):
    S, *_ = spd_case(N, 5000 + N)
    S[bad, bad] = -1.0
    _, info_o = O.chol(S)
    A, info = cg.chol_factor(to_dev(S, dev), nb=nb)
    import torch
    torch.cuda.synchronize()
    assert info_o == bad + 1
    assert int(info.item()) == info_o


def test_empty_is_noop(cg, dev):
    import torch
    e = torch.zeros((0, 0), dtype=torch.float64, device=dev)
    cg.chol_rev(e, e.clone())
    cg.chol_fwd(e, e.clone())
    cg.chol_factor(e.clone())


def test_golden_integer_cases(cg, dev):
    g = load("chol_int.txt")
    A, info = cg.chol_factor(to_dev(g["Sigma"], dev), nb=32)
    assert int(info.item()) == 0
    assert np.abs(A.cpu().numpy() - g["L"]).max() <= 1e-14
    g = load("rev_closed.txt")
    A = cg.chol_rev(to_dev(g["L"], dev), to_dev(g["Lbar"], dev), nb=32).cpu().numpy()
    assert np.abs(A - g["Sbar_sym"]).max() <= 1e-13
    g = load("fwd_closed.txt")
    A = cg.chol_fwd(to_dev(g["L"], dev), to_dev(g["Sdot"], dev), nb=32).cpu().numpy()
    assert np.abs(A - g["Ldot"]).max() <= 1e-13


def test_small_case_identities(cg, dev):
    """N = 256 dense case: adjoint identity between the GPU's own rev and fwd, and central finite
    differences of the GPU factorisation against the GPU forward mode."""
    c = W.small_case()
    S, Lb, Sd = c["Sigma"], c["Lbar"], c["Sdot"]
    A, info = cg.chol_factor(to_dev(S, dev), nb=64)
    L = A.cpu().numpy()
    Sb = cg.chol_rev(to_dev(L, dev), to_dev(Lb, dev), nb=64).cpu().numpy()
    Ld = cg.chol_fwd(to_dev(L, dev), to_dev(np.tril(Sd), dev), nb=64).cpu().numpy()
    lhs = np.sum(Lb * Ld)
    assert np.sum(Sb * Sd) == pytest.approx(lhs, rel=1e-12)
    h = 1e-6
    Lp = cg.chol_factor(to_dev(S + h / 2 * Sd, dev), nb=64)[0].cpu().numpy()
    Lm = cg.chol_factor(to_dev(S - h / 2 * Sd, dev), nb=64)[0].cpu().numpy()
    assert rel((Lp - Lm) / h, Ld) <= 1e-6


@pytest.fixture(scope="module")
def medium():
    c = W.medium_case()
    L, info = O.chol(c["Sigma"])
    assert info == 0
    c["L"] = L
    c["rev"] = O.chol_rev(L, c["Lbar"], "sym")
    c["fwd"] = O.chol_fwd(L, c["Sdot"])
    return c


def test_medium_case_one_sweep(cg, dev, medium):
    """N = 4096 (kappa ~ 8e6) through chol_factor_fwd: L at 1e-10; L-dot, computed with the
    sweep's own L, at the end-to-end gate max(1e-10, 100 kappa u) ~ 1e-7."""
    A, D, info = cg.chol_factor_fwd(to_dev(medium["Sigma"], dev), to_dev(np.tril(medium["Sdot"]), dev), nb=128)
    assert int(info.item()) == 0
    assert rel(A.cpu().numpy(), medium["L"]) <= TOL
    assert rel(D.cpu().numpy(), medium["fwd"]) <= 1e-7


@pytest.mark.parametrize("nb", NBS)
def test_medium_case(cg, dev, medium, nb):
    """N = 4096 squared-exponential kernel (kappa ~ 8e6): factor, and rev/fwd on the oracle's L with
    both diagonal-block variants."""
    A, info = cg.chol_factor(to_dev(medium["Sigma"], dev), nb=nb)
    assert int(info.item()) == 0
    assert rel(A.cpu().numpy(), medium["L"]) <= TOL
    Lt = to_dev(medium["L"], dev)
    for diag in ("auto", "level2"):
        Sb = cg.chol_rev(Lt, to_dev(medium["Lbar"], dev), nb=nb, diag=diag).cpu().numpy()
        assert rel(Sb, medium["rev"]) <= TOL, diag
        Ld = cg.chol_fwd(Lt, to_dev(np.tril(medium["Sdot"]), dev), nb=nb, diag=diag).cpu().numpy()
        assert rel(Ld, medium["fwd"]) <= TOL, diag


def test_repeatable_bitwise(cg, dev):
    S, L, Lb, Sd, junk = spd_case(700, 77)
    Lt = to_dev(L, dev)
    a = cg.chol_rev(Lt, to_dev(Lb, dev)).cpu().numpy()
    b = cg.chol_rev(Lt, to_dev(Lb, dev)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("N,nb", [(1, 32), (65, 32), (257, 64), (300, 128), (513, 128)])
def test_col_major_layout(cg, dev, N, nb):
    """layout='col': the same sweeps on column-major (LAPACK) storage.  The logical lower triangle
    of each input is read (junk in the logical strict upper triangles, L's included, is ignored),
    L is not modified, and the logical results match the oracle: L and L-dot lower triangular with
    a zero strict upper triangle, Sigma-bar in both forms."""
    S, L, Lb, Sd, junk = spd_case(N, 7000 + N)

    def col(x):  # column-major tensor holding the logical matrix x
        return to_dev(x, dev).T.contiguous().T

    A = col(S + junk)
    cg.chol_factor(A, nb=nb, layout="col")
    Lg = A.cpu().numpy()
    assert rel(Lg, O.chol(S)[0]) <= TOL
    assert np.all(np.triu(Lg, 1) == 0)
    Lc = col(L + junk)
    L_before = Lc.cpu().numpy()
    for form in ("sym", "tril"):
        X = col(Lb + junk)
        cg.chol_rev(Lc, X, form=form, nb=nb, layout="col")
        assert rel(X.cpu().numpy(), O.chol_rev(L, Lb, form)) <= TOL, form
    X = col(np.tril(Sd) + junk)
    cg.chol_fwd(Lc, X, nb=nb, layout="col")
    Xg = X.cpu().numpy()
    assert rel(Xg, O.chol_fwd(L, Sd)) <= TOL
    assert np.all(np.triu(Xg, 1) == 0)
    assert np.array_equal(Lc.cpu().numpy(), L_before)


def test_col_major_rejects_row_major_tensors(cg, dev):
    A = to_dev(np.eye(8), dev)
    with pytest.raises(ValueError, match="column-major"):
        cg.chol_factor(A, layout="col")


WIDE_NBS = [16, 48, 80, 144, 192, 256]
WIDE_SIZES = [1, 17, 129, 255, 256, 257, 300, 513, 700]


@pytest.mark.parametrize("nb", WIDE_NBS)
@pytest.mark.parametrize("N", WIDE_SIZES)
def test_block_widths(cg, dev, N, nb):
    """Block widths beyond {32, 64, 128}: multiples of 16 below 128 (ragged inner blocks of the
    diagonal routines) and 144..256, whose diagonal blocks are factored and inverted as two halves.
    Factor, rev (both forms), fwd and the one-sweep factor + fwd against the oracle at 1e-10."""
    S, L, Lb, Sd, junk = spd_case(N, 8000 + N + nb)
    A, info = cg.chol_factor(to_dev(S + junk, dev), nb=nb)
    assert int(info.item()) == 0
    Lg = A.cpu().numpy()
    assert rel(Lg, O.chol(S)[0]) <= TOL and np.all(np.triu(Lg, 1) == 0)
    Lt = to_dev(L, dev)
    for form in ("sym", "tril"):
        X = cg.chol_rev(Lt, to_dev(Lb + junk, dev), form=form, nb=nb).cpu().numpy()
        assert rel(X, O.chol_rev(L, Lb, form)) <= TOL, form
    D = cg.chol_fwd(Lt, to_dev(np.tril(Sd) + junk, dev), nb=nb).cpu().numpy()
    assert rel(D, O.chol_fwd(L, Sd)) <= TOL and np.all(np.triu(D, 1) == 0)
    A2, D2, info = cg.chol_factor_fwd(to_dev(S + junk, dev), to_dev(np.tril(Sd) + junk, dev), nb=nb)
    assert int(info.item()) == 0
    assert rel(A2.cpu().numpy(), O.chol(S)[0]) <= TOL and rel(D2.cpu().numpy(), O.chol_fwd(L, Sd)) <= TOL


@pytest.mark.parametrize("N,bad,nb", [(300, 100, 256), (300, 200, 256), (300, 299, 256), (600, 400, 192)])
def test_wide_block_reports_first_bad_pivot(cg, dev, N, bad, nb):
    """A non-positive pivot in either half of a wide diagonal block is reported 1-based, as LAPACK."""
    S, *_ = spd_case(N, 5100 + bad)
    S[bad, bad] = -1.0
    _, info_o = O.chol(S)
    A, info = cg.chol_factor(to_dev(S, dev), nb=nb)
    assert info_o == bad + 1 and int(info.item()) == info_o


def test_level2_wide_block_unsupported(cg, dev):
    S, L, Lb, Sd, junk = spd_case(300, 8100)
    with pytest.raises(cg.CholError, match="-103"):
        cg.chol_rev(to_dev(L, dev), to_dev(Lb, dev), nb=256, diag="level2")
    with pytest.raises(cg.CholError, match="-103"):
        cg.chol_fwd(to_dev(L, dev), to_dev(np.tril(Sd), dev), nb=192, diag="level2")


def test_medium_case_nb256(cg, dev, medium):
    """The N = 4096 workload (kappa ~ 8e6) at nb = 256: factor at 1e-10 against the oracle's L,
    rev and fwd on the oracle's L at 1e-10, and the one-sweep factor + fwd (its own L, end-to-end
    gate max(1e-10, 100 kappa u))."""
    A, info = cg.chol_factor(to_dev(medium["Sigma"], dev), nb=256)
    assert int(info.item()) == 0
    assert rel(A.cpu().numpy(), medium["L"]) <= TOL
    Lt = to_dev(medium["L"], dev)
    Sb = cg.chol_rev(Lt, to_dev(medium["Lbar"], dev), nb=256).cpu().numpy()
    assert rel(Sb, medium["rev"]) <= TOL
    Ld = cg.chol_fwd(Lt, to_dev(np.tril(medium["Sdot"]), dev), nb=256).cpu().numpy()
    assert rel(Ld, medium["fwd"]) <= TOL
    A2, D2, info = cg.chol_factor_fwd(to_dev(medium["Sigma"], dev), to_dev(np.tril(medium["Sdot"]), dev), nb=256)
    assert int(info.item()) == 0
    assert rel(A2.cpu().numpy(), medium["L"]) <= TOL
    assert rel(D2.cpu().numpy(), medium["fwd"]) <= 1e-7


@pytest.mark.parametrize("n", [200, 300, 1000, 3100])
def test_automatic_block_width(cg, dev, n):
    """nb = 0 takes the width measured per sweep and size -- chol_rev and chol_fwd 256,
    chol_factor and chol_factor_fwd 256 for 256 < n <= 512 and n >= 3072, 128 otherwise, at
    most 128 with the Level-2 diagonal variant -- so its results are bitwise those of the
    explicit call, and the reverse sweep meets the oracle (eqn (symrev)) at 1e-10."""
    import torch
    S, L, Lb, Sd, _ = spd_case(n, 8200 + n)
    fac_nb = 256 if (256 < n <= 512 or n >= 3072) else 128
    A0, i0 = cg.chol_factor(to_dev(S, dev), nb=0)
    A1, i1 = cg.chol_factor(to_dev(S, dev), nb=fac_nb)
    assert int(i0.item()) == 0 and int(i1.item()) == 0 and torch.equal(A0, A1)
    Ld, Lbd, Sdd = to_dev(L, dev), to_dev(Lb, dev), to_dev(np.tril(Sd), dev)
    r0 = cg.chol_rev(Ld, Lbd.clone(), nb=0)
    assert torch.equal(r0, cg.chol_rev(Ld, Lbd.clone(), nb=256))
    assert rel(r0.cpu().numpy(), O.chol_rev(L, Lb)) < TOL
    assert torch.equal(cg.chol_fwd(Ld, Sdd.clone(), nb=0), cg.chol_fwd(Ld, Sdd.clone(), nb=256))
    for fn, src in ((cg.chol_rev, Lbd), (cg.chol_fwd, Sdd)):
        assert torch.equal(fn(Ld, src.clone(), nb=0, diag="level2"), fn(Ld, src.clone(), nb=128, diag="level2"))
    F0 = cg.chol_factor_fwd(to_dev(S, dev), Sdd.clone(), nb=0)
    F1 = cg.chol_factor_fwd(to_dev(S, dev), Sdd.clone(), nb=fac_nb)
    assert torch.equal(F0[0], F1[0]) and torch.equal(F0[1], F1[1])
