"""GPU tests of the reduced-precision single-matrix mode 'f64_trail_f32' (CHOL_PREC_F64_TRAIL_F32):
FP64 storage, trailing contractions on FP32 MFMA, diagonal blocks and panel solves in FP64.

This mode is an approximation of the FP64 result, not an exact reorganisation, so its bar is a
stated relative Frobenius tolerance per result against the FP64 oracle (for rev and fwd on the
oracle's own L, so only the mode's error is measured):

    relL <= 3e-4,   rel Sigma-bar <= 3e-3,   rel L-dot <= 3e-3

on the squared-exponential workloads (N = 4096 and the full N = 16384, condition numbers ~3e4 and
~1e5); a CPU emulation of the same rounding measured 3.5e-5 / 3.4e-4 at N = 4096 and
7.6e-5 / 8.2e-4 at N = 16384.  Every result must also differ from the oracle by more than 1e-9
(the FP64 path is ~1e-13 away), which shows the reduced-precision kernels really ran.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
MODE = "f64_trail_f32"
TOL_L, TOL_SBAR, TOL_LDOT = 3e-4, 3e-3, 3e-3
FLOOR = 1e-9


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as pkg
    pkg.load_library()
    return pkg


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.fixture(scope="module")
def se4096():
    c = W.se_case(4096, W.SEED_LARGE, 0.2, 1e-2)
    L, info = O.chol(c["Sigma"])
    assert info == 0
    c["L"] = L
    c["rev"] = O.chol_rev(L, c["Lbar"], "sym")
    c["fwd"] = O.chol_fwd(L, c["Sdot"])
    return c


@pytest.mark.parametrize("nb", [64, 128])
def test_mixed_n4096(cg, se4096, nb):
    c = se4096
    A, info = cg.chol_factor(to_dev(c["Sigma"]), nb=nb, precision=MODE)
    assert int(info.item()) == 0
    eL = rel(A.cpu().numpy(), c["L"])
    Lt = to_dev(c["L"])
    eS = rel(cg.chol_rev(Lt, to_dev(c["Lbar"]), nb=nb, precision=MODE).cpu().numpy(), c["rev"])
    eD = rel(cg.chol_fwd(Lt, to_dev(np.tril(c["Sdot"])), nb=nb, precision=MODE).cpu().numpy(), c["fwd"])
    print(f"N=4096 nb={nb}: relL {eL:.2e}  rel Sigma-bar {eS:.2e}  rel L-dot {eD:.2e}")
    assert FLOOR < eL <= TOL_L
    assert FLOOR < eS <= TOL_SBAR
    assert FLOOR < eD <= TOL_LDOT


def test_mixed_ragged_and_tril_form(cg):
    """Ragged sizes take the guarded kernels for their edge contractions; the 'tril' output form
    and the zero strict upper triangles behave as in FP64."""
    for n in (1, 300, 1000):
        S, rng = W.dense_spd(n, 2000 + n)
        Lb, Sd = W.lower_normal(n, rng), W.sym_normal(n, rng)
        L = O.chol(S)[0]
        A, info = cg.chol_factor(to_dev(S), nb=128, precision=MODE)
        assert int(info.item()) == 0
        Lg = A.cpu().numpy()
        assert rel(Lg, L) <= TOL_L and np.all(np.triu(Lg, 1) == 0)
        T = cg.chol_rev(to_dev(L), to_dev(Lb), form="tril", nb=128, precision=MODE).cpu().numpy()
        assert rel(T, O.chol_rev(L, Lb, "tril")) <= TOL_SBAR and np.all(np.triu(T, 1) == 0)
        D = cg.chol_fwd(to_dev(L), to_dev(np.tril(Sd)), nb=128, precision=MODE).cpu().numpy()
        assert rel(D, O.chol_fwd(L, Sd)) <= TOL_LDOT and np.all(np.triu(D, 1) == 0)


def test_mixed_full_size_n16384(cg):
    """The benchmark's N = 16384 workload: factor, rev and fwd in the reduced-precision mode
    against the oracle (host LAPACK route) on the same device-built inputs."""
    import torch
    dev = torch.device("cuda:0")
    inp = W.large_case_device(dev, N=16384)
    Sig = inp["Sigma"].cpu().numpy()
    L = O.chol_host(Sig)
    A, info = cg.chol_factor(inp["Sigma"].clone(), nb=128, precision=MODE)
    assert int(info.item()) == 0
    eL = rel(A.cpu().numpy(), L)
    del A, Sig
    Lt = to_dev(L)
    Lbar = inp["Lbar"].cpu().numpy()
    Sb = cg.chol_rev(Lt, inp["Lbar"].clone(), nb=128, precision=MODE).cpu().numpy()
    eS = rel(Sb, O.chol_rev(L, Lbar, "sym"))
    del Sb, Lbar
    Sd = inp["Sdot"].cpu().numpy()
    Ld = cg.chol_fwd(Lt, inp["Sdot"].clone(), nb=128, precision=MODE).cpu().numpy()
    eD = rel(Ld, O.chol_fwd(L, Sd))
    print(f"N=16384 nb=128: relL {eL:.2e}  rel Sigma-bar {eS:.2e}  rel L-dot {eD:.2e}")
    assert FLOOR < eL <= TOL_L
    assert FLOOR < eS <= TOL_SBAR
    assert FLOOR < eD <= TOL_LDOT
