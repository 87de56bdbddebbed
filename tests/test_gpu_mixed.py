"""GPU tests of the reduced-precision single-matrix modes, FP64 storage with the trailing
contractions on FP32 MFMA ('f64_trail_f32', CHOL_PREC_F64_TRAIL_F32) or as split-bfloat16 products
('f64_trail_bf16x3', CHOL_PREC_F64_TRAIL_BF16X3); diagonal blocks and panel solves stay FP64.

These modes approximate the FP64 result, so the bar is a stated relative Frobenius tolerance per
result against the FP64 oracle (rev and fwd on the oracle's own L, so only the mode's error is
measured), on the squared-exponential workloads (N = 4096 and the full N = 16384, condition
numbers ~3e4 and ~1e5):

    f64_trail_f32     relL <= 3e-4, rel Sigma-bar <= 1e-4, rel L-dot <= 3e-5
    f64_trail_bf16x3  relL <= 1e-3, rel Sigma-bar <= 3e-4, rel L-dot <= 3e-4
    f64_trail_bf16x6  relL <= 5e-4, rel Sigma-bar <= 2e-4, rel L-dot <= 3e-5

The Sigma-bar and L-dot bounds are about 10x the largest error measured on MI355X (N = 16384:
FP32 trailing relL 7.6e-5, rel Sigma-bar 7.1e-6, rel L-dot 2.6e-6; split-bf16 relL 3.0e-4,
rel Sigma-bar 2.3e-5, rel L-dot 2.1e-5; split-bf16 x6 relL 4.6e-5, rel Sigma-bar 2.0e-5,
rel L-dot 1.9e-6), so a 10x loss of accuracy fails them; the relL bounds
keep a 3-4x margin over the factor's measured error, which grows with N.  Every result must also
differ from the oracle by more than 1e-9 (the FP64 path is ~1e-13 away), which shows the
reduced-precision kernels really ran.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
TOLS = {"f64_trail_f32": (3e-4, 1e-4, 3e-5), "f64_trail_bf16x3": (1e-3, 3e-4, 3e-4),
        "f64_trail_bf16x6": (5e-4, 2e-4, 3e-5)}
MODES = list(TOLS)
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


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("nb", [64, 128])
def test_mixed_n4096(cg, se4096, nb, mode):
    c = se4096
    tol_l, tol_s, tol_d = TOLS[mode]
    A, info = cg.chol_factor(to_dev(c["Sigma"]), nb=nb, precision=mode)
    assert int(info.item()) == 0
    eL = rel(A.cpu().numpy(), c["L"])
    Lt = to_dev(c["L"])
    eS = rel(cg.chol_rev(Lt, to_dev(c["Lbar"]), nb=nb, precision=mode).cpu().numpy(), c["rev"])
    eD = rel(cg.chol_fwd(Lt, to_dev(np.tril(c["Sdot"])), nb=nb, precision=mode).cpu().numpy(), c["fwd"])
    print(f"{mode} N=4096 nb={nb}: relL {eL:.2e}  rel Sigma-bar {eS:.2e}  rel L-dot {eD:.2e}")
    assert FLOOR < eL <= tol_l
    assert FLOOR < eS <= tol_s
    assert FLOOR < eD <= tol_d


@pytest.mark.parametrize("mode", MODES)
def test_mixed_ragged_and_tril_form(cg, mode):
    """Ragged sizes take the guarded kernels for their edge contractions; the 'tril' output form
    and the zero strict upper triangles behave as in FP64."""
    tol_l, tol_s, tol_d = TOLS[mode]
    for n in (1, 300, 1000):
        S, rng = W.dense_spd(n, 2000 + n)
        Lb, Sd = W.lower_normal(n, rng), W.sym_normal(n, rng)
        L = O.chol(S)[0]
        A, info = cg.chol_factor(to_dev(S), nb=128, precision=mode)
        assert int(info.item()) == 0
        Lg = A.cpu().numpy()
        assert rel(Lg, L) <= tol_l and np.all(np.triu(Lg, 1) == 0)
        T = cg.chol_rev(to_dev(L), to_dev(Lb), form="tril", nb=128, precision=mode).cpu().numpy()
        assert rel(T, O.chol_rev(L, Lb, "tril")) <= tol_s and np.all(np.triu(T, 1) == 0)
        D = cg.chol_fwd(to_dev(L), to_dev(np.tril(Sd)), nb=128, precision=mode).cpu().numpy()
        assert rel(D, O.chol_fwd(L, Sd)) <= tol_d and np.all(np.triu(D, 1) == 0)
        A2, D2, info = cg.chol_factor_fwd(to_dev(S), to_dev(np.tril(Sd)), nb=128, precision=mode)
        assert int(info.item()) == 0
        assert rel(A2.cpu().numpy(), L) <= tol_l and rel(D2.cpu().numpy(), O.chol_fwd(L, Sd)) <= tol_d


@pytest.fixture(scope="module")
def full16384():
    """The benchmark's N = 16384 workload on the device and the oracle's results (host LAPACK route)."""
    import torch
    dev = torch.device("cuda:0")
    inp = W.large_case_device(dev, N=16384)
    L = O.chol_host(inp["Sigma"].cpu().numpy())
    rev = O.chol_rev(L, inp["Lbar"].cpu().numpy(), "sym")
    fwd = O.chol_fwd(L, inp["Sdot"].cpu().numpy())
    return {"inp": inp, "L": L, "rev": rev, "fwd": fwd}


@pytest.mark.parametrize("mode", ["f64"] + MODES)
def test_mixed_full_size_n16384(cg, full16384, mode):
    """The benchmark's N = 16384 workload: factor, rev and fwd in FP64 (1e-10 element-wise against
    the oracle: rev and fwd on the oracle's L) and in the reduced-precision modes, against the
    oracle on the same device-built inputs."""
    inp, L = full16384["inp"], full16384["L"]
    tol_l, tol_s, tol_d = TOLS.get(mode, (1e-10, 1e-10, 1e-10))
    floor = FLOOR if mode in TOLS else 0.0
    A, info = cg.chol_factor(inp["Sigma"].clone(), nb=128, precision=mode)
    assert int(info.item()) == 0
    eL = rel(A.cpu().numpy(), L)
    del A
    Lt = to_dev(L)
    eS = rel(cg.chol_rev(Lt, inp["Lbar"].clone(), nb=128, precision=mode).cpu().numpy(), full16384["rev"])
    eD = rel(cg.chol_fwd(Lt, inp["Sdot"].clone(), nb=128, precision=mode).cpu().numpy(), full16384["fwd"])
    print(f"{mode} N=16384 nb=128: relL {eL:.2e}  rel Sigma-bar {eS:.2e}  rel L-dot {eD:.2e}")
    assert floor <= eL <= tol_l
    assert floor <= eS <= tol_s
    assert floor <= eD <= tol_d
