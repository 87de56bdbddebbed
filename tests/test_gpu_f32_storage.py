"""FP32 storage of the single-matrix calls ('f32': float32 tensors, computed in FP64 on copies inside
the library and rounded to float once on output; 'f32_trail_bf16x3': the same with split-bfloat16
trailing contractions).  Against the FP64 oracle run on the same float inputs widened to FP64, the
'f32' results differ only by that final rounding: relative Frobenius error at most 2^-24 plus the
FP64 gate, so F32_SAME = 1e-7.  'f32_trail_bf16x3' is held to the split-bf16 mode's stated bounds
on the N = 4096 squared-exponential workload."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
F32_SAME = 1e-7


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as pkg
    pkg.load_library()
    return pkg


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def f32(x):
    return np.asarray(x, dtype=np.float32)


def to_dev(x, layout="row"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    return t.T.contiguous().T if layout == "col" else t


def back(t):
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("nb", [64, 128, 256])
@pytest.mark.parametrize("N", [1, 17, 100, 257, 600])
def test_f32_storage_matches_oracle(cg, N, nb, layout):
    S, rng = W.dense_spd(N, 9300 + N)
    Lb, Sd = W.lower_normal(N, rng), W.sym_normal(N, rng)
    junk = np.triu(rng.standard_normal((N, N)) * 1e3, 1)
    Sf, Lbf, Sdf = f32(S), f32(Lb), f32(np.tril(Sd))
    Sw = Sf.astype(np.float64)
    Lo = O.chol(Sw)[0]                                       # the oracle on the float input
    A = to_dev(f32(Sf + junk), layout)
    A, info = cg.chol_factor(A, nb=nb, precision="f32", layout=layout)
    assert int(info.item()) == 0
    Lg = back(A)
    assert rel(Lg, Lo) <= F32_SAME and np.all(np.triu(Lg, 1) == 0)
    Lf = f32(Lo)                                              # a float factor for rev / fwd
    Lw = Lf.astype(np.float64)
    Lt = to_dev(f32(Lf + junk), layout)
    for form in ("sym", "tril"):
        X = cg.chol_rev(Lt, to_dev(f32(Lbf + junk), layout), form=form, nb=nb, precision="f32", layout=layout)
        assert rel(back(X), O.chol_rev(Lw, Lbf.astype(np.float64), form)) <= F32_SAME, form
    D = cg.chol_fwd(Lt, to_dev(f32(Sdf + junk), layout), nb=nb, precision="f32", layout=layout)
    Sd_w = Sdf.astype(np.float64)
    Dg = back(D)
    assert rel(Dg, O.chol_fwd(Lw, Sd_w)) <= F32_SAME and np.all(np.triu(Dg, 1) == 0)
    if layout == "row":
        A2, D2, info = cg.chol_factor_fwd(to_dev(f32(Sf + junk)), to_dev(f32(Sdf + junk)), nb=nb, precision="f32")
        assert int(info.item()) == 0
        assert rel(back(A2), Lo) <= F32_SAME
        assert rel(back(D2), O.chol_fwd(Lo, Sd_w)) <= F32_SAME


def test_f32_storage_split_bf16_n4096(cg):
    """'f32_trail_bf16x3' on the N = 4096 squared-exponential workload (lengthscale 0.2): within the
    split-bf16 mode's stated bounds of the oracle on the float inputs, and visibly different from
    the 'f32' result (the reduced kernels ran)."""
    c = W.se_case(4096, W.SEED_LARGE, 0.2, 1e-2)
    Sf, Lbf, Sdf = f32(c["Sigma"]), f32(c["Lbar"]), f32(np.tril(c["Sdot"]))
    Lo = O.chol(Sf.astype(np.float64))[0]
    Lf = f32(Lo)
    Lw = Lf.astype(np.float64)
    want_s = O.chol_rev(Lw, Lbf.astype(np.float64))
    want_d = O.chol_fwd(Lw, Sdf.astype(np.float64))
    out = {}
    for mode in ("f32", "f32_trail_bf16x3"):
        A, info = cg.chol_factor(to_dev(Sf), nb=128, precision=mode)
        assert int(info.item()) == 0
        S_ = back(cg.chol_rev(to_dev(Lf), to_dev(Lbf), nb=128, precision=mode))
        D_ = back(cg.chol_fwd(to_dev(Lf), to_dev(Sdf), nb=128, precision=mode))
        out[mode] = (rel(back(A), Lo), rel(S_, want_s), rel(D_, want_d))
        print(f"{mode} N=4096: relL {out[mode][0]:.2e}  rel Sigma-bar {out[mode][1]:.2e}  rel L-dot {out[mode][2]:.2e}")
    assert max(out["f32"]) <= F32_SAME
    eL, eS, eD = out["f32_trail_bf16x3"]
    assert 1e-6 < eL <= 1e-3 and 1e-7 < eS <= 3e-4 and 1e-7 < eD <= 3e-4
