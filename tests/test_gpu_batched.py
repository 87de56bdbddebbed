"""GPU parity of the one-launch batched forms against the FP64 oracle.

Tolerance 1e-10 relative Frobenius per problem, as for the single-matrix calls (same algorithms,
same L as the oracle for rev/fwd).  The Gaussian-process mode is checked against the oracle's loss
and reverse sweep, and against the closed form Sigma-bar = (Sigma^-1 - a a^T)/2, a = Sigma^-1 y.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10
SIZES = [1, 2, 16, 31, 64, 100, 128, 129, 200, 256, 257, 300, 384, 511, 512, 7, 130, 255]


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as pkg
    pkg.load_library()
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


def problems(sizes, seed):
    out = []
    for i, n in enumerate(sizes):
        S, rng = W.dense_spd(n, seed + 17 * i)
        L = sla.cholesky(S, lower=True)
        out.append({"S": S, "L": L, "Lb": W.lower_normal(n, rng), "Sd": W.sym_normal(n, rng),
                    "y": rng.standard_normal(n),
                    "junk": np.triu(rng.standard_normal((n, n)) * 1e3, 1)})
    return out


def test_factor_batched(cg, dev):
    P = problems(SIZES, 100)
    mats = [to_dev(p["S"] + p["junk"], dev) for p in P]
    info = cg.chol_factor_batched(mats)
    assert info.cpu().tolist() == [0] * len(P)
    for p, m in zip(P, mats):
        Lg = m.cpu().numpy()
        Lo, _ = O.chol(p["S"])
        assert rel(Lg, Lo) <= TOL
        assert np.all(np.triu(Lg, 1) == 0)


@pytest.mark.parametrize("form", ["sym", "tril"])
def test_rev_batched(cg, dev, form):
    P = problems(SIZES, 200)
    Ls = [to_dev(p["L"], dev) for p in P]
    As = [to_dev(p["Lb"] + p["junk"], dev) for p in P]
    cg.chol_rev_batched(Ls, As, form=form)
    for p, a in zip(P, As):
        assert rel(a.cpu().numpy(), O.chol_rev(p["L"], p["Lb"], form)) <= TOL


def test_fwd_batched(cg, dev):
    P = problems(SIZES, 300)
    Ls = [to_dev(p["L"], dev) for p in P]
    As = [to_dev(np.tril(p["Sd"]) + p["junk"], dev) for p in P]
    cg.chol_fwd_batched(Ls, As)
    for p, a in zip(P, As):
        got = a.cpu().numpy()
        assert rel(got, O.chol_fwd(p["L"], p["Sd"])) <= TOL
        assert np.all(np.triu(got, 1) == 0)


def test_gp_batched(cg, dev):
    import torch
    P = problems(SIZES, 400)
    As = [to_dev(p["S"], dev) for p in P]
    Gs = [torch.empty_like(a) for a in As]
    ys = [to_dev(p["y"], dev) for p in P]
    f, info = cg.chol_gp_nll_batched(As, ys, Gs)
    assert info.cpu().tolist() == [0] * len(P)
    f = f.cpu().numpy()
    for i, (p, g) in enumerate(zip(P, Gs)):
        Lo, _ = O.chol(p["S"])
        fo, Lbar = O.gp_loss_and_lbar(Lo, p["y"])
        assert f[i] == pytest.approx(fo, rel=1e-11, abs=1e-12)
        Gg = g.cpu().numpy()
        assert rel(Gg, O.chol_rev(Lo, Lbar)) <= TOL
        a = np.linalg.solve(p["S"], p["y"])
        assert rel(Gg, 0.5 * (np.linalg.inv(p["S"]) - np.outer(a, a))) <= 1e-9


def test_gp_batched_prebuilt_tables(cg, dev):
    """Prebuilt Batch / Vecs pointer tables give bitwise the same losses and gradients as plain
    tensor lists, on repeated calls."""
    import torch
    P = problems(SIZES, 401)
    S = [to_dev(p["S"], dev) for p in P]
    ys = [to_dev(p["y"], dev) for p in P]
    A1, G1 = [s.clone() for s in S], [torch.empty_like(s) for s in S]
    f1, i1 = cg.chol_gp_nll_batched(A1, ys, G1)
    A2, G2 = [s.clone() for s in S], [torch.empty_like(s) for s in S]
    Ab, Gb, yv = cg.Batch(A2), cg.Batch(G2), cg.Vecs(ys)
    for _ in range(2):
        for a, s in zip(A2, S):
            a.copy_(s)
        f2, i2 = cg.chol_gp_nll_batched(Ab, yv, Gb)
        assert torch.equal(i1, i2) and torch.equal(f1, f2)
        assert all(torch.equal(g1, g2) for g1, g2 in zip(G1, G2))
    with pytest.raises(ValueError):
        cg.chol_gp_nll_batched(Ab, cg.Vecs(ys[:-1]), Gb)


def test_batched_info_and_isolation(cg, dev):
    """A non-SPD problem gets its LAPACK-style info without disturbing its neighbours."""
    sizes = [150, 40, 300]
    P = problems(sizes, 500)
    bad = P[1]["S"].copy()
    bad[9, 9] = -1.0
    mats = [to_dev(P[0]["S"], dev), to_dev(bad, dev), to_dev(P[2]["S"], dev)]
    info = cg.chol_factor_batched(mats).cpu().tolist()
    assert info == [0, O.chol(bad)[1], 0] and info[1] == 10
    for k in (0, 2):
        assert rel(mats[k].cpu().numpy(), O.chol(P[k]["S"])[0]) <= TOL


def test_alone_equals_in_batch_bitwise(cg, dev):
    P = problems(SIZES, 600)
    k = SIZES.index(384)
    alone = [to_dev(P[k]["Lb"], dev)]
    cg.chol_rev_batched([to_dev(P[k]["L"], dev)], alone)
    Ls = [to_dev(p["L"], dev) for p in P]
    As = [to_dev(p["Lb"], dev) for p in P]
    cg.chol_rev_batched(Ls, As)
    assert np.array_equal(alone[0].cpu().numpy(), As[k].cpu().numpy())


def test_batched_matches_single_path(cg, dev):
    P = problems([384], 700)[0]
    one = cg.chol_rev(to_dev(P["L"], dev), to_dev(P["Lb"], dev), nb=128).cpu().numpy()
    As = [to_dev(P["Lb"], dev)]
    cg.chol_rev_batched([to_dev(P["L"], dev)], As)
    assert rel(As[0].cpu().numpy(), one) <= 1e-13


def test_gp_batch_of_2048(cg, dev):
    """The batched workload: 2048 matrices, n log-uniform in [16, 512], Sigma = A A^T/n + 0.1 I,
    y ~ N(0,1); 16 sampled problems checked against the oracle and the closed form."""
    import torch
    case = W.batch_case()
    As = [to_dev(S, dev) for S in case["Sigma"]]
    Gs = [torch.empty_like(a) for a in As]
    ys = [to_dev(y, dev) for y in case["y"]]
    f, info = cg.chol_gp_nll_batched(As, ys, Gs)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    f = f.cpu().numpy()
    rng = np.random.default_rng(9)
    for i in rng.choice(len(As), size=16, replace=False):
        S, y = case["Sigma"][i], case["y"][i]
        Lo, _ = O.chol(S)
        fo, Lbar = O.gp_loss_and_lbar(Lo, y)
        assert f[i] == pytest.approx(fo, rel=1e-11)
        assert rel(Gs[i].cpu().numpy(), O.chol_rev(Lo, Lbar)) <= TOL
        assert rel(As[i].cpu().numpy(), Lo) <= TOL


def test_split_plans_equal_one_plan_bitwise(cg, dev):
    """Batches of 1024 problems or more run as two plans (the even- and the odd-indexed problems)
    on two streams; each problem's loss, factor and gradient are bitwise those of the same problem
    in a small batch, which runs as one plan on one stream."""
    import torch
    case = W.batch_case(batch=1031, seed=4242)
    pick = [0, 1, 2, 514, 515, 1029, 1030, int(np.argmax(case["sizes"]))]
    As = [to_dev(S, dev) for S in case["Sigma"]]
    Gs = [torch.empty_like(a) for a in As]
    ys = [to_dev(y, dev) for y in case["y"]]
    f, info = cg.chol_gp_nll_batched(As, ys, Gs)
    As2 = [to_dev(case["Sigma"][i], dev) for i in pick]
    Gs2 = [torch.empty_like(a) for a in As2]
    f2, info2 = cg.chol_gp_nll_batched(As2, [ys[i] for i in pick], Gs2)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0 and int((info2 != 0).sum()) == 0
    for k, i in enumerate(pick):
        assert torch.equal(f[i], f2[k])
        assert torch.equal(As[i], As2[k]) and torch.equal(Gs[i], Gs2[k])


# ------------------------------------------------------------------------------------------------
# FP32 storage.  chol_fwd_batched widens each problem to FP64 and rounds once on output: against
# the oracle on the same float inputs the only difference is that rounding (relative Frobenius
# error at most 2^-24 plus the FP64 gate), F32_SAME = 1e-7.  The factor, reverse and GP calls
# compute in FP64 inside each block step and round every value they store to FP32 (the matrices
# are updated in place between steps): against the oracle on the same float inputs, stated
# relL <= 3e-7, rel Sigma-bar <= 7e-6, rel f <= 6e-7 (measured on the SIZES problems 3.4e-8,
# 6.8e-7, 5.6e-8: about a tenth).  End to end against the FP64 oracle on the FP64 inputs (input
# rounding amplified by conditioning, kappa <= 41 on the batched workload): stated relL <= 3e-7,
# rel Sigma-bar <= 3e-6, rel f <= 1e-6 (measured over 64 sampled problems 5.8e-8, 4.2e-7, 1.9e-7).
F32_SAME = 1e-7
F32_STEP_L, F32_STEP_SBAR, F32_STEP_F = 3e-7, 7e-6, 6e-7


def f32(x):
    return np.asarray(x, dtype=np.float32)


def widened(x):
    return f32(x).astype(np.float64)


def test_factor_batched_f32(cg, dev):
    P = problems(SIZES, 1100)
    mats = [to_dev(f32(p["S"] + p["junk"]), dev) for p in P]
    info = cg.chol_factor_batched(mats)
    assert info.cpu().tolist() == [0] * len(P)
    for p, m in zip(P, mats):
        Lg = m.cpu().numpy().astype(np.float64)
        assert rel(Lg, O.chol(widened(p["S"]))[0]) <= F32_STEP_L
        assert rel(Lg, O.chol(p["S"])[0]) <= 3e-7
        assert np.all(np.triu(Lg, 1) == 0)


@pytest.mark.parametrize("form", ["sym", "tril"])
def test_rev_batched_f32(cg, dev, form):
    P = problems(SIZES, 1200)
    Ls = [to_dev(f32(p["L"]), dev) for p in P]
    As = [to_dev(f32(p["Lb"] + p["junk"]), dev) for p in P]
    cg.chol_rev_batched(Ls, As, form=form)
    for p, a in zip(P, As):
        want = O.chol_rev(widened(p["L"]), widened(p["Lb"]), form)
        assert rel(a.cpu().numpy().astype(np.float64), want) <= F32_STEP_SBAR


def test_fwd_batched_f32(cg, dev):
    P = problems(SIZES, 1300)
    Ls = [to_dev(f32(p["L"]), dev) for p in P]
    As = [to_dev(f32(np.tril(p["Sd"]) + p["junk"]), dev) for p in P]
    cg.chol_fwd_batched(Ls, As)
    for p, a in zip(P, As):
        got = a.cpu().numpy().astype(np.float64)
        assert rel(got, O.chol_fwd(widened(p["L"]), widened(p["Sd"]))) <= F32_SAME
        assert np.all(np.triu(got, 1) == 0)


def test_gp_batched_f32(cg, dev):
    import torch
    P = problems(SIZES, 1400)
    As = [to_dev(f32(p["S"]), dev) for p in P]
    Gs = [torch.empty_like(a) for a in As]
    ys = [to_dev(f32(p["y"]), dev) for p in P]
    f, info = cg.chol_gp_nll_batched(As, ys, Gs)
    assert f.dtype == torch.float32
    assert info.cpu().tolist() == [0] * len(P)
    f = f.cpu().numpy().astype(np.float64)
    for i, (p, g) in enumerate(zip(P, Gs)):
        Lo, _ = O.chol(widened(p["S"]))
        fo, Lbar = O.gp_loss_and_lbar(Lo, widened(p["y"]))
        assert f[i] == pytest.approx(fo, rel=F32_STEP_F, abs=1e-30)
        assert rel(g.cpu().numpy().astype(np.float64), O.chol_rev(Lo, Lbar)) <= F32_STEP_SBAR
        assert rel(As[i].cpu().numpy().astype(np.float64), Lo) <= F32_STEP_L


def test_f32_alone_equals_in_batch_bitwise(cg, dev):
    P = problems(SIZES, 1500)
    k = SIZES.index(257)
    alone = [to_dev(f32(P[k]["S"]), dev)]
    cg.chol_factor_batched(alone)
    mats = [to_dev(f32(p["S"]), dev) for p in P]
    cg.chol_factor_batched(mats)
    assert np.array_equal(alone[0].cpu().numpy(), mats[k].cpu().numpy())


def test_gp_batch_of_2048_f32(cg, dev):
    """The batched workload stored in FP32: 16 sampled problems end to end against the FP64 oracle
    on the FP64 inputs, at the stated tolerances."""
    import torch
    case = W.batch_case()
    As = [to_dev(f32(S), dev) for S in case["Sigma"]]
    Gs = [torch.empty_like(a) for a in As]
    ys = [to_dev(f32(y), dev) for y in case["y"]]
    f, info = cg.chol_gp_nll_batched(As, ys, Gs)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    f = f.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(19)
    worst = [0.0, 0.0, 0.0]
    for i in rng.choice(len(As), size=16, replace=False):
        S, y = case["Sigma"][i], case["y"][i]
        Lo, _ = O.chol(S)
        fo, Lbar = O.gp_loss_and_lbar(Lo, y)
        e = (rel(As[i].cpu().numpy().astype(np.float64), Lo),
             rel(Gs[i].cpu().numpy().astype(np.float64), O.chol_rev(Lo, Lbar)),
             abs(f[i] - fo) / abs(fo))
        worst = [max(a, b) for a, b in zip(worst, e)]
    print(f"FP32 storage end to end: relL {worst[0]:.2e}, rel Sigma-bar {worst[1]:.2e}, rel f {worst[2]:.2e}")
    assert worst[0] <= 3e-7 and worst[1] <= 3e-6 and worst[2] <= 1e-6
