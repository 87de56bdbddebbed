"""GPU tests of the torch.autograd wrappers (x -> Sigma -> L -> f of Sec. 2).

* cholesky / cholesky_batched: Sigma.grad equals the oracle's reverse sweep (symmetric form) for
  the same L-bar; recompute=True gives the same bits; torch.autograd.gradcheck through a symmetric
  parametrisation Sigma = X X^T / n + I.
* gp_neg_log_lik on the batched GP workload (2048 matrices, n log-uniform in [16, 512]): directional
  central differences on 16 sampled matrices, 8 random symmetric directions and 32 random single
  entries each, h = 1e-6, relative tolerance 1e-6 plus the rounding floor of a difference
  quotient, n * u * F / h with F = sum |log L_ii| + |L^-1 y|^2 / 2 (the size of the terms whose
  rounding the quotient amplifies); Sigma.grad against the closed form (Sigma^-1 - a a^T)/2,
  a = Sigma^-1 y.
* the whole chain: d f / d lengthscale of a squared-exponential kernel by autograd against a
  central difference in the lengthscale.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2


@pytest.fixture(scope="module")
def ag():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as pkg
    pkg.load_library()
    from paper_1602_07527_amd import autograd
    return autograd


@pytest.fixture(scope="module")
def dev(ag):
    import torch
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dev, grad=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return t.requires_grad_(grad)


@pytest.mark.parametrize("n,nb", [(300, 128), (257, 64), (40, 32)])
@pytest.mark.parametrize("recompute", [False, True])
def test_cholesky_grad_matches_oracle(ag, dev, n, nb, recompute):
    S, rng = W.dense_spd(n, 800 + n)
    Lbar = W.lower_normal(n, rng)
    Sig = to_dev(S, dev, grad=True)
    L, info = ag.cholesky_ex(Sig, recompute=recompute, nb=nb)
    assert int(info.item()) == 0
    L.backward(to_dev(Lbar, dev))
    Lo, _ = O.chol(S)
    assert rel(L.detach().cpu().numpy(), Lo) <= 1e-10
    assert rel(Sig.grad.cpu().numpy(), O.chol_rev(Lo, Lbar, "sym")) <= 1e-10


def test_cholesky_recompute_same_bits(ag, dev):
    S, rng = W.dense_spd(384, 901)
    Lbar = to_dev(W.lower_normal(384, rng), dev)
    grads = []
    for rc in (False, True):
        Sig = to_dev(S, dev, grad=True)
        ag.cholesky(Sig, recompute=rc).backward(Lbar)
        grads.append(Sig.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])


def test_cholesky_gradcheck(ag, dev):
    import torch
    n = 12
    X = torch.from_numpy(np.random.default_rng(902).standard_normal((n, n))).to(dev).requires_grad_()
    Wt = torch.from_numpy(np.random.default_rng(903).standard_normal((n, n))).to(dev)

    def f(X):
        Sig = X @ X.T / n + torch.eye(n, dtype=X.dtype, device=X.device)
        return (ag.cholesky(Sig, nb=32) * Wt).sum()

    assert torch.autograd.gradcheck(f, (X,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_cholesky_batched_grad(ag, dev):
    sizes = [5, 64, 130, 300, 512]
    Sigs, Lbars, Ss = [], [], []
    for i, n in enumerate(sizes):
        S, rng = W.dense_spd(n, 910 + i)
        Ss.append(S)
        Sigs.append(to_dev(S, dev, grad=True))
        Lbars.append(W.lower_normal(n, rng))
    Ls, info = ag.cholesky_batched(Sigs)
    assert info.cpu().tolist() == [0] * len(sizes)
    loss = sum((L * to_dev(Lb, dev)).sum() for L, Lb in zip(Ls, Lbars))
    loss.backward()
    for S, Sig, Lb in zip(Ss, Sigs, Lbars):
        Lo, _ = O.chol(S)
        assert rel(Sig.grad.cpu().numpy(), O.chol_rev(Lo, Lb, "sym")) <= 1e-10


def test_gp_grad_closed_form_and_weights(ag, dev):
    import torch
    sizes = [16, 100, 257, 512]
    Ss, ys = [], []
    for i, n in enumerate(sizes):
        S, rng = W.dense_spd(n, 920 + i, shift=0.1)
        Ss.append(S)
        ys.append(rng.standard_normal(n))
    for recompute in (False, True):
        Sigs = [to_dev(S, dev, grad=True) for S in Ss]
        f, info = ag.gp_neg_log_lik(Sigs, [to_dev(y, dev) for y in ys], recompute=recompute)
        assert info.cpu().tolist() == [0] * len(sizes)
        w = torch.arange(1, len(sizes) + 1, dtype=torch.float64, device=dev)
        (f * w).sum().backward()
        for b, (S, y, Sig) in enumerate(zip(Ss, ys, Sigs)):
            a = np.linalg.solve(S, y)
            want = (b + 1) * 0.5 * (np.linalg.inv(S) - np.outer(a, a))
            assert rel(Sig.grad.cpu().numpy(), want) <= 1e-9
            fo, _ = O.gp_loss_and_lbar(O.chol(S)[0], y)
            assert float(f[b].detach()) == pytest.approx(fo, rel=1e-11)


def test_gp_rejects_grad_in_y(ag, dev):
    S, rng = W.dense_spd(20, 930, shift=0.1)
    f, _ = ag.gp_neg_log_lik([to_dev(S, dev, grad=True)], [to_dev(rng.standard_normal(20), dev, grad=True)])
    with pytest.raises(NotImplementedError):
        f.sum().backward()


def test_gp_central_differences_batch_workload(ag, dev):
    """Sampled problems of the 2048-matrix workload; perturbations are built on the host in FP64 and
    the exact representable difference (Sigma+) - (Sigma-) is what the analytic side is paired with."""
    import torch
    case = W.batch_case()
    pick = np.random.default_rng(931).choice(len(case["Sigma"]), size=16, replace=False)
    rng = np.random.default_rng(932)
    h = 1e-6
    plus, minus, owner = [], [], []
    for i in pick:
        S = case["Sigma"][i]
        n = S.shape[0]
        dirs = [W.sym_normal(n, rng) for _ in range(8)]
        for _ in range(32):
            k, l = rng.integers(0, n, size=2)
            E = np.zeros((n, n))
            E[k, l] = E[l, k] = 1.0
            dirs.append(E)
        for E in dirs:
            plus.append(S + h * E)
            minus.append(S - h * E)
            owner.append(i)
    Sigs = [to_dev(case["Sigma"][i], dev, grad=True) for i in pick]
    f0, info = ag.gp_neg_log_lik(Sigs, [to_dev(case["y"][i], dev) for i in pick])
    assert int((info != 0).sum()) == 0
    f0.sum().backward()
    G = {i: s.grad.cpu().numpy() for i, s in zip(pick, Sigs)}
    fp, ip = ag.gp_neg_log_lik([to_dev(P, dev) for P in plus], [to_dev(case["y"][i], dev) for i in owner])
    fm, im = ag.gp_neg_log_lik([to_dev(M, dev) for M in minus], [to_dev(case["y"][i], dev) for i in owner])
    assert int((ip != 0).sum()) == 0 and int((im != 0).sum()) == 0
    fp, fm = fp.cpu().numpy(), fm.cpu().numpy()
    F = {}
    for i in pick:
        Lo, _ = O.chol(case["Sigma"][i])
        F[i] = float(np.sum(np.abs(np.log(np.diag(Lo))))
                     + 0.5 * np.sum(sla.solve_triangular(Lo, case["y"][i], lower=True) ** 2))
    worst = 0.0
    for c, i in enumerate(owner):
        fd = (fp[c] - fm[c]) / (2 * h)
        an = float(np.sum(G[i] * (plus[c] - minus[c]))) / (2 * h)
        floor = case["Sigma"][i].shape[0] * U64 * F[i] / h
        err = abs(fd - an)
        assert err <= 1e-6 * abs(an) + floor, (i, c, fd, an)
        worst = max(worst, err / (abs(an) + floor))
    print(f"worst scaled FD error {worst:.3g} over {len(owner)} directions")


def test_chain_lengthscale(ag, dev):
    """x -> Sigma(ell) -> L -> f: autograd d f / d ell against a central difference in ell."""
    import torch
    rng = np.random.default_rng(940)
    n = 200
    X = torch.from_numpy(rng.uniform(0, 1, (n, 3))).to(dev)
    y = torch.from_numpy(rng.standard_normal(n)).to(dev)
    D = torch.cdist(X, X) ** 2

    def loss(ell):
        Sig = torch.exp(-D / (2 * ell * ell)) + 1e-2 * torch.eye(n, dtype=D.dtype, device=dev)
        return ag.gp_neg_log_lik([Sig], [y])[0][0]

    ell = torch.tensor(0.3, dtype=torch.float64, device=dev, requires_grad=True)
    loss(ell).backward()
    h = 1e-6
    with torch.no_grad():
        fd = (loss(ell + h) - loss(ell - h)) / (2 * h)
    assert float(ell.grad) == pytest.approx(float(fd), rel=1e-6)
