"""Full-size (N = 16384) GPU checks on the benchmark's workload, in the benchmark's launch
configuration (nb = 128), by properties that hold at any size and need only O(N^2) host/device
work beyond the calls themselves:

  factor : leading-block property (the leading n0 x n0 block of chol(Sigma) is chol of Sigma's
           leading block -> compared with the oracle), sampled entries of L L^T against Sigma,
           positive diagonal, zero strict upper triangle.
  rev    : closed forms (f = Tr(C Sigma) with low-rank-plus-diagonal symmetric C gives Sigma-bar = C;
           L-bar = L gives I/2; L-bar = diag(1/L_ii) gives Sigma^-1/2, probed as 2 Sbar (Sigma x) = x);
           an L-bar supported on the leading block gives zero outside it and the oracle's answer
           inside.
  fwd    : Sigma-dot = Sigma gives L/2; Sigma-dot = D L^T + L D (D diagonal) gives D; leading block.
  both   : adjoint identity Tr(Lbar^T Ldot) = sum_ij Sbar_ij Sdot_ij with the GPU's own results.
Tolerances: 1e-10 relative for the closed forms and the leading blocks (measured ~1e-14 on the
CPU oracle at N = 2048 with the same kernel family), 1e-9 for the inverse probe (it also carries
the conditioning of Sigma, kappa ~ 1e5, through the product Sigma x).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
N = 16384
NB = 128
N0 = 1536          # leading block compared element-wise with the oracle


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as cg
    cg.load_library()
    dev = torch.device("cuda:0")
    inp = W.large_case_device(dev, N=N)
    ws_bytes = max(cg.workspace_bytes(op, N, NB) for op in ("factor", "rev", "fwd"))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L, info = cg.chol_factor(inp["Sigma"].clone(), nb=NB, workspace=ws)
    torch.cuda.synchronize()
    return {"cg": cg, "dev": dev, "ws": ws, "L": L, "info": int(info.item()), **inp}


def trel(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_factor_properties(big):
    import torch
    L, S = big["L"], big["Sigma"]
    assert big["info"] == 0
    assert bool(torch.isfinite(L).all())
    assert bool((torch.diagonal(L) > 0).all())
    assert float(torch.triu(L, 1).abs().max()) == 0.0
    Lo, info = O.chol(S[:N0, :N0].cpu().numpy())
    assert info == 0
    assert np.linalg.norm(L[:N0, :N0].cpu().numpy() - Lo) / np.linalg.norm(Lo) <= 1e-10
    g = torch.Generator(device=big["dev"])
    g.manual_seed(11)
    i = torch.randint(0, N, (4096,), device=big["dev"], generator=g)
    j = torch.randint(0, N, (4096,), device=big["dev"], generator=g)
    lhs = (L[i] * L[j]).sum(dim=1)
    scale = torch.sqrt(torch.diagonal(S)[i] * torch.diagonal(S)[j])
    assert float(((lhs - S[i, j]).abs() / scale).max()) <= 20 * N * 1.1e-16


def test_rev_closed_forms(big):
    import torch
    cg, L, dev, ws = big["cg"], big["L"], big["dev"], big["ws"]
    g = torch.Generator(device=dev)
    g.manual_seed(12)
    u, v, d = (torch.randn(N, dtype=torch.float64, device=dev, generator=g) for _ in range(3))
    # f = Tr(C Sigma), C = u v^T + v u^T + diag(d):  L-bar = tril(2 C L), Sigma-bar = C
    Lb = 2.0 * (torch.outer(u, v @ L) + torch.outer(v, u @ L) + d[:, None] * L)
    Sb = cg.chol_rev(L, Lb.tril_(), nb=NB, workspace=ws)
    C = torch.outer(u, v) + torch.outer(v, u) + torch.diag(d)
    assert trel(Sb, C) <= 1e-10
    del Sb, Lb, C
    # f = (1/2) Tr(Sigma): L-bar = L  ->  I/2
    Sb = cg.chol_rev(L, L.clone(), nb=NB, workspace=ws)
    eye = torch.eye(N, dtype=torch.float64, device=dev)
    assert trel(Sb, 0.5 * eye) <= 1e-10
    del Sb, eye
    # f = (1/2) log det Sigma: L-bar = diag(1/L_ii) -> Sigma^-1 / 2, probed with random x
    Sb = cg.chol_rev(L, torch.diag(1.0 / torch.diagonal(L)), nb=NB, workspace=ws)
    x = torch.randn(N, dtype=torch.float64, device=dev, generator=g)
    y = 2.0 * (Sb @ (big["Sigma"] @ x))
    assert trel(y, x) <= 1e-9


def test_rev_leading_block(big):
    import torch
    cg, L = big["cg"], big["L"]
    Lb = torch.zeros_like(L)
    Lb[:N0, :N0] = big["Lbar"][:N0, :N0]
    Sb = cg.chol_rev(L, Lb, nb=NB, workspace=big["ws"])
    assert float(Sb[N0:].abs().max()) == 0.0 and float(Sb[:, N0:].abs().max()) == 0.0
    want = O.chol_rev(L[:N0, :N0].cpu().numpy(), big["Lbar"][:N0, :N0].cpu().numpy())
    got = Sb[:N0, :N0].cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-10


def test_fwd_closed_forms_and_leading_block(big):
    import torch
    cg, L, dev, ws = big["cg"], big["L"], big["dev"], big["ws"]
    Ld = cg.chol_fwd(L, big["Sigma"].tril(), nb=NB, workspace=ws)
    assert trel(Ld, 0.5 * L) <= 1e-10
    g = torch.Generator(device=dev)
    g.manual_seed(13)
    d = torch.randn(N, dtype=torch.float64, device=dev, generator=g)
    Sd = (d[:, None] * L.T + L * d[None, :]).tril().contiguous()     # lower of D L^T + L D
    Ld = cg.chol_fwd(L, Sd, nb=NB, workspace=ws)
    assert trel(Ld, torch.diag(d)) <= 1e-10
    del Sd
    Ld = cg.chol_fwd(L, big["Sdot"].clone(), nb=NB, workspace=ws)
    want = O.chol_fwd(L[:N0, :N0].cpu().numpy(), big["Sdot"][:N0, :N0].cpu().numpy())
    got = Ld[:N0, :N0].cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-10
    big["Ldot"] = Ld


def test_adjoint_identity_full_size(big):
    import torch
    cg, L = big["cg"], big["L"]
    Ld = big.get("Ldot")
    if Ld is None:
        Ld = cg.chol_fwd(L, big["Sdot"].clone(), nb=NB, workspace=big["ws"])
    Sb = cg.chol_rev(L, big["Lbar"].clone(), nb=NB, workspace=big["ws"])
    Sd = big["Sdot"]
    Sd_full = Sd + Sd.tril(-1).T
    lhs = float((big["Lbar"] * Ld).sum())
    rhs = float((Sb * Sd_full).sum())
    assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), float((big["Lbar"].abs() * Ld.abs()).sum()))
