"""GPU tests of the fused batched factor + reverse sweep and of the continuous-batching serving loop.

* chol_factor_rev_batched: L against the oracle's factor, Sigma-bar against the oracle's reverse
  sweep on the oracle's L (1e-10; these matrices have condition number below 50), FP64 and FP32
  storage (FP32: against the oracle on the float inputs, 1e-7).
* serving: a Poisson request stream (n log-uniform in [64, 1536], squared-exponential kernels in
  2-D); every result of the mix is bitwise equal to the same request served alone; sampled results
  match the oracle within the end-to-end tolerance max(1e-10, 100 kappa u) (each side factors for
  itself, so conditioning enters); the admitted footprint never exceeds the budget; the
  reduced-precision mode stays within its stated tolerances.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
U64 = np.finfo(np.float64).eps / 2


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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_factor_rev_batched(cg, dtype):
    import torch
    sizes = [1, 17, 64, 128, 129, 200, 257, 384, 512]
    S_list, Lb_list = [], []
    for i, n in enumerate(sizes):
        S, rng = W.dense_spd(n, 3000 + i)
        S_list.append(S)
        Lb_list.append(W.lower_normal(n, rng))
    cast = (lambda x: x) if dtype == "f64" else (lambda x: x.astype(np.float32))
    A = [to_dev(cast(S)) for S in S_list]
    G = [to_dev(cast(Lb)) for Lb in Lb_list]
    info = cg.chol_factor_rev_batched(A, G)
    assert info.cpu().tolist() == [0] * len(sizes)
    # FP32 storage rounds the values each block step stores (stated in include/cholgrad.h):
    # against the oracle on the same float inputs relL <= 3e-7, rel Sigma-bar <= 7e-6
    tol_l, tol_s = (1e-10, 1e-10) if dtype == "f64" else (3e-7, 7e-6)
    for S, Lb, a, g in zip(S_list, Lb_list, A, G):
        S, Lb = cast(S).astype(np.float64), cast(Lb).astype(np.float64)
        L = O.chol(S)[0]
        assert rel(a.cpu().numpy().astype(np.float64), L) <= tol_l
        assert rel(g.cpu().numpy().astype(np.float64), O.chol_rev(L, Lb)) <= tol_s
    del torch


def _trace(seconds, hi=1536, seed=77):
    return W.serve_trace(rate=200.0, seconds=seconds, lo=64, hi=hi, seed=seed)


def _make_inputs(tr):
    import torch
    dev = torch.device("cuda:0")
    return lambda i: W.se_request_device(tr["n"][i], tr["lengthscale"][i], tr["seed"][i], dev)


def _request(serve, rid, Sigma, Lbar):
    """A request whose launch waits for its inputs, written on the current stream (the server
    launches on streams of its own)."""
    import torch
    ev = torch.cuda.Event()
    ev.record()
    return serve.Request(rid, Sigma, Lbar, ready=ev)


@pytest.fixture(scope="module")
def served(cg):
    """One 3-second stream through an FP64 server; results of every request copied to the host."""
    from paper_1602_07527_amd import serve
    tr = _trace(3.0)
    srv = serve.Server("cuda:0", hbm_budget=8 << 30)
    res = {}

    def keep(r):
        res[r.rid] = (int(r.info.item()), r.L.cpu().numpy(), r.Sbar.cpu().numpy(), r.route)

    done, wall = serve.replay(srv, tr["t"], _make_inputs(tr), on_done=keep)
    summary = serve.latency_summary(done, wall)
    print("serving summary:", summary, "launches:", srv.launches)
    return {"trace": tr, "res": res, "server": srv, "summary": summary}


def test_serve_completes_everything(served):
    tr, res, srv = served["trace"], served["res"], served["server"]
    assert len(res) == len(tr["t"])
    assert all(v[0] == 0 for v in res.values())
    assert srv.in_use == 0 and srv.idle()
    assert srv.peak_in_use <= srv.hbm_budget
    assert srv.launches["small"] >= 1 and srv.launches["large"] >= 1
    # continuous batching: small requests shared launches
    assert srv.launches["small"] < sum(1 for v in res.values() if v[3] == "small")


def test_serve_alone_equals_mix_bitwise(cg, served):
    from paper_1602_07527_amd import serve
    tr, res = served["trace"], served["res"]
    rng = np.random.default_rng(5)
    small = [i for i in res if res[i][3] == "small"]
    large = [i for i in res if res[i][3] == "large"]
    pick = list(rng.choice(small, size=min(6, len(small)), replace=False)) + \
        list(rng.choice(large, size=min(6, len(large)), replace=False))
    make = _make_inputs(tr)
    for i in pick:
        srv = serve.Server("cuda:0", hbm_budget=8 << 30)
        Sigma, Lbar = make(i)
        r = srv.submit(_request(serve, int(i), Sigma, Lbar))
        srv.drain()
        assert int(r.info.item()) == 0
        assert np.array_equal(r.L.cpu().numpy(), res[i][1]), f"L of request {i} (n={tr['n'][i]})"
        assert np.array_equal(r.Sbar.cpu().numpy(), res[i][2]), f"Sigma-bar of request {i}"


def test_serve_results_match_oracle(cg, served):
    tr, res = served["trace"], served["res"]
    make = _make_inputs(tr)
    ids = sorted(res, key=lambda i: tr["n"][i])
    pick = [ids[0], ids[len(ids) // 3], ids[len(ids) // 2]] + [i for i in ids if 520 <= tr["n"][i] <= 900][:2]
    for i in pick:
        Sigma, Lbar = make(i)
        S, Lb = Sigma.cpu().numpy(), np.tril(Lbar.cpu().numpy())
        L = O.chol(S)[0]
        kappa = np.linalg.cond(S)
        tol = max(1e-10, 100 * kappa * U64)
        assert rel(res[i][1], L) <= tol, (i, tr["n"][i])
        assert rel(res[i][2], O.chol_rev(L, Lb)) <= tol, (i, tr["n"][i], kappa)


def test_serve_under_a_tight_budget(cg):
    """A budget that holds about one large request at a time: requests wait for memory, are
    admitted in arrival order, and every one completes."""
    from paper_1602_07527_amd import serve
    tr = _trace(0.5, seed=78)
    srv = serve.Server("cuda:0", hbm_budget=1)
    alone = lambda n: srv.footprint(n) + (srv.group_workspace(1, n) if n <= serve.SMALL_MAX else 0)
    budget = max(alone(int(n)) for n in tr["n"]) + alone(64)
    srv = serve.Server("cuda:0", hbm_budget=budget)
    order = []
    done, wall = serve.replay(srv, tr["t"], _make_inputs(tr), on_done=lambda r: order.append(r.t_admit))
    assert len(done) == len(tr["t"])
    assert all(int(r.info.item()) == 0 for r in done)
    assert srv.peak_in_use <= budget
    admits = [r.t_admit for r in sorted(done, key=lambda r: r.rid)]
    assert admits == sorted(admits)                     # nobody overtook an earlier request


# Stated per-request accuracy of mixed-precision serving ('f64_trail_f32': factor and reverse sweep
# of every request above the batched size limit with FP32-MFMA trailing contractions, each request
# on its own L) on the serving workload (n log-uniform in [64, 4096], 2-D squared-exponential
# kernels with lengthscale U[0.1, 0.5] + 1e-3 I, condition numbers up to ~2e6).  Measured on
# MI355X over 420 requests of the 60 s stream (400 drawn at random plus the 20 with the largest
# n * lengthscale): rel Sigma-bar p50 2.7e-3, p95 8.9e-3, max 9.2e-3; relL max 2.7e-4.
SERVE_MIXED_REL_SBAR = 2e-2
SERVE_MIXED_REL_L = 6e-4


def test_serve_mixed_precision_within_stated_tolerance(cg):
    """Mixed-precision served results against the oracle (each side factors for itself), for
    requests of moderate size, at the stated per-request bounds."""
    from paper_1602_07527_amd import serve
    tr = _trace(1.0, seed=79)
    big = [i for i in range(len(tr["t"])) if 600 <= tr["n"][i] <= 1100][:3]
    assert big
    make = _make_inputs(tr)
    srv = serve.Server("cuda:0", hbm_budget=8 << 30, precision="f64_trail_f32")
    reqs = []
    for i in big:
        Sigma, Lbar = make(i)
        reqs.append(srv.submit(_request(serve, int(i), Sigma, Lbar)))
    srv.drain()
    for i, r in zip(big, reqs):
        Sigma, Lbar = make(i)
        S, Lb = Sigma.cpu().numpy(), np.tril(Lbar.cpu().numpy())
        L = O.chol_host(S)
        eL = rel(r.L.cpu().numpy(), L)
        eS = rel(r.Sbar.cpu().numpy(), O.chol_rev(L, Lb))
        print(f"mixed serving n={tr['n'][i]}: relL {eL:.2e} rel Sigma-bar {eS:.2e}")
        assert 1e-9 < eS <= SERVE_MIXED_REL_SBAR and eL <= SERVE_MIXED_REL_L


def test_serve_mixed_precision_worst_requests(cg):
    """The worst-conditioned requests of the 60 s serving stream (largest n * lengthscale, n near
    4096 and lengthscale near 0.5): the mixed-precision served Sigma-bar against the oracle for the
    two worst, and against the FP64 served result (itself within max(1e-10, 100 kappa u) of the
    oracle) for the next six, all at the stated per-request bounds."""
    import torch
    from paper_1602_07527_amd import serve
    tr = W.serve_trace(rate=200.0, seconds=60.0)
    worst = [int(i) for i in np.argsort(tr["n"] * tr["lengthscale"])[::-1][:8]]
    make = _make_inputs(tr)
    for rank, i in enumerate(worst):
        out = {}
        for mode in ("f64", "f64_trail_f32"):
            srv = serve.Server("cuda:0", hbm_budget=8 << 30, precision=mode)
            Sigma, Lbar = make(i)
            r = srv.submit(_request(serve, i, Sigma, Lbar))
            srv.drain()
            assert int(r.info.item()) == 0
            out[mode] = r
        mixed, f64 = out["f64_trail_f32"], out["f64"]
        if rank < 2:
            Sigma, Lbar = make(i)
            S, Lb = Sigma.cpu().numpy(), np.tril(Lbar.cpu().numpy())
            L = O.chol_host(S)
            eL = rel(mixed.L.cpu().numpy(), L)
            eS = rel(mixed.Sbar.cpu().numpy(), O.chol_rev(L, Lb))
            ref = "oracle"
        else:
            nrm = lambda x: float(torch.linalg.norm(x))
            eL = nrm(mixed.L - f64.L) / nrm(f64.L)
            eS = nrm(mixed.Sbar - f64.Sbar) / nrm(f64.Sbar)
            ref = "FP64 served"
        print(f"mixed serving n={tr['n'][i]} lengthscale={tr['lengthscale'][i]:.3f}: relL {eL:.2e} "
              f"rel Sigma-bar {eS:.2e} (vs {ref})")
        assert 1e-9 < eS <= SERVE_MIXED_REL_SBAR and eL <= SERVE_MIXED_REL_L
