"""chol_rev_noalloc (the allocation-free chol_rev on the library's static device scratch) against
chol_rev with a caller's workspace and against the FP64 oracle, through the C ABI: two calls in a
row, the second on a smaller problem (the scratch keeps the first call's contents), at the 1e-10
FP64 gate on a shared L."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_chol_rev_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1602_07527_amd as cg
    lib = cg.load_library()
    dev = torch.device("cuda:0")
    for n, nb, form, seed in ((4096, 128, "sym", 9101), (1000, 64, "tril", 9102)):
        S, rng = W.dense_spd(n, seed)
        L = O.chol_host(S)
        Lb = W.lower_normal(n, rng)
        Lt = torch.from_numpy(L).to(dev)
        want = cg.chol_rev(Lt, torch.from_numpy(Lb).to(dev), form=form, nb=nb).cpu().numpy()
        A = torch.from_numpy(Lb).to(dev)
        stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        rc = lib.chol_rev_noalloc(0, n, Lt.data_ptr(), n, A.data_ptr(), n, 1 if form == "tril" else 0, nb, stream)
        assert rc == 0
        got = A.cpu().numpy()
        print(f"noalloc n={n} nb={nb} {form}: vs chol_rev {rel(got, want):.2e}, "
              f"vs oracle {rel(got, O.chol_rev(L, Lb, form)):.2e}")
        assert rel(got, want) <= TOL
        assert rel(got, O.chol_rev(L, Lb, form)) <= TOL
        if form == "sym":
            assert np.array_equal(got, got.T)
        else:
            assert np.all(np.triu(got, 1) == 0)
