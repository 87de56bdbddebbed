"""Host-side pieces of the serving loop: the admission policy and the request-stream recipe."""
import numpy as np

import workloads as W
from paper_1602_07527_amd.serve import admit


class R:
    def __init__(self, n, footprint):
        self.n, self.footprint = n, footprint


def test_admission_is_in_order_and_within_budget():
    pend = [R(600, 40), R(100, 10), R(2000, 100), R(50, 5)]
    small, large, used = admit(pend, in_use=0, budget=120, small_max=512, max_group=8)
    assert [r.n for r in large] == [600] and [r.n for r in small] == [100]
    assert used == 50                     # the 2000 does not fit, and nothing overtakes it
    small, large, used = admit(pend, in_use=0, budget=1000, small_max=512, max_group=8)
    assert len(small) == 2 and len(large) == 2 and used == 155


def test_admission_respects_the_group_cap_and_current_use():
    pend = [R(64, 1) for _ in range(10)]
    small, large, used = admit(pend, in_use=0, budget=100, small_max=512, max_group=4)
    assert len(small) == 4 and not large and used == 4
    small, large, used = admit(pend, in_use=97, budget=100, small_max=512, max_group=64)
    assert len(small) == 3 and used == 100
    assert admit([], 0, 1, 512, 4) == ([], [], 0)


def test_serve_trace_recipe():
    t = W.serve_trace(rate=200.0, seconds=60.0)
    m = len(t["t"])
    assert abs(m - 12000) < 4 * np.sqrt(12000)          # Poisson count
    assert np.all(np.diff(t["t"]) > 0) and t["t"][-1] < 60.0
    assert t["n"].min() >= 64 and t["n"].max() <= 4096
    assert abs(np.median(t["n"]) - 512) < 40              # log-uniform median sqrt(64 * 4096)
    assert t["lengthscale"].min() >= 0.1 and t["lengthscale"].max() <= 0.5
    t2 = W.serve_trace(rate=200.0, seconds=60.0)
    assert np.array_equal(t["n"], t2["n"]) and np.array_equal(t["seed"], t2["seed"])


def test_admission_charges_the_group_workspace():
    """A small group is charged exactly the workspace of its one batched launch (group_ws(count,
    max n)) on top of the requests' own buffers; a request whose share does not fit stops the walk."""
    ws = lambda count, n_max: 1000 * count + n_max          # any monotone workspace size
    pend = [R(100, 10), R(300, 10), R(200, 10), R(800, 50)]
    small, large, used = admit(pend, 0, 10 ** 6, 512, 8, ws)
    assert [r.n for r in small] == [100, 300, 200] and [r.n for r in large] == [800]
    assert used == 30 + ws(3, 300) + 50
    small, large, used = admit(pend, 0, 10 + ws(1, 100) + 10 + ws(2, 300) - ws(1, 100), 512, 8, ws)
    assert [r.n for r in small] == [100, 300] and not large
    assert used == 20 + ws(2, 300)


def test_admission_footprint_equals_the_library_workspace():
    """With the library's batched workspace size, what admission charges for a group of small
    requests is what their launch allocates: own buffers + chol_batched_workspace_bytes."""
    from paper_1602_07527_amd import _binding as B
    own = lambda n: 2 * 8 * n * n
    pend = [R(n, own(n)) for n in (64, 500, 17, 256, 300)]
    small, large, used = admit(pend, 0, 1 << 40, 512, 256, B.batched_workspace_bytes)
    assert len(small) == 5 and not large
    assert used == sum(own(r.n) for r in pend) + B.batched_workspace_bytes(5, 500)
    # a launch of a few requests no longer reserves the workspace of a full grid
    assert B.batched_workspace_bytes(1, 512) * 100 < B.batched_workspace_bytes(256, 512)
