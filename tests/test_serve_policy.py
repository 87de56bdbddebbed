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
