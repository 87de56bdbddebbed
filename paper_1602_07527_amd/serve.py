"""Continuous-batching request loop for factor + reverse-sweep solves of uneven size.

Each request is one Sec. 2 forward/backward pair on the device: Sigma -> L (chol_factor, L kept on
the device for the backward pass) and L-bar -> Sigma-bar (chol_rev on that L).  The caller hands
over two device buffers, Sigma and L-bar; the loop works in place on them (Sigma's buffer ends up
holding L, L-bar's holds Sigma-bar) and gives them back when the request completes.

Scheduling, one `step()` at a time on the host:
  * retire: launches whose completion event has fired release their workspace; their requests
    complete (latency = completion seen - arrival);
  * admit: pending requests are admitted strictly in arrival order while the HBM footprint of
    everything admitted and not yet completed stays within `hbm_budget` bytes (a request's
    footprint: its two n x n FP64 buffers plus its workspace; a group of small requests is
    charged the workspace of its one batched launch);
  * launch: the admitted requests with n <= small_max (512) form ONE batched launch per step
    (chol_factor_rev_batched: one call for the whole group) on the small-request
    stream; larger ones are launched one by one (chol_factor + chol_rev), each on whichever of
    the large-request streams has the fewest launches in flight.  Requests that arrive while
    earlier launches are still running are admitted and launched as soon as memory allows, so
    their work overlaps on the device with what is already there.
Routing depends only on n and the precision mode, never on load, and every kernel is
deterministic, so a request's result is bitwise the same alone and in any mix.

Streams (all default priority): the large-request streams (two by default) and the library's side
stream for each, the small-request stream, and the caller's stream, on which the inputs are
written (a request may carry an event that the launch waits for).  Each library call enqueues its
whole sequence under the library's lock and waits only on events it recorded itself, so streams
that share a hardware queue cannot deadlock each other; sharing only costs overlap.  Precision
'f64' runs everything in FP64; 'f64_trail_f32' runs the large requests with FP32-MFMA trailing
contractions (the batched small requests stay FP64).  Stated per-request accuracy of the mixed
mode on the serving workload (2-D squared-exponential kernels, n <= 4096, condition numbers up to
~2e6; each request on its own L): relative Frobenius error <= 2e-2 in Sigma-bar and <= 6e-4 in L
against the FP64 result (measured on MI355X: Sigma-bar p95 8.9e-3, max 9.2e-3).
"""
import time
from collections import deque

import numpy as np
import torch

from . import _binding as B

SMALL_MAX = B.BATCH_NMAX


class Request:
    """One factor + reverse-sweep solve.  Sigma and Lbar are n x n float64 device tensors (only
    their lower triangles are read); after completion Sigma holds L and Lbar holds Sigma-bar."""

    __slots__ = ("rid", "n", "Sigma", "Lbar", "ready", "t_arrive", "t_admit", "t_done", "info",
                 "route", "footprint")

    def __init__(self, rid, Sigma, Lbar, ready=None, t_arrive=None):
        n = B._square("Sigma", Sigma)
        if B._square("Lbar", Lbar) != n or Lbar.device != Sigma.device:
            raise ValueError("Sigma and Lbar must have the same size and device")
        self.rid = rid
        self.n = n
        self.Sigma = Sigma
        self.Lbar = Lbar
        self.ready = ready                      # optional torch.cuda.Event: inputs are written
        self.t_arrive = time.perf_counter() if t_arrive is None else t_arrive
        self.t_admit = None
        self.t_done = None
        self.info = None                        # device int32 tensor of one element
        self.route = None
        self.footprint = 0

    @property
    def L(self):
        return self.Sigma

    @property
    def Sbar(self):
        return self.Lbar

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive


def admit(pending, in_use, budget, small_max, max_group, group_ws=None):
    """The admission policy, without side effects: walk the pending requests in arrival order and
    take each while the footprint fits (in_use + cost <= budget) and the small group has room
    (at most max_group requests with n <= small_max); stop at the first that does not fit, so no
    request is overtaken.  A large request costs its footprint.  A small request costs its own
    footprint plus what it adds to the workspace of the one batched launch the small group makes:
    group_ws(count, n_max) is that launch's workspace in bytes (None: no workspace), so the group
    is charged exactly group_ws(len(small), max n).  Returns (small, large, new_in_use)."""
    small, large = [], []
    ws_now, n_max = 0, 0
    for r in pending:
        cost = r.footprint
        if r.n <= small_max:
            if len(small) >= max_group:
                break
            nm = max(n_max, r.n)
            ws_next = group_ws(len(small) + 1, nm) if group_ws is not None else 0
            cost += ws_next - ws_now
        if in_use + cost > budget:
            break
        if r.n <= small_max:
            small.append(r)
            ws_now, n_max = ws_next, nm
        else:
            large.append(r)
        in_use += cost
    return small, large, in_use


class _Launch:
    __slots__ = ("event", "requests", "workspace", "info", "footprint", "keep", "stream")


def _device_array(values, device):
    """int64 host values -> device tensor through pinned memory, copied asynchronously on the
    current stream (no host synchronisation)."""
    host = torch.tensor(values, dtype=torch.int64).pin_memory()
    return host.to(device, non_blocking=True)


class Server:
    """See the module docstring.  Not thread-safe: drive it from one host thread."""

    def __init__(self, device, hbm_budget, precision="f64", small_max=SMALL_MAX, max_group=256, nb=0,
                 large_streams=2):
        if precision not in ("f64", "f64_trail_f32"):
            raise ValueError("precision must be 'f64' or 'f64_trail_f32'")
        if not 1 <= small_max <= SMALL_MAX:
            raise ValueError(f"small_max must be in [1, {SMALL_MAX}]")
        if not 1 <= large_streams <= 4:
            raise ValueError("large_streams must be in [1, 4]")
        B.load_library()
        self.device = torch.device(device)
        self.hbm_budget = int(hbm_budget)
        self.precision = precision
        self.small_max = small_max
        self.max_group = max_group
        self.nb = nb  # 0: the library's measured width per sweep and size
        self.streams_large = [torch.cuda.Stream(self.device) for _ in range(large_streams)]
        self.stream_small = torch.cuda.Stream(self.device)
        self.pending = deque()
        self.running = deque()
        self.in_use = 0            # bytes admitted and not yet completed
        self.peak_in_use = 0
        self.completed = 0
        self.launches = {"small": 0, "large": 0}

    @staticmethod
    def group_workspace(count, n_max):
        """Workspace bytes of one batched launch of `count` small requests of size <= n_max."""
        return B.batched_workspace_bytes(count, n_max)

    def footprint(self, n):
        """Device bytes a request of size n holds by itself while admitted: its two FP64 buffers,
        plus, for a large request, its single-matrix workspace.  A small request's share of its
        group's batched workspace is charged at admission (see admit)."""
        own = 2 * 8 * n * n
        if n > self.small_max:
            return own + max(B.workspace_bytes(op, n, self.nb, self.precision) for op in ("factor", "rev"))
        return own

    def submit(self, req):
        if req.n == 0:
            raise ValueError("empty request")
        if req.Sigma.device != self.device:
            raise ValueError("request on another device")
        req.route = "small" if req.n <= self.small_max else "large"
        req.footprint = self.footprint(req.n)
        alone = req.footprint + (self.group_workspace(1, req.n) if req.route == "small" else 0)
        if alone > self.hbm_budget:
            raise ValueError(f"request {req.rid} needs {alone} bytes, above the budget")
        self.pending.append(req)
        return req

    def idle(self):
        return not self.pending and not self.running

    def step(self):
        """Retire finished launches, then admit and launch what fits.  Returns the requests that
        completed in this step."""
        done = self._retire()
        small, large, in_use = admit(self.pending, self.in_use, self.hbm_budget, self.small_max,
                                     self.max_group, self.group_workspace)
        taken = len(small) + len(large)
        if taken:
            now = time.perf_counter()
            for _ in range(taken):
                self.pending.popleft().t_admit = now
            self.in_use = in_use
            self.peak_in_use = max(self.peak_in_use, in_use)
            if small:
                self._launch_small(small)
            for r in large:
                self._launch_large(r)
        return done

    def drain(self, poll_s=20e-6):
        out = []
        while not self.idle():
            out += self.step()
            if self.running:
                time.sleep(poll_s)
        return out

    def _retire(self):
        done = []
        still = deque()
        now = None
        for ln in self.running:
            if ln.event.query():
                now = now or time.perf_counter()
                for r in ln.requests:
                    r.t_done = now
                    done.append(r)
                self.in_use -= ln.footprint
                ln.workspace = ln.keep = None
            else:
                still.append(ln)
        self.running = still
        self.completed += len(done)
        return done

    def _launch_small(self, reqs):
        s = self.stream_small
        ln = _Launch()
        ln.stream = -1
        with torch.cuda.stream(s):
            for r in reqs:
                if r.ready is not None:
                    s.wait_event(r.ready)
            sizes = [r.n for r in reqs]
            n_dev = _device_array(sizes, self.device)
            a_ptr = _device_array([r.Sigma.data_ptr() for r in reqs], self.device)
            a_ld = _device_array([r.Sigma.stride(0) for r in reqs], self.device)
            g_ptr = _device_array([r.Lbar.data_ptr() for r in reqs], self.device)
            g_ld = _device_array([r.Lbar.stride(0) for r in reqs], self.device)
            n_max = max(sizes)
            ln.workspace = torch.empty(B.batched_workspace_bytes(len(reqs), n_max), dtype=torch.uint8,
                                       device=self.device)
            ln.info = torch.empty(len(reqs), dtype=torch.int32, device=self.device)
            B._check("chol_factor_rev_batched", B.load_library().chol_factor_rev_batched(
                B.PREC_F64, len(reqs), n_dev.data_ptr(), a_ptr.data_ptr(), a_ld.data_ptr(), g_ptr.data_ptr(),
                g_ld.data_ptr(), n_max, B.SBAR_SYM, ln.info.data_ptr(), ln.workspace.data_ptr(),
                ln.workspace.numel(), B._stream(self.device)))
            ln.event = torch.cuda.Event()
            ln.event.record(s)
        ln.keep = (n_dev, a_ptr, a_ld, g_ptr, g_ld)
        for i, r in enumerate(reqs):
            r.info = ln.info[i:i + 1]
            r.Sigma.record_stream(s)
            r.Lbar.record_stream(s)
        ln.requests = reqs
        ln.footprint = sum(r.footprint for r in reqs) + ln.workspace.numel()   # as admit charged it
        self.launches["small"] += 1
        self.running.append(ln)

    def _launch_large(self, r):
        busy = [0] * len(self.streams_large)
        for other in self.running:
            if other.stream >= 0:
                busy[other.stream] += 1
        si = min(range(len(busy)), key=lambda i: busy[i])
        s = self.streams_large[si]
        ln = _Launch()
        ln.stream = si
        with torch.cuda.stream(s):
            if r.ready is not None:
                s.wait_event(r.ready)
            ln.workspace = torch.empty(max(B.workspace_bytes(op, r.n, self.nb, self.precision)
                                           for op in ("factor", "rev")), dtype=torch.uint8, device=self.device)
            _, ln.info = B.chol_factor(r.Sigma, nb=self.nb, workspace=ln.workspace, precision=self.precision)
            B.chol_rev(r.Sigma, r.Lbar, form="sym", nb=self.nb, workspace=ln.workspace, precision=self.precision)
            ln.event = torch.cuda.Event()
            ln.event.record(s)
        ln.keep = None
        r.info = ln.info
        r.Sigma.record_stream(s)
        r.Lbar.record_stream(s)
        ln.requests = [r]
        ln.footprint = r.footprint
        self.launches["large"] += 1
        self.running.append(ln)


def replay(server, arrivals, make_inputs, on_done=None, poll_s=20e-6, keep_buffers=False):
    """Drive `server` with an arrival schedule: arrivals[i] is request i's arrival time in seconds
    from the start; at that time make_inputs(i) -> (Sigma, Lbar) writes its inputs on the caller's
    current stream and the request is submitted with an event on that stream.  Latency runs from
    the scheduled arrival, so a loop that falls behind is charged for it.  Calls on_done(request)
    for every completion; afterwards the request's device buffers (its L and Sigma-bar) are
    released unless keep_buffers, so a long stream holds only the requests in flight.  Returns
    (completed requests, wall seconds)."""
    arrivals = np.asarray(arrivals, dtype=np.float64)
    done_all = []
    t0 = time.perf_counter()
    i = 0
    while i < len(arrivals) or not server.idle():
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i] <= now:
            Sigma, Lbar = make_inputs(i)
            ev = torch.cuda.Event()
            ev.record()
            server.submit(Request(i, Sigma, Lbar, ready=ev, t_arrive=t0 + arrivals[i]))
            i += 1
        done = server.step()
        for r in done:
            if on_done is not None:
                on_done(r)
            if not keep_buffers:
                r.Sigma = r.Lbar = None
        done_all += done
        if not done and (i >= len(arrivals) or arrivals[i] > time.perf_counter() - t0):
            time.sleep(poll_s)
    return done_all, time.perf_counter() - t0


def latency_summary(requests, wall_s):
    """p50 / p99 / mean latency in ms, solves/s, per route counts."""
    lat = np.array([r.latency for r in requests]) * 1e3
    out = {"requests": len(requests), "wall_s": round(wall_s, 3),
           "solves_per_s": round(len(requests) / wall_s, 1) if wall_s > 0 else None}
    if len(lat):
        out.update({"p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "mean_ms": round(float(lat.mean()), 3)})
    for route in ("small", "large"):
        sel = np.array([r.latency for r in requests if r.route == route]) * 1e3
        if len(sel):
            out[f"{route}_requests"] = int(len(sel))
            out[f"{route}_p50_ms"] = round(float(np.percentile(sel, 50)), 3)
            out[f"{route}_p99_ms"] = round(float(np.percentile(sel, 99)), 3)
    return out
