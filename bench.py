#!/usr/bin/env python3
"""Benchmark of the blocked Cholesky derivative path on one MI355X.

Workload: the N = 16384 squared-exponential kernel matrix (3-D inputs, lengthscale 0.2,
nugget 1e-2), built on the device from a fixed seed.  One step is the whole path on it:
    L = chol_factor(Sigma);  Sigma-bar = chol_rev(L, L-bar);  L-dot = chol_fwd(L, Sigma-dot)
(each preceded by a device copy of its input, since the calls work in place).  The reported value
is chol_rev's throughput, (2/3) N^3 flops per call over the event-timed duration of the chol_rev
calls inside the timed steps; per-call figures for all three sweeps are reported beside it.
Each step also runs the batched form once: 2048 SPD matrices (n log-uniform in [16, 512]) through
factor + Gaussian-process loss + reverse sweep in one launch; its solves/s and launch-time
percentiles are reported under "batched", and those of the same matrices in FP32 storage under
"batched_f32".  The three sweeps in the reduced-precision modes (trailing contractions on FP32
MFMA, or as split-bfloat16 MFMA products) are timed alone under "f64_trail_f32" and
"f64_trail_bf16x3"; the headline value stays the FP64 path's.  The three sweeps on the
N = 4096 workload (lengthscale 0.3, nugget 1e-4) are timed for nb = 64, 128 and 256 under
"n4096_by_nb", and one call of each on the N = 256 dense case under "n256_latency".  Under
"serving", a 60 s Poisson stream of factor + chol_rev requests of uneven size runs through the
continuous-batching loop (paper_1602_07527_amd.serve) in both precision modes (p50/p99 latency and
solves/s), then compressed in time to find where each mode saturates, with the per-request error of
the mixed mode against the FP64 one.

Roofline: the dominant kernel (chol_rev's panel contraction) is timed per launch by HIP events the
library records around each launch on the call's stream, in a kernel-timing pass of one or two
extra steps after the timed ones (the events leave the GPU idle for a few microseconds per launch,
so the timed steps run without them).

Output: one JSON line on stdout.  `--gpus` above 1 is refused (single-GPU build).

HBM traffic of the dominant kernel: run this script twice under `rocprofv3 --pmc FETCH_SIZE` and
`--pmc WRITE_SIZE` with `--steps 1 --warmup 0 --cpu-sample 0 --batch-launches 0
--calibration-mib 1024` (the calibration is one plain elementwise copy, torch.neg, of a known
size, whose counters give the scale factor), then `--ingest-pmc FETCH.csv WRITE.csv
--calibration-mib 1024` writes the per-launch record that later runs report as roofline.traffic
while the kernel source and the sweep code that chooses its launches are unchanged.
"""
import csv
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chol_rev TFLOP/s at N=16384 (% MFMA peak); batched solves/s + p99 latency"
FP64_PEAK_TFLOPS = 78.6          # MI355X dense FP64 matrix (MFMA) peak
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_rev_panel_contraction.json")
GEMM_SOURCE = os.path.join(ROOT, "paper_1602_07527_amd", "csrc", "cg_gemm.hpp")
SCHEDULE_SOURCE = os.path.join(ROOT, "paper_1602_07527_amd", "csrc", "cholgrad.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hashes():
    """SHA-256 of the contraction kernel's source and of the sweep code that chooses its launches
    (shapes, splits): a traffic record is valid only for the pair it was taken with."""
    return {"kernel_source_sha256": hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest(),
            "schedule_source_sha256": hashlib.sha256(open(SCHEDULE_SOURCE, "rb").read()).hexdigest()}


def traffic_for(hashes):
    """HBM bytes per launch of the reverse-sweep contraction from the committed rocprofv3 PMC
    record, or None when there is none or the kernel or its launch schedule has changed since it
    was taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if any(rec.get(k) != v for k, v in hashes.items()):
        return None
    return rec.get("hbm_bytes_per_launch")


TARGET_KERNEL = "gemm_f64_dma_kernel<false, false, 1, 0, false, true>"
CALIBRATION_KERNEL = "neg_kernel"


def _pmc_rows(path, counter):
    """(kernel name, grid size, value) per dispatch of a rocprofv3 counter_collection.csv."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            rows.append((r["Kernel_Name"], int(float(r.get("Grid_Size", 0) or 0)), float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"{path}: no {counter} rows")
    return rows


def ingest_pmc(fetch_csv, write_csv, calibration_mib):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what they read for the calibration copy
    of known size and record the per-launch HBM bytes of the reverse-sweep contraction."""
    known = calibration_mib * 2 ** 20
    rec = {"kernel": TARGET_KERNEL, **source_hashes(),
           "calibration": f"torch.neg of {calibration_mib} MiB float64 (reads and writes {known} bytes)"}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows(path, counter)
        cal = [v for k, g, v in rows if CALIBRATION_KERNEL in k]
        tgt = [v for k, g, v in rows if TARGET_KERNEL in k]
        if not cal or not tgt:
            raise SystemExit(f"{path}: calibration ({len(cal)}) or target ({len(tgt)}) dispatches missing")
        factor = known / (max(cal) * 1024.0)
        per[counter] = {"launches": len(tgt), "raw_kib_per_launch": sum(tgt) / len(tgt),
                        "calibration_raw_kib": max(cal), "scale": factor,
                        "bytes_per_launch": factor * 1024.0 * sum(tgt) / len(tgt)}
    rec["counters"] = per
    rec["hbm_bytes_per_launch"] = per["FETCH_SIZE"]["bytes_per_launch"] + per["WRITE_SIZE"]["bytes_per_launch"]
    os.makedirs(os.path.dirname(TRAFFIC_RECORD), exist_ok=True)
    with open(TRAFFIC_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


def cpu_baseline(Sigma_dev, Lbar_dev, n_sample):
    """The oracle's chol_rev (eqn (symrev), host LAPACK) on the leading n_sample block of the same
    workload: the leading block of a Cholesky factor is the factor of the leading block."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()
                       if p.get("user_api") == "blas"] or [1])
    except Exception:      # threadpoolctl missing: fall back to the affinity mask
        threads = len(os.sched_getaffinity(0))
    S = Sigma_dev[:n_sample, :n_sample].cpu().numpy()
    Lb = Lbar_dev[:n_sample, :n_sample].cpu().numpy()
    L, info = oracle.chol(S)
    assert info == 0
    t0 = time.perf_counter()
    oracle.chol_rev(L, Lb)
    dt = time.perf_counter() - t0
    flops = 2.0 / 3.0 * n_sample ** 3
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle chol_rev (eqn symrev, FP64, host LAPACK) on the leading "
                      f"{n_sample}x{n_sample} block of the same N=16384 workload, one call, "
                      f"{dt:.2f} s"}


def batched_setup(dev, dtype=None):
    """The batched workload on the device: 2048 matrices, n log-uniform in [16, 512],
    Sigma = A A^T/n + 0.1 I, y ~ N(0,1), packed back to back in one buffer (so the per-step input
    copy is one device copy) with per-matrix row-major views; float64, or float32 storage."""
    import numpy as np
    import torch
    import paper_1602_07527_amd as cg
    import workloads
    case = workloads.batch_case()
    sizes = [int(n) for n in case["sizes"]]
    offs = np.concatenate([[0], np.cumsum([n * n for n in sizes])])
    host = np.empty(int(offs[-1]))
    for i, S in enumerate(case["Sigma"]):
        host[offs[i]:offs[i + 1]] = S.ravel()
    dtype = dtype or torch.float64
    master = torch.from_numpy(host).to(dev).to(dtype)
    work = torch.empty_like(master)
    grad = torch.empty_like(master)
    views = lambda buf: [buf[offs[i]:offs[i + 1]].view(n, n) for i, n in enumerate(sizes)]
    ys = cg.Vecs([torch.from_numpy(y).to(dev).to(dtype) for y in case["y"]])
    A, G = cg.Batch(views(work)), cg.Batch(views(grad))
    ws = torch.empty(cg.batched_workspace_bytes(len(sizes), max(sizes), A.prec), dtype=torch.uint8, device=dev)
    f = torch.empty(len(sizes), dtype=dtype, device=dev)
    info = torch.empty(len(sizes), dtype=torch.int32, device=dev)
    n3 = float(sum(n ** 3 for n in sizes))
    n2 = float(sum(n * n for n in sizes))
    return {"master": master, "work": work, "A": A, "G": G, "ys": ys, "ws": ws, "f": f, "info": info,
            "batch": len(sizes), "flops": n3 / 3.0 + 2.0 / 3.0 * n3, "bytes": 2.0 * master.element_size() * n2}


def batched_run(cg, b):
    b["work"].copy_(b["master"])
    cg.chol_gp_nll_batched(b["A"], b["ys"], b["G"], f=b["f"], info=b["info"], workspace=b["ws"])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--nb", type=int, default=0,
                    help="block width of all three sweeps (0: the measured per-sweep choice, "
                         "256 for the FP64 sweeps, chol_fwd 128 in the reduced-precision modes)")
    ap.add_argument("--batch-launches", type=int, default=50,
                    help="timed launches of the batched path for its latency percentiles")
    ap.add_argument("--cpu-sample", type=int, default=10240,
                    help="leading-block size for the CPU oracle baseline (0 skips it)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served request stream (0 skips it)")
    ap.add_argument("--n4096-steps", type=int, default=5,
                    help="timed passes of the N=4096 sweeps for each nb (0 skips them)")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="timed passes of each reduced-precision mode and of chol_factor_fwd (0 skips them)")
    ap.add_argument("--calibration-mib", type=int, default=0,
                    help="run one plain elementwise copy of this size first (PMC calibration)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc runs into the traffic record and exit")
    args = ap.parse_args()
    if args.ingest_pmc:
        if args.calibration_mib <= 0:
            raise SystemExit("--ingest-pmc needs the --calibration-mib of the profiled runs")
        ingest_pmc(*args.ingest_pmc, args.calibration_mib)
        return
    if args.gpus != 1:
        print(f"bench.py: the path is measured on one GPU (no multi-GPU sharding); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1602_07527_amd as cg
    import workloads

    cg.load_library()
    dev = torch.device("cuda:0")
    n = args.n
    # Block widths per sweep (measured on MI355X at N = 16384: chol_rev 54.1 ms at nb = 256 against
    # 55.9 ms at 128, chol_factor 35.6 against 36.6, chol_fwd 50.9 against 54.2 (with the 128 x 256
    # paired tiles; 59.3 against 56.9 before them), the one-sweep factor + forward 87.1 against
    # 93.2).  The reduced-precision forward sweep keeps 128: its contractions take no wide tiles.
    nb_rev, nb_fac, nb_fwd = (args.nb, args.nb, args.nb) if args.nb else (256, 256, 256)
    nb_ff = args.nb or 256
    nb_fwd_mixed = args.nb or 128
    log(f"[bench] building the N={n} workload on the device")
    inp = workloads.large_case_device(dev, N=n)
    Sigma, Lbar, Sdot = inp["Sigma"], inp["Lbar"], inp["Sdot"]
    A = torch.empty_like(Sigma)
    Ab = torch.empty_like(Sigma)
    Ad = torch.empty_like(Sigma)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_bytes = max(cg.workspace_bytes(op, n, b) for op in ("factor", "rev", "fwd") for b in {nb_rev, nb_fac, nb_fwd, nb_ff, nb_fwd_mixed})
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(2)] for k in ("f", "r", "d", "b", "r2", "d2")}
    times = {"f": 0.0, "r": 0.0, "d": 0.0, "b": 0.0}
    if args.calibration_mib > 0:
        src = torch.ones(args.calibration_mib * 2 ** 17, dtype=torch.float64, device=dev)
        torch.neg(src, out=torch.empty_like(src))
        torch.cuda.synchronize()
        del src
        log(f"[bench] calibration copy of {args.calibration_mib} MiB done")
    log("[bench] building the batched workload (2048 matrices)")
    bat = batched_setup(dev)

    def step(record):
        A.copy_(Sigma)
        if record: ev["f"][0].record()
        cg.chol_factor(A, nb=nb_fac, workspace=ws, info=info)
        if record: ev["f"][1].record()
        Ab.copy_(Lbar)
        if record: ev["r"][0].record()
        cg.chol_rev(A, Ab, nb=nb_rev, workspace=ws)
        if record: ev["r"][1].record()
        Ad.copy_(Sdot)
        if record: ev["d"][0].record()
        cg.chol_fwd(A, Ad, nb=nb_fwd, workspace=ws)
        if record: ev["d"][1].record()
        bat["work"].copy_(bat["master"])
        if record: ev["b"][0].record()
        cg.chol_gp_nll_batched(bat["A"], bat["ys"], bat["G"], f=bat["f"], info=bat["info"], workspace=bat["ws"])
        if record: ev["b"][1].record()

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    if int(info.item()) != 0:
        raise RuntimeError(f"chol_factor reported info={int(info.item())}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        for k in times:
            times[k] += ev[k][0].elapsed_time(ev[k][1])
        log(f"[bench] timed step {i + 1}/{args.steps}: rev {ev['r'][0].elapsed_time(ev['r'][1]):.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # Kernel-level timing for the roofline: the same step again with the library's HIP events
    # around every panel-contraction launch (recorded on the stream the kernels run on).  A pass
    # of its own, because the events between launches leave the GPU idle for a few microseconds
    # each (about 1.8 ms per chol_rev call), which the timed steps above must not include.
    prof_steps = max(1, min(args.steps, 2))
    cg.profile_begin()
    for i in range(prof_steps):
        step(False)
        torch.cuda.synchronize()
    prof = cg.profile_end()
    log(f"[bench] kernel-timing pass of {prof_steps} step(s) done")
    if int(info.item()) != 0:
        raise RuntimeError(f"chol_factor reported info={int(info.item())}")
    if not bool(torch.isfinite(Ab).all()) or not bool(torch.isfinite(Ad).all()):
        raise RuntimeError("non-finite result")
    if int((bat["info"] != 0).sum()) != 0 or not bool(torch.isfinite(bat["f"]).all()):
        raise RuntimeError("batched factorisation failed")

    # Latency of one call on the N = 256 dense workload (A A^T/N + I, host-built; nb = 0, the
    # library's width per sweep and size: 128 for chol_factor, 256 for chol_rev and chol_fwd):
    # median of 20 event-timed calls each.
    small = None
    if args.n4096_steps > 0:
        import statistics
        log("[bench] N=256 call latency")
        c = workloads.small_case()
        S256 = torch.from_numpy(c["Sigma"]).to(dev)
        Lb256 = torch.from_numpy(c["Lbar"]).to(dev)
        Sd256 = torch.from_numpy(c["Sdot"]).to(dev).tril()
        A3, B3, D3 = torch.empty_like(S256), torch.empty_like(S256), torch.empty_like(S256)
        ws3 = torch.empty(max(cg.workspace_bytes(op, 256, 0) for op in ("factor", "rev", "fwd")),
                          dtype=torch.uint8, device=dev)
        info3 = torch.empty(1, dtype=torch.int32, device=dev)
        t = {"f": [], "r": [], "d": []}
        for i in range(21):
            A3.copy_(S256)
            B3.copy_(Lb256)
            D3.copy_(Sd256)
            torch.cuda.synchronize()
            ev["f"][0].record()
            cg.chol_factor(A3, nb=0, workspace=ws3, info=info3)
            ev["f"][1].record()
            ev["r"][0].record()
            cg.chol_rev(A3, B3, nb=0, workspace=ws3)
            ev["r"][1].record()
            ev["d"][0].record()
            cg.chol_fwd(A3, D3, nb=0, workspace=ws3)
            ev["d"][1].record()
            torch.cuda.synchronize()
            if i > 0:
                for k in t:
                    t[k].append(ev[k][0].elapsed_time(ev[k][1]) * 1e3)
        if int(info3.item()) != 0:
            raise RuntimeError("N=256 chol_factor failed")
        small = {"workload": "dense SPD N=256 (A A^T/N + I), nb=0 (library choice: chol_factor 128, "
                             "chol_rev and chol_fwd 256); median of 20 event-timed calls",
                 "chol_factor_us": round(statistics.median(t["f"]), 1),
                 "chol_rev_us": round(statistics.median(t["r"]), 1),
                 "chol_fwd_us": round(statistics.median(t["d"]), 1)}
        del A3, B3, D3, ws3

    # The N = 4096 workload (3-D squared-exponential kernel, lengthscale 0.3, nugget 1e-4, built on
    # the device) for each block width nb: the three sweeps timed alone (median of the timed
    # passes, after one untimed pass).
    by_nb = None
    if args.n4096_steps > 0:
        import statistics
        log("[bench] N=4096 sweeps by nb")
        m = workloads.se_case_device(4096, workloads.SEED_MEDIUM, 0.3, 1e-4, dev)
        n2 = 4096
        A2, B2, D2 = torch.empty_like(m["Sigma"]), torch.empty_like(m["Sigma"]), torch.empty_like(m["Sigma"])
        ws2 = torch.empty(max(cg.workspace_bytes(op, n2, nbv) for op in ("factor", "rev", "fwd") for nbv in (64, 128, 256)),
                          dtype=torch.uint8, device=dev)
        info2 = torch.empty(1, dtype=torch.int32, device=dev)
        by_nb = {"workload": "squared-exponential kernel matrix N=4096 (3-D inputs, lengthscale 0.3, nugget "
                             "1e-4, built on the device); median of the timed passes per nb; chol_rev/chol_fwd "
                             "with the default (symbolic) diagonal-block variant and, as *_level2_ms, with the "
                             "Level-2 one"}
        for nbv in (64, 128, 256):
            t = {"f": [], "r": [], "d": []}
            for i in range(args.n4096_steps + 1):
                A2.copy_(m["Sigma"])
                ev["f"][0].record()
                cg.chol_factor(A2, nb=nbv, workspace=ws2, info=info2)
                ev["f"][1].record()
                B2.copy_(m["Lbar"])
                ev["r"][0].record()
                cg.chol_rev(A2, B2, nb=nbv, workspace=ws2)
                ev["r"][1].record()
                D2.copy_(m["Sdot"])
                ev["d"][0].record()
                cg.chol_fwd(A2, D2, nb=nbv, workspace=ws2)
                ev["d"][1].record()
                torch.cuda.synchronize()
                if i > 0:
                    for k in t:
                        t[k].append(ev[k][0].elapsed_time(ev[k][1]))
            if int(info2.item()) != 0:
                raise RuntimeError(f"N=4096 chol_factor failed at nb={nbv}")
            med = {k: statistics.median(v) for k, v in t.items()}
            by_nb[f"nb{nbv}"] = {
                "chol_factor_ms": round(med["f"], 3), "chol_factor_tflops": round(n2 ** 3 / 3.0 / (med["f"] * 1e-3) / 1e12, 2),
                "chol_rev_ms": round(med["r"], 3), "chol_rev_tflops": round(2.0 / 3.0 * n2 ** 3 / (med["r"] * 1e-3) / 1e12, 2),
                "chol_fwd_ms": round(med["d"], 3), "chol_fwd_tflops": round(2.0 / 3.0 * n2 ** 3 / (med["d"] * 1e-3) / 1e12, 2)}
        # The Level-2 diagonal-block variant (blocks up to 128 wide), in a pass of its own on the
        # last factor (A2).
        for nbv in (64, 128):
            t = {"r2": [], "d2": []}
            for i in range(args.n4096_steps + 1):
                B2.copy_(m["Lbar"])
                ev["r2"][0].record()
                cg.chol_rev(A2, B2, nb=nbv, workspace=ws2, diag="level2")
                ev["r2"][1].record()
                D2.copy_(m["Sdot"])
                ev["d2"][0].record()
                cg.chol_fwd(A2, D2, nb=nbv, workspace=ws2, diag="level2")
                ev["d2"][1].record()
                torch.cuda.synchronize()
                if i > 0:
                    for k in t:
                        t[k].append(ev[k][0].elapsed_time(ev[k][1]))
            by_nb[f"nb{nbv}"]["chol_rev_level2_ms"] = round(statistics.median(t["r2"]), 3)
            by_nb[f"nb{nbv}"]["chol_fwd_level2_ms"] = round(statistics.median(t["d2"]), 3)
        del m, A2, B2, D2, ws2

    # chol_factor_fwd: potrf and the forward sweep in one pass, timed alone after one untimed pass.
    fused = None
    if args.mixed_steps > 0:
        log("[bench] chol_factor_fwd (one sweep)")
        fused_ms = 0.0
        for i in range(args.mixed_steps + 1):
            A.copy_(Sigma)
            Ad.copy_(Sdot)
            ev["f"][0].record()
            cg.chol_factor_fwd(A, Ad, nb=nb_ff, workspace=ws, info=info)
            ev["f"][1].record()
            torch.cuda.synchronize()
            if i > 0:
                fused_ms += ev["f"][0].elapsed_time(ev["f"][1]) / args.mixed_steps
        if int(info.item()) != 0:
            raise RuntimeError("chol_factor_fwd failed")
        fused = {"chol_factor_fwd_ms": round(fused_ms, 3),
                 "tflops": round(n ** 3 / (fused_ms * 1e-3) / 1e12, 3),
                 "separate_ms": None}

    # The reduced-precision modes (trailing contractions on FP32 MFMA, or as three bfloat16 MFMA
    # products of split operands) on the same workload: the three sweeps timed alone, after one
    # untimed pass.
    MODE_TEXT = {"f64_trail_f32": "FP64 storage; trailing contractions on FP32 MFMA",
                 "f64_trail_bf16x3": "FP64 storage; trailing contractions as hi*hi + hi*lo + lo*hi "
                                     "bfloat16 MFMA products with FP32 accumulation",
                 "f64_trail_bf16x6": "FP64 storage; trailing contractions as six bfloat16 MFMA products "
                                     "of three-part split operands with FP32 accumulation"}
    mixed = {}
    for mode in (MODE_TEXT if args.mixed_steps > 0 else ()):
        log(f"[bench] {mode} sweeps")
        mt = {"f": 0.0, "r": 0.0, "d": 0.0}
        for i in range(args.mixed_steps + 1):
            A.copy_(Sigma)
            ev["f"][0].record()
            cg.chol_factor(A, nb=nb_fac, workspace=ws, info=info, precision=mode)
            ev["f"][1].record()
            Ab.copy_(Lbar)
            ev["r"][0].record()
            cg.chol_rev(A, Ab, nb=nb_rev, workspace=ws, precision=mode)
            ev["r"][1].record()
            Ad.copy_(Sdot)
            ev["d"][0].record()
            cg.chol_fwd(A, Ad, nb=nb_fwd_mixed, workspace=ws, precision=mode)
            ev["d"][1].record()
            torch.cuda.synchronize()
            if i > 0:
                for k in mt:
                    mt[k] += ev[k][0].elapsed_time(ev[k][1]) / args.mixed_steps
        if int(info.item()) != 0:
            raise RuntimeError(f"{mode} chol_factor failed")
        mixed[mode] = {"mode": MODE_TEXT[mode] + "; diagonal blocks and panel solves FP64 (accuracy "
                                                 "stated and tested separately)",
                       "steps": args.mixed_steps,
                       "nb": {"chol_rev": nb_rev, "chol_factor": nb_fac, "chol_fwd": nb_fwd_mixed},
                       "chol_rev_ms": round(mt["r"], 3),
                       "chol_rev_tflops": round(2.0 / 3.0 * n ** 3 / (mt["r"] * 1e-3) / 1e12, 3),
                       "chol_factor_ms": round(mt["f"], 3),
                       "chol_factor_tflops": round(n ** 3 / 3.0 / (mt["f"] * 1e-3) / 1e12, 3),
                       "chol_fwd_ms": round(mt["d"], 3),
                       "chol_fwd_tflops": round(2.0 / 3.0 * n ** 3 / (mt["d"] * 1e-3) / 1e12, 3)}

    # Launch-time distribution of the one-launch batched path (factor + loss + reverse sweep), for
    # FP64 storage (the bench workload) and FP32 storage of the same matrices.
    import numpy as np

    def launch_times(b, launches):
        lat = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(launches):
            b["work"].copy_(b["master"])
            e0.record()
            cg.chol_gp_nll_batched(b["A"], b["ys"], b["G"], f=b["f"], info=b["info"], workspace=b["ws"])
            e1.record()
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1))
        if int((b["info"] != 0).sum()) != 0 or not bool(torch.isfinite(b["f"]).all()):
            raise RuntimeError("batched factorisation failed")
        return np.array(lat)

    def batched_summary(b, lat, storage):
        p50 = float(np.percentile(lat, 50))
        return {"workload": f"2048 SPD matrices, n log-uniform in [16, 512], A A^T/n + 0.1 I, {storage} "
                            "storage; one launch = factor + GP loss + chol_rev per matrix (chol_gp_nll_batched)",
                "launches": int(len(lat)), "ms_p50": round(p50, 3),
                "ms_p99": round(float(np.percentile(lat, 99)), 3),
                "solves_per_s": round(b["batch"] / (p50 * 1e-3), 1),
                "tflops": round(b["flops"] / (p50 * 1e-3) / 1e12, 3),
                "gbps_algorithmic": round(b["bytes"] / (p50 * 1e-3) / 1e9, 1)}

    lat = launch_times(bat, args.batch_launches) if args.batch_launches > 0 else \
        np.array([times["b"] / args.steps])   # no separate launches: the in-step time
    batched = batched_summary(bat, lat, "FP64")
    batched["in_step_ms"] = round(times["b"] / args.steps, 3)
    batched_f32 = None
    if args.batch_launches > 0:
        log("[bench] FP32-storage batched launches")
        bat32 = batched_setup(dev, torch.float32)
        batched_f32 = batched_summary(bat32, launch_times(bat32, args.batch_launches), "FP32")
        del bat32

    # Serving: the Poisson request stream (200 requests/s, n log-uniform in [64, 4096], 2-D
    # squared-exponential kernels), factor + chol_rev per request through the continuous-batching
    # loop, in FP64 and with FP32-MFMA trailing contractions for the large requests; then the same
    # stream compressed in time (its first requests offered at higher rates) to find where each
    # mode saturates, and the per-request error of the mixed mode against the FP64 one.
    serving = None
    if args.serve_seconds > 0:
        from paper_1602_07527_amd import serve
        tr = workloads.serve_trace(rate=200.0, seconds=args.serve_seconds)
        make = lambda i: workloads.se_request_device(tr["n"][i], tr["lengthscale"][i], tr["seed"][i], dev)
        serving = {"workload": f"Poisson arrivals at 200/s for {args.serve_seconds:g} s ({len(tr['t'])} "
                               "requests), n log-uniform in [64, 4096], SE kernel on U[0,1]^2 (lengthscale "
                               "U[0.1, 0.5]) + 1e-3 I, L-bar = tril N(0,1); one request = chol_factor + "
                               "chol_rev; HBM budget 64 GiB; inputs built on the device as each request "
                               "arrives (included in the latency)", "n_mean": round(float(tr["n"].mean()), 1)}
        for mode in ("f64", "f64_trail_f32"):
            log(f"[bench] serving {args.serve_seconds:g} s in {mode}")
            srv = serve.Server(dev, hbm_budget=64 << 30, precision=mode)
            done, wall = serve.replay(srv, tr["t"], make)
            if any(int(r.info.item()) != 0 for r in done):
                raise RuntimeError("a served factorisation failed")
            serving[mode] = serve.latency_summary(done, wall)
            serving[mode]["launches"] = dict(srv.launches)
            serving[mode]["peak_admitted_gib"] = round(srv.peak_in_use / 2 ** 30, 3)
            del done, srv
        # Saturation: the first SAT_REQ requests of the same stream with their arrival times divided
        # by rate / 200, per mode; sustained = completed / wall clock.
        SAT_REQ = min(len(tr["t"]), 1500)
        sat = {"requests_per_point": SAT_REQ,
               "note": "offered rate = the stream's first requests with arrival times compressed; their "
                       "inputs are built once beforehand and each arrival is a device copy of them, so "
                       "the host loop's input generation does not cap the rate; p99 includes queueing "
                       "once the offered rate exceeds what the loop sustains"}
        log(f"[bench] serving saturation: building the inputs of the first {SAT_REQ} requests")
        pool = [make(i) for i in range(SAT_REQ)]
        make_sat = lambda i: (pool[i][0].clone(), pool[i][1].clone())
        for mode in ("f64", "f64_trail_f32"):
            pts = []
            for rate in (400.0, 600.0, 800.0, 1000.0, 1200.0):
                log(f"[bench] serving saturation {mode} at {rate:g}/s")
                # every point starts from an empty allocator cache (the previous point's blocks
                # are released outside the timed replay)
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                srv = serve.Server(dev, hbm_budget=64 << 30, precision=mode)
                done, wall = serve.replay(srv, tr["t"][:SAT_REQ] * (200.0 / rate), make_sat)
                lat = np.array([r.latency for r in done]) * 1e3
                pts.append({"offered_per_s": rate, "solves_per_s": round(len(done) / wall, 1),
                            "p50_ms": round(float(np.percentile(lat, 50)), 3),
                            "p99_ms": round(float(np.percentile(lat, 99)), 3)})
                del done, srv
            sat[mode] = pts
        serving["saturation"] = sat
        del pool
        # Per-request error of the mixed mode: a seeded sample of the stream plus its ten
        # worst-conditioned requests (largest n * lengthscale), each solved in both modes on the same
        # GPU; relative Frobenius error of L and Sigma-bar against the FP64 result (which is within
        # max(1e-10, 100 kappa u) of the oracle).
        log("[bench] serving: mixed-precision error sample")
        rng = np.random.default_rng(17)
        pick = np.unique(np.concatenate([rng.choice(len(tr["t"]), size=min(150, len(tr["t"])), replace=False),
                                         np.argsort(tr["n"] * tr["lengthscale"])[-10:]]))
        eL, eS = [], []
        for i in pick:
            if tr["n"][i] <= serve.SMALL_MAX:   # small requests are served by the FP64 batched path
                eL.append(0.0)
                eS.append(0.0)
                continue
            res = {}
            for mode in ("f64", "f64_trail_f32"):
                S_i, Lb_i = make(int(i))
                Lf, _ = cg.chol_factor(S_i, precision=mode)
                cg.chol_rev(Lf, Lb_i, precision=mode)
                res[mode] = (Lf, Lb_i)
            (L64, S64), (L32, S32) = res["f64"], res["f64_trail_f32"]
            eL.append(float(torch.linalg.norm(L32 - L64) / torch.linalg.norm(L64)))
            eS.append(float(torch.linalg.norm(S32 - S64) / torch.linalg.norm(S64)))
        eL, eS = np.array(eL), np.array(eS)
        serving["f64_trail_f32"]["error_vs_f64"] = {
            "requests": int(len(pick)), "rel_sbar_p50": float(np.percentile(eS, 50)),
            "rel_sbar_p95": float(np.percentile(eS, 95)), "rel_sbar_max": float(eS.max()),
            "rel_l_max": float(eL.max()), "stated_bound_rel_sbar": 2e-2, "stated_bound_rel_l": 6e-4,
            "note": "requests with n <= 512 run on the FP64 batched path in both modes (error 0)"}

    K = args.steps
    ms_step = (t1 - t0) * 1e3 / K
    if fused is not None:
        fused["separate_ms"] = round((times["f"] + times["d"]) / K, 3)
    f_rev = 2.0 / 3.0 * n ** 3
    f_fac = n ** 3 / 3.0
    rev_ms = times["r"] / K
    fac_ms = times["f"] / K
    fwd_ms = times["d"] / K
    rev_tflops = f_rev / (rev_ms * 1e-3) / 1e12

    k_ms, k_flops, k_bytes, k_launch = prof["rev"]
    achieved = k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
    traffic = traffic_for(source_hashes())
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "gemm_f64_dma_kernel<false,false,1,0,false,true> (reverse-sweep panel contraction, 128x256 tiles, FP64 MFMA, stream-K)",
                "kernel_avg_us": round(k_ms * 1e3 / max(k_launch, 1), 2),
                "algorithmic_bytes_per_launch": round(k_bytes / max(k_launch, 1)),
                "algorithmic_flops_per_launch": round(k_flops / max(k_launch, 1)),
                "launches_per_step": k_launch // prof_steps,
                "kernel_timing": f"library HIP events around each launch, {prof_steps} extra step(s) after the timed ones"}

    out = {
        "metric": METRIC, "value": round(rev_tflops, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"squared-exponential kernel matrix N={n} (3-D inputs, lengthscale "
                               f"0.2, nugget 1e-2); step = chol_factor + chol_rev + chol_fwd",
                   "n": n, "nb": {"chol_rev": nb_rev, "chol_factor": nb_fac, "chol_fwd": nb_fwd,
                                  "chol_factor_fwd": nb_ff}},
        "pct_fp64_peak": round(100 * rev_tflops / FP64_PEAK_TFLOPS, 2),
        "chol_rev_ms": round(rev_ms, 3), "chol_factor_ms": round(fac_ms, 3),
        "chol_fwd_ms": round(fwd_ms, 3),
        "chol_factor_tflops": round(f_fac / (fac_ms * 1e-3) / 1e12, 3),
        "chol_fwd_tflops": round(f_rev / (fwd_ms * 1e-3) / 1e12, 3),
        "roofline": roofline,
        "batched": batched,
        "batched_f32": batched_f32,
        "n256_latency": small,
        "n4096_by_nb": by_nb,
        "factor_fwd_one_sweep": fused,
        "f64_trail_f32": mixed.get("f64_trail_f32"),
        "f64_trail_bf16x3": mixed.get("f64_trail_bf16x3"),
        "f64_trail_bf16x6": mixed.get("f64_trail_bf16x6"),
        "serving": serving,
    }
    if args.cpu_sample > 0:
        log(f"[bench] timing the CPU oracle on a {args.cpu_sample} sample")
        out["cpu_baseline"] = cpu_baseline(Sigma, Lbar, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
