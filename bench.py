#!/usr/bin/env python3
"""Benchmark of the 4-point homography hot path on one MI355X.

Headline (the timed steps): the batched ACA solve of 2^26 random quadruples
(fp32 SoA planes in HBM, double-precision arithmetic, 9 fp32 planes + a flag
byte out); value = homographies per second. One step = one launch over the
whole batch, inputs resident in HBM before timing starts.

The JSON line also carries the roofline of the solver kernel, the CPU oracle
timed on a bounded sample of the same workload, and secondary measurements of
the other stages of the path (SKS, small-batch latency, the three-point affine,
the simplified SK, RANSAC scoring, batched and adaptive RANSAC, the
differentiable pipeline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4-pt homographies/s + RANSAC hyp·pts/s vs plain form, 1 MI355X, ≤1e-5 rel err"
HBM_PEAK_GBS = 8000.0
BYTES_PER_QUAD = 64 + 36 + 1      # 16 fp32 in, 9 fp32 out, 1 flag byte
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "solve4_aca_2p26_traffic.json")
SOLVER_SOURCES = [os.path.join(ROOT, "paper_2402_18008_amd", "csrc", f)
                  for f in ("solve.hip", "solver_dev.hpp")]


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def solver_hash():
    h = hashlib.sha256()
    for p in SOLVER_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def oracle_fp64_error():
    """The oracle's own float64 error against the exact rational DLT per
    workload (max and p99 over 512 problems), as stored beside the tests by a
    script that calls only the oracle; None if the file is absent."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_fp64_error.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return {k: {"max": v["max"], "p99": v["p99"], "n": v["n"]} for k, v in t.items()}


def measured_traffic(n):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current solver source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != solver_hash() or t.get("n") != n:
        return None
    return t.get("bytes_per_launch")


def write_traffic(fetch_dir, write_dir, n):
    """Solver HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counters
    (KiB per dispatch), each scaled by what the same counter reads for a plain
    copy of known size in the same run; written to TRAFFIC_FILE."""
    import csv
    from collections import defaultdict

    def per_kernel(folder, counter):
        per = defaultdict(list)
        with open(os.path.join(folder, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return {k: 1024.0 * sum(v) / len(v) for k, v in per.items()}

    def pick(d, key):
        ks = [k for k in d if key in k]
        if len(ks) != 1:
            raise SystemExit(f"expected one kernel matching {key!r}, found {ks}")
        return d[ks[0]]

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = 8 * n * 4                      # the 8 source planes, each way
    f_copy, w_copy = pick(fetch, "stream_copy4_kernel"), pick(write, "stream_copy4_kernel")
    f_sol, w_sol = pick(fetch, "solve4_kernel<0>"), pick(write, "solve4_kernel<0>")
    ff, wf = copy_bytes / f_copy, copy_bytes / w_copy
    cmd = ("rocprofv3 --pmc {c} --output-format csv -d gpurun_out/pmc_{c} -o run -- python3 "
           "bench.py --part solver --with-copy --steps 3 --warmup 1 --no-cpu-baseline "
           "--gen-workers 1")
    out = {
        "kernel": "solve4_kernel<ACA>", "n": n, "source_hash": solver_hash(),
        "command_fetch": cmd.format(c="FETCH_SIZE"), "command_write": cmd.format(c="WRITE_SIZE"),
        "command_summary": "python3 bench.py --traffic-from gpurun_out/pmc_FETCH_SIZE "
                           "gpurun_out/pmc_WRITE_SIZE",
        "fetch_kib_per_dispatch": f_sol / 1024, "write_kib_per_dispatch": w_sol / 1024,
        "copy_fetch_kib_per_dispatch": f_copy / 1024, "copy_write_kib_per_dispatch": w_copy / 1024,
        "copy_bytes_each_way": copy_bytes, "fetch_factor": ff, "write_factor": wf,
        "fetch_bytes": f_sol * ff, "write_bytes": w_sol * wf,
        "bytes_per_launch": f_sol * ff + w_sol * wf,
        "algorithmic_bytes_per_launch": BYTES_PER_QUAD * n,
    }
    out["traffic_over_algorithmic"] = out["bytes_per_launch"] / out["algorithmic_bytes_per_launch"]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def burst_us(fn, stream, launches=200, warmup=10):
    """Per-launch time of `launches` back-to-back eager calls under one event pair
    (host launch cost included where it exceeds the kernel's)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / launches


def graph_us(fn, stream, per_graph=100, replays=10):
    """Per-launch time of fn() replayed from a captured graph of `per_graph`
    back-to-back calls (no host launch cost)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(replays):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / (per_graph * replays)
    del g
    return us


def time_interleaved(fns, rounds, warmup, stream):
    """Per-call times (ms) of several forms queued alternately (order reversed every other
    round) without synchronising in between: the host stays ahead, each interval is the GPU's
    time for one call, and every form sees the same clock state."""
    import torch
    for _ in range(warmup):
        for f in fns.values():
            f()
    torch.cuda.synchronize()
    keys = list(fns)
    evs = {k: [] for k in keys}
    for r in range(rounds):
        for k in (keys if r % 2 == 0 else keys[::-1]):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fns[k]()
            b.record(stream)
            evs[k].append((a, b))
    torch.cuda.synchronize()
    return {k: [a.elapsed_time(b) for a, b in v] for k, v in evs.items()}


def time_launches(fn, steps, warmup, stream):
    """Run fn() warmup times, then time `steps` calls with one event pair each.
    Returns (total_ms, per_launch_ms list)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop), [a.elapsed_time(b) for a, b in evs]


_CB = {}


def _oracle_chunk(rng):
    """Worker: the float64 oracle ACA on quadruples [a, b) of the arrays the
    parent set up before forking (no copy through the pool)."""
    a, b = rng
    import numpy as np
    from oracle import homography as hg
    t = time.perf_counter()
    hg.aca64(_CB["src"][:, a:b].astype(np.float64), _CB["dst"][:, a:b].astype(np.float64))
    return time.perf_counter() - t


def cpu_baseline(src, dst, n_sample, workers):
    """The float64 oracle ACA (NumPy) over the first n_sample quadruples, in
    2^20 chunks over a process pool."""
    import multiprocessing as mp
    chunk = 1 << 20
    jobs = [(a, min(a + chunk, n_sample)) for a in range(0, n_sample, chunk)] * 2
    _CB["src"], _CB["dst"] = src, dst
    ctx = mp.get_context("fork")
    pool = ctx.Pool(workers)
    try:
        pool.map(_oracle_chunk, jobs[:workers])          # warm the workers
        t = time.perf_counter()
        cpu_s = sum(pool.map(_oracle_chunk, jobs))
        wall = time.perf_counter() - t
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return dict(value=2 * n_sample / wall, unit="homographies/s", cores=workers, kind="oracle",
                sample=f"float64 NumPy ACA, two passes over the first {n_sample} quadruples of "
                       f"the same workload, {len(jobs)} chunks of 2^20 over {workers} processes "
                       f"({cpu_s:.1f} s of CPU time, {wall:.2f} s wall)")


SK_BYTES = 32 + 36 + 1            # 8 fp32 in, 9 fp32 out, 1 flag byte
AFFINE_BYTES = 48 + 24 + 1        # 12 fp32 in, 6 fp32 out, 1 flag byte


def stream_ceilings(stream, S, D, H, F, solver_GBps):
    """Streaming rates with no arithmetic: a plain copy, and each solver's exact
    read/write mix and launch shape (16 -> 9 planes + flags for hg_solve4,
    8 -> 9 for the simplified SK, 12 -> 6 for the affine map)."""
    import numpy as np
    import torch
    import paper_2402_18008_amd as hgpu
    n = S.shape[1]
    out = {}
    C = torch.empty_like(S)
    t, p = time_launches(lambda: hgpu.hg_stream_copy(S, C), 20, 3, stream)
    out["copy_GBps"] = 2 * S.numel() * 4 / (np.mean(p) * 1e-3) / 1e9
    del C
    X = torch.empty((16, n), dtype=torch.float32, device=S.device)
    X[:8].copy_(S)
    X[8:].copy_(D)
    for name, n_in, n_out in (("solve4_16to9", 16, 9), ("sk_8to9", 8, 9),
                              ("affine_12to6", 12, 6)):
        xi, ho = X[:n_in], H[:n_out]
        t, p = time_launches(lambda: hgpu.hg_stream_planes(xi, n_out, out=ho, flags=F), 20, 3,
                             stream)
        out[f"{name}_GBps"] = (4 * (n_in + n_out) + 1) * n / (np.mean(p) * 1e-3) / 1e9
    del X
    torch.cuda.synchronize()
    out["solve4_frac_of_its_mix"] = solver_GBps / out["solve4_16to9_GBps"]
    return out


def bench_sk(stream, n, workers, steps=20, warmup=3):
    """Simplified SK: n images of one pattern, one launch."""
    import numpy as np
    import torch
    import synth
    import paper_2402_18008_amd as hgpu
    log(f"simplified SK: generating {n} pattern images")
    D = torch.from_numpy(synth.pattern_images(n, 1, workers=workers)).cuda()
    H = torch.empty((9, n), dtype=torch.float32, device=D.device)
    F = torch.empty(n, dtype=torch.uint8, device=D.device)
    obj = [float(v) for v in synth.PATTERN]
    t, p = time_launches(lambda: hgpu.hg_solve_sk(obj, D, H=H, flags=F), steps, warmup, stream)
    k = float(np.mean(p))
    return {"sk_simplified": {"n": n, "homographies_per_s": n / (t / steps * 1e-3),
                              "kernel_ms": k, "bytes_per_unit": SK_BYTES,
                              "GBps": SK_BYTES * n / (k * 1e-3) / 1e9,
                              "frac_hbm": SK_BYTES * n / (k * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def bench_affine(stream, S, D, steps=20, warmup=3):
    """Three-point affine on the first three points of the quadruple batch."""
    import numpy as np
    import torch
    import paper_2402_18008_amd as hgpu
    n = S.shape[1]
    A = torch.empty((6, n), dtype=torch.float32, device=S.device)
    F = torch.empty(n, dtype=torch.uint8, device=S.device)
    s6, d6 = S[:6], D[:6]
    t, p = time_launches(lambda: hgpu.hg_solve3_affine(s6, d6, A=A, flags=F), steps, warmup,
                         stream)
    k = float(np.mean(p))
    return {"affine3": {"n": n, "maps_per_s": n / (t / steps * 1e-3), "kernel_ms": k,
                        "bytes_per_unit": AFFINE_BYTES,
                        "GBps": AFFINE_BYTES * n / (k * 1e-3) / 1e9,
                        "frac_hbm": AFFINE_BYTES * n / (k * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def host_info():
    """CPU model and the cores this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def _oracle_ransac_job(job):
    """One pair's oracle RANSAC (a process-pool job; the oracle is imported
    in the worker)."""
    from oracle import ransac as oref
    corr, n_hyp, seed, pair = job
    oref.ransac_ref(corr, n_hyp, 3.0, seed, pair=pair)
    return corr.shape[1]


def cpu_oracle_extras():
    """The oracle on the other workloads, timed on the host (bounded samples):
    the host's CPU model and core count; ACA and SKS on one core (4096
    quadruples and a 2^20 chunk); single-pair RANSAC scoring (float64 NumPy,
    one process); the differentiable pipeline (torch float64 autograd through
    the DLT solve)."""
    import torch
    import synth
    from oracle import ransac as oref
    from oracle import warp as ow
    import numpy as np
    from oracle import homography as hg
    out = {"host": host_info()}
    # the 4096-quadruple workload (seed 0) and a 2^20 chunk, each method on one core
    for label, n_q in (("quads_4096", 4096), ("quads_2p20", 1 << 20)):
        s, d, _ = synth.quadruples(n_q, 0)
        s, d = s.astype(np.float64), d.astype(np.float64)
        rates = {}
        for name, fn in (("aca", hg.aca64), ("sks", hg.sks64)):
            reps, t = 0, time.perf_counter()
            while True:
                fn(s, d)
                reps += 1
                dt = time.perf_counter() - t
                if dt > 0.5:
                    break
            rates[f"{name}_homographies_per_s"] = reps * n_q / dt
        out[label] = {**rates, "cores": 1,
                      "sample": f"float64 NumPy oracle ACA and SKS over {n_q} quadruples, repeated "
                                f"for at least 0.5 s, one process"}
    cs = synth.config2()
    t = time.perf_counter()
    oref.ransac_ref(cs.corr, 4096, 3.0, 2)
    dt_r = time.perf_counter() - t
    # all cores: the single-pair workload in every worker process at once, and
    # every 8th pair of the 512-pair batch spread over the workers
    workers = max(1, min(16, host_info()["usable_cpus"]))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_ransac_job, [(cs.corr[:, :64], 64, 2, 0)] * workers)   # warm the workers
        t = time.perf_counter()
        pool.map(_oracle_ransac_job, [(cs.corr, 4096, 2, 0)] * workers, chunksize=1)
        dt_r_all = time.perf_counter() - t
        cb = synth.config3()
        jobs = [(np.ascontiguousarray(cb.corr[:, cb.off[p]:cb.off[p + 1]]), 1024, 3, p)
                for p in range(0, 512, 8)]
        jobs.sort(key=lambda j: -j[0].shape[1])
        t = time.perf_counter()
        pool.map(_oracle_ransac_job, jobs, chunksize=1)
        dt_b = time.perf_counter() - t
    hp_b = float(sum(j[0].shape[1] for j in jobs)) * 1024
    pb = synth.patches(64, 4)
    t = time.perf_counter()
    ow.loss_and_grad(pb.offsets, pb.img, pb.tgt)
    dt_w = time.perf_counter() - t
    return {**out,
            "ransac_2000x4096": {"hyp_pts_per_s": 2000 * 4096 / dt_r, "seconds": dt_r, "cores": 1,
                                 "sample": "oracle RANSAC (Philox + Floyd, float64 ACA, float64 "
                                           "transfer-error test) on the full single-pair workload"},
            "ransac_2000x4096_all_cores": {
                "hyp_pts_per_s": workers * 2000 * 4096 / dt_r_all, "seconds": dt_r_all,
                "cores": workers,
                "sample": f"the same single-pair oracle run in {workers} processes at once "
                          f"(aggregate rate)"},
            "ransac_batched_512x1024": {
                "hyp_pts_per_s": hp_b / dt_b, "seconds": dt_b, "cores": workers,
                "sample": f"oracle RANSAC on every 8th pair of the 512-pair batch (64 pairs, "
                          f"{hp_b:.3g} hyp-pts, 1024 hypotheses each) over {workers} processes"},
            "warp_l1_128x128": {"patches_per_s": 64 / dt_w, "seconds": dt_w,
                                "cores": torch.get_num_threads(),
                                "sample": "float64 autograd through the DLT solve, bilinear warp "
                                          "and L1, forward + backward, 64 patches of 128 x 128"}}


FP32_FLOP_PER_HYP_PT = 21   # the division-free test as 21 FLOP (FMA = 2): 3 rows x 2 FMA,
                            # 2 FMA residuals, mul + FMA norm, (tau w)^2; the kernel folds
                            # tau into the operands and issues 12 VALU instructions
FP32_PEAK_TFLOPS = 157.3     # the published FP32 vector peak, for packed (two-wide) FP32
                             # instructions, which these kernels do not issue
FP32_UNPACKED_TFLOPS = 78.6  # one FP32 FMA per lane and cycle: 256 CUs x 64 lanes x 2 x 2.4 GHz


def bench_ransac_single(stream):
    """N = 2000 correspondences, 30 % inliers, 4096 hypotheses, tau = 3 px:
    fused (scoring kernel + mask kernel) against plain (solve, score, argmax,
    mask). us_per_call: median over calls timed one by one (an event pair
    around each call); us_per_call_back_to_back: 200 calls queued between one
    event pair."""
    import numpy as np
    import torch

    import synth
    import paper_2402_18008_amd as hgpu
    from paper_2402_18008_amd import _abi
    cs = synth.config2()
    corr = torch.from_numpy(cs.corr).cuda()
    n, nh = corr.shape[1], 4096
    ws = torch.empty(hgpu.hg_ransac_ws_bytes(n, nh), dtype=torch.uint8, device="cuda")
    bh = torch.empty(9, device="cuda")
    bc = torch.empty(1, dtype=torch.int32, device="cuda")
    bi = torch.empty(1, dtype=torch.int32, device="cuda")
    mk = torch.empty(n, dtype=torch.uint8, device="cuda")
    hc = torch.empty(nh, dtype=torch.int32, device="cuda")
    res = {}
    for name in ("hg_ransac", "hg_ransac_plain"):
        fn = getattr(_abi.lib(), name)
        args = (corr.data_ptr(), n, n, nh, 3.0, 2, bh.data_ptr(), bc.data_ptr(), bi.data_ptr(),
                mk.data_ptr(), hc.data_ptr(), ws.data_ptr(), ws.numel(), stream.cuda_stream)
        t, p = time_launches(lambda: fn(*args), 200, 20, stream)
        us = float(np.median(p) * 1e3)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(200):
            fn(*args)
        b.record(stream)
        b.synchronize()
        us_b2b = a.elapsed_time(b) / 200 * 1e3
        res[name] = {"us_per_call": us, "us_per_call_back_to_back": us_b2b,
                     "hyp_pts_per_s": n * nh / (us * 1e-6)}
    return {"ransac_2000x4096": {"fused": res["hg_ransac"], "plain": res["hg_ransac_plain"],
                                 "fused_speedup": res["hg_ransac_plain"]["us_per_call"]
                                 / res["hg_ransac"]["us_per_call"]}}


def bench_ransac_batched(stream):
    """512 uneven pairs (N ~ U{100..8000}), 1024 hypotheses each: the
    persistent kernel (autotuned, replayed from a HIP graph) against a host
    loop of 512 single-pair fused calls."""
    import numpy as np
    import torch

    import synth
    import paper_2402_18008_amd as hgpu
    from paper_2402_18008_amd import _abi
    cb = synth.config3()
    corr = torch.from_numpy(cb.corr).cuda()
    off = torch.from_numpy(cb.off).cuda()
    nh = 1024
    hyp_pts = float(np.diff(cb.off).sum()) * nh
    br = hgpu.BatchedRansac(corr, off, nh, 3.0, 3)
    tune = br.autotune(cb.off)
    g = br.graph(tune)
    # graph replays and direct launches interleaved, so that both see the same clock state
    pg, pd = [], []
    for _ in range(3):
        g.launch()
        br.run(tune)
    for _ in range(20):
        pg += time_launches(g.launch, 1, 0, stream)[1]
        pd += time_launches(lambda: br.run(tune), 1, 0, stream)[1]
    ms_graph = float(np.median(pg))
    ms_direct = float(np.median(pd))
    g.close()
    # plain per-problem form: one fused single-pair call per pair, host loop
    total = corr.shape[1]
    L = _abi.lib()
    ws = torch.empty(hgpu.hg_ransac_ws_bytes(8000, nh), dtype=torch.uint8, device="cuda")
    bh = torch.empty(9, device="cuda")
    bc = torch.empty(1, dtype=torch.int32, device="cuda")
    bi = torch.empty(1, dtype=torch.int32, device="cuda")
    mk = torch.empty(total, dtype=torch.uint8, device="cuda")
    base = corr.data_ptr()
    calls = [(base + 4 * int(cb.off[q]), int(cb.off[q + 1] - cb.off[q]), total, nh, 3.0, 3,
              bh.data_ptr(), bc.data_ptr(), bi.data_ptr(), mk.data_ptr() + int(cb.off[q]), None,
              ws.data_ptr(), ws.numel(), stream.cuda_stream) for q in range(len(cb.off) - 1)]

    def loop():
        bad = 0
        for a in calls:
            bad |= L.hg_ransac(*a)
        if bad:
            raise RuntimeError("hg_ransac failed in the per-pair loop")
    t, p = time_launches(loop, 5, 1, stream)
    ms_plain = float(np.median(p))
    # adaptive termination (99 % confidence, cap 1024) on the same pairs
    ar = hgpu.AdaptiveRansac(corr, off, nh, 3.0, 3, confidence=0.99)
    # at most 4 workgroups per CU: more rounds in flight at once means more speculative
    # rounds past the stopping points (the library does the same when given no shape)
    t, p = time_launches(lambda: ar.run((tune[0], 64, min(tune[2], 4))), 20, 3, stream)
    ms_adaptive = float(np.median(p))
    n_eval = ar.n_evaluated.cpu().numpy()
    # HO-SVD refit of every pair on the inlier mask the persistent kernel produced
    br.run(tune)
    Hr = torch.empty((br.n_pairs, 9), dtype=torch.float32, device="cuda")
    ur = torch.empty(br.n_pairs, dtype=torch.int32, device="cuda")
    fr = torch.empty(br.n_pairs, dtype=torch.uint8, device="cuda")
    t, p = time_launches(lambda: hgpu.hg_refit_ho(corr, off, br.mask, Hr, ur, fr, off_host=cb.off),
                         20, 3, stream)
    ms_refit = float(np.median(p))
    rate = hyp_pts / (ms_graph * 1e-3)
    return {"ransac_batched_512x1024": {
        "hyp_pts": hyp_pts, "tuning": list(tune),
        "persistent_graph_ms": ms_graph, "persistent_direct_ms": ms_direct,
        "plain_host_loop_ms": ms_plain, "hyp_pts_per_s": rate,
        "speedup_vs_plain": ms_plain / ms_graph,
        "fp32_tflops": FP32_FLOP_PER_HYP_PT * rate / 1e12,
        "fp32_frac_of_peak": FP32_FLOP_PER_HYP_PT * rate / 1e12 / FP32_PEAK_TFLOPS,
        "fp32_frac_of_unpacked_peak": FP32_FLOP_PER_HYP_PT * rate / 1e12 / FP32_UNPACKED_TFLOPS,
        "adaptive_ms": ms_adaptive, "adaptive_mean_hyps_evaluated": float(n_eval.mean()),
        "adaptive_hyp_pts": float((np.diff(cb.off) * n_eval).sum()),
        "refit_ho_ms": ms_refit, "refit_points": int(total),
        "refit_points_per_s": total / (ms_refit * 1e-3)}}


def bench_diff(stream):
    """B = 1024 patches of 128 x 128: offsets -> H -> warp -> L1, forward and
    backward to the offsets; recompute form against the stored-intermediate
    form."""
    import numpy as np
    import torch

    import synth
    import paper_2402_18008_amd as hgpu
    pb = synth.config4()
    off = torch.from_numpy(pb.offsets).cuda()
    img = torch.from_numpy(pb.img).cuda()
    tgt = torch.from_numpy(pb.tgt).cuda()
    B, S = img.shape[0], img.shape[-1]
    # inputs rotated through 4 copies so that the 256 MB last-level cache does not hold them
    imgs = [img.clone() for _ in range(4)]
    tgts = [tgt.clone() for _ in range(4)]
    gl = torch.ones(B, device="cuda")
    state = {"k": 0}
    w = float(S - 1)

    def recompute():
        k = state["k"] = (state["k"] + 1) % 4
        H = hgpu.hg_aca_rect_fwd(off, 0.0, 0.0, w, 1.0)
        hgpu.hg_warp_l1_fwd(H, imgs[k], tgts[k])
        gH = hgpu.hg_warp_l1_bwd(H, imgs[k], tgts[k], gl)
        hgpu.hg_aca_rect_bwd(off, gH, 0.0, 0.0, w, 1.0)

    def stored():
        k = state["k"] = (state["k"] + 1) % 4
        H = hgpu.hg_aca_rect_fwd(off, 0.0, 0.0, w, 1.0)
        Wp = hgpu.hg_warp_store_fwd(H, imgs[k])
        hgpu.hg_l1_fwd(Wp, tgts[k])
        gW = hgpu.hg_l1_bwd(Wp, tgts[k], gl)
        gH = hgpu.hg_warp_bwd_from_grad(H, imgs[k], gW)
        hgpu.hg_aca_rect_bwd(off, gH, 0.0, 0.0, w, 1.0)

    def fused():
        k = state["k"] = (state["k"] + 1) % 4
        hgpu.hg_photometric_fwd(off, imgs[k], tgts[k])
        hgpu.hg_photometric_bwd(off, imgs[k], tgts[k], gl)

    def single():
        # loss and unit gradient in one pass, then the backward's scaling by grad_loss
        k = state["k"] = (state["k"] + 1) % 4
        _, g = hgpu.hg_photometric_fwd_grad(off, imgs[k], tgts[k])
        hgpu.hg_scale_grad(g, gl)

    ts = time_interleaved({"single": single, "fused": fused, "recompute": recompute,
                           "stored": stored}, 40, 4, stream)
    ms_1 = float(np.median(ts["single"]))
    ms_f = float(np.median(ts["fused"]))
    ms_r = float(np.median(ts["recompute"]))
    ms_s = float(np.median(ts["stored"]))
    min_bytes = 2 * B * S * S * 4          # img and tgt read once
    out = {"warp_l1_1024x128x128": {
        "single_pass_ms": ms_1, "fused_ms": ms_f, "recompute_ms": ms_r, "stored_ms": ms_s,
        "patches_per_s": B / (ms_1 * 1e-3),
        "effective_GBps": min_bytes / (ms_1 * 1e-3) / 1e9,
        "frac_hbm": min_bytes / (ms_1 * 1e-3) / 1e12 / 8.0,
        "speedup_vs_stored": ms_s / ms_1}}
    # general-quadrilateral ACA and its reverse mode over 2^20 problems (one thread each)
    src, dst, _ = synth.quadruples(1 << 20, 9)
    S4 = torch.from_numpy(np.ascontiguousarray(src.T)).cuda()
    D4 = torch.from_numpy(np.ascontiguousarray(dst.T)).cuda()
    gH4 = torch.ones((1 << 20, 9), dtype=torch.float64, device="cuda")
    t, p = time_launches(lambda: hgpu.hg_aca_fwd(S4, D4), 20, 3, stream)
    ms_af = float(np.median(p))
    t, p = time_launches(lambda: hgpu.hg_aca_bwd(S4, D4, gH4), 20, 3, stream)
    ms_ab = float(np.median(p))
    nq = 1 << 20
    out["aca_general_2p20"] = {"fwd_ms": ms_af, "bwd_ms": ms_ab,
                               "fwd_GBps": nq * (64 + 72) / (ms_af * 1e-3) / 1e9,
                               "bwd_GBps": nq * (64 + 72 + 64) / (ms_ab * 1e-3) / 1e9}
    # six-solve iterative refinement (solve, warp + L1 backward, reverse mode, step,
    # then the final loss): eager launches against one graph replay
    o = off.clone()
    R = hgpu.Refine(img, tgt, o, iters=6, step=20.0)
    t, p = time_launches(R.run, 20, 3, stream)
    ms_e = float(np.median(p))
    G = R.graph()
    t, p = time_launches(G.launch, 20, 3, stream)
    ms_g = float(np.median(p))
    G.close()
    out["refine_6iter_1024x128x128"] = {"eager_ms": ms_e, "graph_ms": ms_g,
                                        "kernels_per_pass": 4 * 6 + 3,
                                        "patches_per_s": B / (ms_g * 1e-3)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 26, help="quadruples (default 2^26)")
    ap.add_argument("--part", default="all",
                    choices=["all", "solver", "sk", "affine", "ransac", "batched", "diff"],
                    help="run only one stage (for profiler runs); the JSON line then carries "
                         "only that stage")
    ap.add_argument("--solver-only", action="store_true", help="same as --part solver")
    ap.add_argument("--with-copy", action="store_true",
                    help="with --part solver: also run a plain 4 GiB device copy (reference "
                         "for hardware byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU run: write the solver's measured HBM traffic per launch from "
                         "two rocprofv3 --pmc output folders (FETCH_SIZE, then WRITE_SIZE) of "
                         "'--part solver --with-copy' runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="host processes for input generation (fewer under a profiler)")
    args = ap.parse_args()
    if args.solver_only:
        args.part = "solver"
    if args.traffic_from:
        write_traffic(*args.traffic_from, args.n)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): every kernel "
              f"of the hot path runs on a single GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    stream = torch.cuda.current_stream()
    if args.part in ("ransac", "batched", "diff"):
        fn = {"ransac": bench_ransac_single, "batched": bench_ransac_batched,
              "diff": bench_diff}[args.part]
        print(json.dumps({"part": args.part, **fn(stream)}), flush=True)
        return

    import synth
    import paper_2402_18008_amd as hgpu

    workers = max(1, min(args.gen_workers, os.cpu_count() or 1))
    n = args.n
    if args.part == "sk":
        print(json.dumps({"part": "sk", **bench_sk(stream, n, workers, args.steps,
                                                   args.warmup)}), flush=True)
        return
    log(f"generating {n} quadruples with {workers} processes")
    t0 = time.perf_counter()
    src, dst, lab = synth.quadruples_parallel(n, 1, degenerate_every=100, workers=workers)
    log(f"generated in {time.perf_counter() - t0:.1f} s; copying to the GPU")
    dev = torch.device("cuda", 0)
    S = torch.from_numpy(src).to(dev)
    D = torch.from_numpy(dst).to(dev)
    H = torch.empty((9, n), dtype=torch.float32, device=dev)
    F = torch.empty(n, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    if args.part == "affine":
        print(json.dumps({"part": "affine", **bench_affine(stream, S, D, args.steps,
                                                           args.warmup)}), flush=True)
        return

    def step():
        hgpu.hg_solve4(S, D, hgpu.HG_ACA, H=H, flags=F)

    log(f"timing {args.steps} steps after {args.warmup} warmup")
    total_ms, per = time_launches(step, args.steps, args.warmup, stream)
    ms_step = total_ms / args.steps
    kern_ms = float(np.mean(per))
    value = n / (ms_step * 1e-3)
    achieved = BYTES_PER_QUAD * n / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(n)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "homographies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched ACA 4-point solve of {n} random quadruples "
                               f"(1% near-degenerate), fp32 SoA planes in HBM, 9 fp32 planes "
                               f"+ flag byte out", "n": n, "method": "ACA"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "solve4_kernel<ACA>", "kernel_ms": kern_ms,
                     "bytes_per_unit": BYTES_PER_QUAD},
    }
    extra = {}
    if args.part == "solver" and args.with_copy:
        # copies of the 4 GiB source planes (S.numel() * 4 bytes each way): one with
        # the solver's access pattern, one by torch; references for byte counters
        C = torch.empty_like(S)
        for _ in range(2):
            hgpu.hg_stream_copy(S, C)
            torch.neg(S, out=C)
        torch.cuda.synchronize()
        extra["copy_bytes_each_way"] = S.numel() * 4
        del C
    if args.part == "all":
        # SKS on the same batch
        def sks():
            hgpu.hg_solve4(S, D, hgpu.HG_SKS, H=H, flags=F)
        t, p = time_launches(sks, 20, 3, stream)
        extra["sks_2p26"] = {"homographies_per_s": n / (t / 20 * 1e-3),
                             "GBps": BYTES_PER_QUAD * n / (np.mean(p) * 1e-3) / 1e9}
        extra["stream_ceilings"] = stream_ceilings(stream, S, D, H, F, achieved)
        # batch-size sweep (the sizes of the paper's GPU table, then larger): time per launch
        # of a prefix of the same planes (plane stride stays 2^26)
        sweep = {}
        for m in (1, 10, 100, 1000, 10000, 100000, 1000000, 10000000, n):
            sm_, dm_, hm_, fm_ = S[:, :m], D[:, :m], H[:, :m], F[:m]
            reps = 200 if m <= 100000 else 30
            t, p = time_launches(lambda: hgpu.hg_solve4(sm_, dm_, hgpu.HG_ACA, H=hm_, flags=fm_),
                                 reps, 10, stream)
            us = float(np.median(p)) * 1e3
            sweep[str(m)] = {"us_per_launch": us, "homographies_per_s": m / (us * 1e-6)}
            if m <= 1000000:
                # averaged over back-to-back launches, as the paper's table is: eager, and
                # replayed from a graph (checked against the eager result)
                ref = hm_.clone()
                hm_.zero_()
                gus = graph_us(lambda: hgpu.hg_solve4(sm_, dm_, hgpu.HG_ACA, H=hm_, flags=fm_),
                               stream)
                assert torch.equal(hm_, ref), f"graph-replayed solve differs at n = {m}"
                bus = burst_us(lambda: hgpu.hg_solve4(sm_, dm_, hgpu.HG_ACA, H=hm_, flags=fm_),
                               stream)
                sweep[str(m)].update(us_per_launch_burst=bus, us_per_launch_graph=gus)
        extra["aca_batch_size_sweep"] = sweep
        # small batch latency: 4096 quadruples
        for meth, name in ((hgpu.HG_ACA, "aca"), (hgpu.HG_SKS, "sks")):
            s4, d4 = S[:, :4096], D[:, :4096]
            h4, f4 = H[:, :4096], F[:4096]
            t, p = time_launches(lambda: hgpu.hg_solve4(s4, d4, meth, H=h4, flags=f4), 200, 20,
                                 stream)
            extra[f"{name}_4096_us_per_launch"] = float(np.median(p) * 1e3)
        extra.update(bench_affine(stream, S, D))
        extra.update(bench_sk(stream, n, workers))
        extra.update(bench_ransac_single(stream))
        extra.update(bench_ransac_batched(stream))
        extra.update(bench_diff(stream))
    out["extra"] = extra
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(src, dst, n, workers)
        if args.part == "all":
            extra["cpu_oracle"] = cpu_oracle_extras()
    if args.part == "all":
        extra["oracle_fp64_error"] = oracle_fp64_error()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
