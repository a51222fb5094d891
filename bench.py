#!/usr/bin/env python3
"""Benchmark of the whole hot path on one MI355X.

One step = one gs_score_all call on data already resident in HBM: R0 by TSQR (FP64),
the segment anchors (FP64), the FP32 Givens walk and the write of the complete score
table (m * 2^(m-1) BIC values).  Workload: m = 26 variables, n = 5000 samples from a
seeded linear-Gaussian DAG (edge probability 0.15, weights +-U[0.3, 1.0]);
872,415,232 families, a 3.49 GB FP32 table.

Prints one JSON line.  Besides the contract fields it carries
  roofline      the walk kernel against the HBM write roofline (4 algorithmic
                bytes per family), timed with HIP events on the launch stream;
  valu          the walk's algorithmic FP32 flops against the FP32 vector peak without
                packed instructions (78.6 TFLOP/s: the library is built with packed FP32
                switched off);
  fp64_walk     the same step with the walk in FP64 (families/s);
  fp32_vs_fp64  max relative RSS difference of the two walks over the whole table;
  concurrent    the same step for a list of independent datasets of the same shape
                through gs_score_all_many, three in flight at once (a serving loop's
                throughput; the first table is checked bit-identical to a single call);
  batched       256 bootstrap datasets (m 12..18, n 200..2000) in one graph replay of
                gs_score_batched, with the autotuned cap on k, against 256 sequential
                gs_score_all calls with the same plans;
  adjoint       forward + hand-written backward at m = 14, n = 500 (the loss
                sum_c logsumexp_S(-BIC)); the backward takes R0 and the anchors from
                the forward, as in a training step (bwd_full_ms: forming them again);
  adjoint_headline  the same on the benchmark's workload (FP32 backward with and
                without the forward's R0 and anchors, FP64 backward);
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload, with the
                largest difference between those oracle values and the GPU table
                (measured after the timed region);
  host          CPU model, host threads, git revision (when the tree has one) and a
                hash of the library sources.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 78.6  # non-packed FP32 (packed FP32 is switched off in the build)
WORKLOADS = {"c3_m26_n5000": "c3_m26_n5000", "c2_m20_n1000": "c2_m20_n1000",
             "c1_m8_n200": "c1_m8_n200"}


def runtime_T(m: int) -> int:
    """Flops of the paper's serial walk (Sec. 5 closed form, middle term 6 * 2^m)."""
    return 3 * m * (1 << m) + 6 * (1 << m) - 3 * m * m - 9 * m - 6


def walk_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("walk.hip", "walk_program.hpp"):
        with open(os.path.join(ROOT, "paper_1901_07643_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per walk launch from the committed PMC summary, if it was taken on
    the current walk kernel source."""
    path = os.path.join(ROOT, "profiles", f"walk_f32_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("walk_source_hash") != walk_source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(X, m, sample: int, table, seed: int = 1):
    """Times the oracle on `sample` random families, then compares those values with
    the GPU's BIC table (a device tensor) on the same indices."""
    import numpy as np
    import torch

    import oracle
    threads = oracle.default_threads()
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    idx = rng.choice(m * (1 << (m - 1)), size=sample, replace=False).astype(np.int64)
    t0 = time.perf_counter()
    ref = oracle.score_indices(X, idx, oracle.OUT_BIC, threads=threads)
    dt = time.perf_counter() - t0
    got = table[torch.as_tensor(idx, device=table.device)].double().cpu().numpy()
    dbic = float(np.abs(got - ref).max())
    return {"value": sample / dt, "unit": "families/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} uniformly drawn families of the same table (BIC, FP64 "
                      f"Householder per family), {dt:.2f} s",
            "gpu_vs_oracle": {"families": sample, "max_abs_bic_err": dbic,
                              "implied_max_rel_rss_err": math.expm1(dbic / n)}}


def host_info() -> dict:
    import subprocess
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rev = None
    try:
        r = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True,
                           text=True, timeout=10)
        rev = r.stdout.strip() or None if r.returncode == 0 else None
    except (OSError, subprocess.SubprocessError):
        pass
    h = hashlib.sha256()
    for sub in ("paper_1901_07643_amd/csrc", "include"):
        d = os.path.join(ROOT, sub)
        for f in sorted(os.listdir(d)):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "host_threads": threads, "git_rev": rev,
            "source_sha16": h.hexdigest()[:16]}


def _event_ms(fn, steps: int, stream) -> float:
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(steps: int, stream):
    """256 bootstrap resamples: one graph replay per step vs 256 gs_score_all calls."""
    import torch

    import paper_1901_07643_amd as gs
    from datagen import bootstrap_batch
    from paper_1901_07643_amd import tune
    Xh = bootstrap_batch()
    shapes = [(X.shape[1], X.shape[0]) for X in Xh]
    Xs = [torch.as_tensor(X, device="cuda") for X in Xh]
    outs = [torch.empty(gs.num_families(m), dtype=torch.float32, device="cuda") for m, _ in shapes]
    cap, cap_ms = tune.tune_batch(shapes, reps=3)
    ks = tune.batch_k(shapes, cap)
    b = gs.Batch(shapes, k=ks)
    b.score(Xs, outs=outs, use_graph=True)  # capture + status check
    ms_graph = _event_ms(lambda: b.score(Xs, outs=outs, use_graph=True, check_status=False),
                         steps, stream)
    ms_eager = _event_ms(lambda: b.score(Xs, outs=outs, use_graph=False, check_status=False),
                         steps, stream)
    st = b.status()
    info = b.info
    b.close()
    plans = [gs.Plan(m, k, 5) for (m, _), k in zip(shapes, ks)]
    seq_steps = max(2, steps // 4)

    def sequential():
        for X, o, p in zip(Xs, outs, plans):
            gs.score_all(X, plan=p, out=o, check_status=False)
    sequential()
    ms_seq = _event_ms(sequential, seq_steps, stream)
    for p in plans:
        if p.status() != gs.GS_OK:
            raise SystemExit("batched workload: bad device status")
    # the plain FP64 walk, dataset after dataset
    outs64 = [torch.empty(gs.num_families(m), dtype=torch.float64, device="cuda") for m, _ in shapes]

    def sequential64():
        for X, o, p in zip(Xs, outs64, plans):
            gs.score_all(X, plan=p, out=o, precision="fp64", check_status=False)
    sequential64()
    ms_seq64 = _event_ms(sequential64, 2, stream)
    del outs64
    fam = info["total_families"]
    if any(x != gs.GS_OK for x in st):
        raise SystemExit(f"batched workload: device status {st}")
    return {"workload": "256 bootstrap resamples, m 12..18, n 200..2000", "families": fam,
            "value": fam / (ms_graph * 1e-3), "unit": "families/s", "ms_per_step": ms_graph,
            "eager_ms": ms_eager, "sequential_ms": ms_seq,
            "sequential_value": fam / (ms_seq * 1e-3), "speedup_vs_sequential": ms_seq / ms_graph,
            "fp64_sequential_value": fam / (ms_seq64 * 1e-3), "fp64_sequential_ms": ms_seq64,
            "roofline": {"bound": "hbm", "achieved": 4.0 * fam / (ms_graph * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": 4.0 * fam / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "note": "4 B per family written, whole graph replay"},
            "tuned_k_cap": cap, "cap_ms": {str(k): v for k, v in cap_ms.items()},
            "waves": info["total_waves"], "segments": info["total_segments"],
            "walk_waves_per_simd": 4}


def bench_concurrent(m: int, n: int, cfg, steps: int, in_flight: int, ref_out, X0, stream):
    """steps datasets of the workload's shape through gs_score_all_many with in_flight
    of them in progress at once (in_flight distinct datasets, cycled; each slot keeps
    its own table); the families/s of the whole job."""
    import torch

    import paper_1901_07643_amd as gs
    from datagen import linear_gaussian
    dev = X0.device
    nfam = gs.num_families(m)
    Xs = [X0] + [torch.as_tensor(linear_gaussian(m, n, cfg.p_edge, cfg.lo, cfg.hi,
                                                 seed=cfg.seed + 1000 + i), device=dev)
                 for i in range(1, in_flight)]
    outs = [torch.empty(nfam, dtype=torch.float32, device=dev) for _ in range(in_flight)]
    plan = gs.Plan(m)
    Xl = [Xs[i % in_flight] for i in range(steps)]
    Ol = [outs[i % in_flight] for i in range(steps)]
    gs.score_all_many(Xl[:2 * in_flight], plan=plan, outs=Ol[:2 * in_flight], in_flight=in_flight)
    ms = _event_ms(lambda: gs.score_all_many(Xl, plan=plan, outs=Ol, in_flight=in_flight,
                                             check_status=False), 1, stream) / steps
    if any(st != gs.GS_OK for st in plan.many_status()):
        raise SystemExit(f"concurrent workload: device status {plan.many_status()}")
    identical = bool(torch.equal(outs[0], ref_out))
    plan.close()
    del outs
    torch.cuda.synchronize()
    return {"datasets_in_flight": in_flight, "datasets": steps, "ms_per_dataset": ms,
            "value": nfam / (ms * 1e-3), "unit": "families/s",
            "entry_point": "gs_score_all_many",
            "table_identical_to_single_call": identical}


def bench_reduce(X, plan, steps: int, stream):
    """The fused consumer gs_score_reduce on the same workload: per child the minimum BIC
    and its parent set and ln sum exp(-BIC) (and the 8 best parent sets), with no table
    written.  One step = R0, anchors, the reducing walk and the per-child merge."""
    import paper_1901_07643_amd as gs
    nfam = gs.num_families(plan.m)
    res = {}
    for top in (0, 8):
        gs.score_reduce(X, plan=plan, top_k=top)
        plan.set_timing(True)
        ms = _event_ms(lambda: gs.score_reduce(X, plan=plan, top_k=top, check_status=False),
                       steps, stream)
        stage, _ = plan.timing()
        plan.set_timing(False)
        res[f"top{top}"] = {"value": nfam / (ms * 1e-3), "unit": "families/s",
                            "ms_per_step": ms, "walk_and_merge_ms": stage[2],
                            "r0_qr_ms": stage[0], "anchors_ms": stage[1]}
    res["note"] = ("no table written; the walk then does the Givens steps, the BIC scores "
                   "and the per-lane folds only")
    return res


def bench_adjoint(steps: int, stream):
    """Forward and backward of the loss sum_c logsumexp_S(-BIC) at m = 14, n = 500 (its
    parity against the oracle's closed-form gradient is a GPU test)."""
    import torch

    import paper_1901_07643_amd as gs
    from datagen import CONFIGS, config_data
    cfg = CONFIGS["c5_m14_n500"]
    Xh = config_data("c5_m14_n500")
    X = torch.as_tensor(Xh, device="cuda")
    m, n = cfg.m, cfg.n
    plan = gs.Plan(m)
    nfam = gs.num_families(m)
    dX = torch.empty((n, m), dtype=torch.float64, device="cuda")
    bic = gs.score_all(X, plan=plan)
    dbic = (-torch.softmax(-bic.view(m, -1).double(), dim=1)).float().reshape(-1).contiguous()
    gs.score_backward(X, dbic, plan=plan, out=dX)
    ms_fwd = _event_ms(lambda: gs.score_all(X, plan=plan, out=bic, check_status=False), steps,
                       stream)
    # a training step runs the forward, then the backward on the same X: the backward takes
    # R0 and the anchors the forward left in the plan (gs_plan_set_reuse)
    ms_bwd = _event_ms(lambda: gs.score_backward(X, dbic, plan=plan, out=dX, check_status=False,
                                                 reuse_front=True), steps, stream)
    ms_bwd_full = _event_ms(lambda: gs.score_backward(X, dbic, plan=plan, out=dX,
                                                      check_status=False, reuse_front=False),
                            steps, stream)
    out64 = torch.empty(nfam, dtype=torch.float64, device="cuda")
    gs.score_all(X, plan=plan, out=out64, precision="fp64")
    ms_fwd64 = _event_ms(lambda: gs.score_all(X, plan=plan, out=out64, precision="fp64",
                                              check_status=False), steps, stream)
    bwd_bytes = 4.0 * nfam + 8.0 * 2 * n * m  # dscores read once; X read, dX written
    res = {"workload": "c5_m14_n500", "families": nfam, "fwd_ms": ms_fwd, "bwd_ms": ms_bwd,
           "bwd_full_ms": ms_bwd_full,
           "value": nfam / ((ms_fwd + ms_bwd) * 1e-3), "unit": "families/s (fwd+bwd)",
           "bwd_over_fwd": ms_bwd / ms_fwd,
           "fp64_walk_value": nfam / (ms_fwd64 * 1e-3), "fp64_walk_ms": ms_fwd64,
           "roofline": {"bound": "latency", "achieved": bwd_bytes / (ms_bwd * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": bwd_bytes / (ms_bwd * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "note": "backward: algorithmic bytes (dscores, X, dX) per call; at "
                                "114,688 families the call is launch and latency bound"}}
    return res


def bench_adjoint_headline(X, workload: str, steps: int, stream):
    """Forward and backward on the benchmark's workload (at m = 26, n = 5000 the plan has
    k = 13 and the reverse walk starts from anchors formed in the walk's final ordering).
    FP32 backward with and without the forward's R0 and anchors, and the FP64 backward."""
    import torch

    import paper_1901_07643_amd as gs
    n, m = X.shape
    plan = gs.Plan(m)
    nfam = gs.num_families(m)
    dX = torch.empty((n, m), dtype=torch.float64, device="cuda")
    bic = gs.score_all(X, plan=plan)
    dbic = (-torch.softmax(-bic.view(m, -1).double(), dim=1)).float().reshape(-1).contiguous()
    gs.score_backward(X, dbic, plan=plan, out=dX)
    ms_fwd = _event_ms(lambda: gs.score_all(X, plan=plan, out=bic, check_status=False), steps,
                       stream)
    ms_bwd = _event_ms(lambda: gs.score_backward(X, dbic, plan=plan, out=dX, check_status=False,
                                                 reuse_front=True), steps, stream)
    ms_bwd_full = _event_ms(lambda: gs.score_backward(X, dbic, plan=plan, out=dX,
                                                      check_status=False, reuse_front=False),
                            steps, stream)
    del bic, dbic
    out64 = gs.score_all(X, plan=plan, precision="fp64")
    d64 = (-torch.softmax(-out64.view(m, -1), dim=1)).reshape(-1).contiguous()
    del out64
    gs.score_backward(X, d64, plan=plan, precision="fp64", out=dX)
    ms_bwd64 = _event_ms(lambda: gs.score_backward(X, d64, plan=plan, precision="fp64", out=dX,
                                                   check_status=False, reuse_front=False),
                         steps, stream)
    del d64
    plan.close()
    torch.cuda.empty_cache()
    return {"workload": workload, "families": nfam, "fwd_ms": ms_fwd, "bwd_ms": ms_bwd,
            "bwd_full_ms": ms_bwd_full, "bwd_fp64_ms": ms_bwd64,
            "value": nfam / ((ms_fwd + ms_bwd) * 1e-3), "unit": "families/s (fwd+bwd)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_m26_n5000", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=131072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-walk comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-reduce", action="store_true", help="skip the fused reduction")
    ap.add_argument("--concurrent", type=int, default=3,
                    help="datasets in flight for the concurrent measurement (0: skip)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the scoring path runs on one GPU (got --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1901_07643_amd as gs
    from datagen import CONFIGS, config_data

    cfg = CONFIGS[args.workload]
    m, n = cfg.m, cfg.n
    X_host = config_data(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X = torch.as_tensor(X_host, device=dev)
    plan = gs.Plan(m)
    info = plan.info
    nfam = gs.num_families(m)
    out = torch.empty(nfam, dtype=torch.float32, device=dev)
    print(f"# workload {args.workload}: m={m} n={n} families={nfam} plan={info}", file=sys.stderr,
          flush=True)

    if args.calib_copy_mb:
        nb = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        gs.score_all(X, plan=plan, what="bic", precision="fp32", out=out, check_status=False)
    torch.cuda.synchronize()
    st = plan.status()
    if st != gs.GS_OK:
        raise SystemExit(f"device status {st}: {gs.last_error()}")

    plan.set_timing(True)
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        gs.score_all(X, plan=plan, what="bic", precision="fp32", out=out, check_status=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    stage_ms, cnt = plan.timing()
    plan.set_timing(False)
    print(f"# timed {args.steps} steps: {ms_step:.4f} ms/step (wall {wall:.3f} s); stages "
          f"qr {stage_ms[0]:.4f} anchors {stage_ms[1]:.4f} walk {stage_ms[2]:.4f} ms",
          file=sys.stderr, flush=True)

    value = nfam / (ms_step * 1e-3)
    walk_s = stage_ms[2] * 1e-3
    alg_bytes = 4.0 * nfam                       # one FP32 table write per family
    achieved_gbs = alg_bytes / walk_s / 1e9
    traffic = load_traffic(args.workload)
    alg_flops = runtime_T(m) + 4.0 * nfam        # Givens steps + RSS and BIC per family
    valu_tflops = alg_flops / walk_s / 1e12

    res = {
        "metric": "families scored/s (BIC) at m=26,n=5000; % FP32 VALU peak; FP32 vs FP64 walk"
        if args.workload == "c3_m26_n5000"
        else f"families scored/s (BIC) at m={m},n={n}",
        "value": value,
        "unit": "families/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "families": nfam,
                   "edge_prob": cfg.p_edge, "weights": [cfg.lo, cfg.hi], "seed": cfg.seed,
                   "walk": "fp32", "anchors": "fp64", "output": "bic",
                   "plan": {"k": info["k"], "ks": info["ks"], "segments": info["num_segments"]}},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": "walk_kernel<float,5,true,4>",
                     "kernel_ms": stage_ms[2]},
        "valu": {"achieved": valu_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": valu_tflops / FP32_VECTOR_PEAK_TFLOPS,
                 "note": "algorithmic flops (Sec. 5 T(m) + 4 per family) over the walk time, "
                         "against the non-packed FP32 vector peak"},
        "stages_ms": {"r0_qr": stage_ms[0], "anchors": stage_ms[1], "walk": stage_ms[2],
                      "call": stage_ms[3]},
    }

    if args.concurrent > 1:
        res["concurrent"] = bench_concurrent(m, n, cfg, args.steps, args.concurrent, out, X,
                                             stream)
        print(f"# {args.concurrent} datasets in flight: "
              f"{res['concurrent']['ms_per_dataset']:.4f} ms per dataset", file=sys.stderr,
              flush=True)

    if not args.no_fp64:
        out64 = torch.empty(nfam, dtype=torch.float64, device=dev)
        gs.score_all(X, plan=plan, what="bic", precision="fp64", out=out64, check_status=False)
        torch.cuda.synchronize()
        k64 = max(2, args.steps // 4)
        plan.set_timing(True)
        e0.record(stream)
        for _ in range(k64):
            gs.score_all(X, plan=plan, what="bic", precision="fp64", out=out64, check_status=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / k64
        st64, cnt64 = plan.timing()
        plan.set_timing(False)
        walk64_ms = st64[2] if cnt64 else None
        res["fp64_walk"] = {"value": nfam / (ms64 * 1e-3), "unit": "families/s",
                            "ms_per_step": ms64, "steps": k64}
        if walk64_ms:
            gbs = 8.0 * nfam / (walk64_ms * 1e-3) / 1e9
            res["fp64_walk"]["roofline"] = {
                "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "kernel": "walk_kernel<double,5,true,1>",
                "kernel_ms": walk64_ms, "note": "8 B per family (the FP64 table write)"}
        gs.score_all(X, plan=plan, what="rss", precision="fp64", out=out64, check_status=False)
        gs.score_all(X, plan=plan, what="rss", precision="fp32", out=out, check_status=False)
        worst = 0.0
        for lo in range(0, nfam, 1 << 27):
            hi = min(nfam, lo + (1 << 27))
            rel = ((out[lo:hi].double() - out64[lo:hi]).abs() / out64[lo:hi]).max().item()
            worst = max(worst, rel)
        res["fp32_vs_fp64"] = {"max_rel_rss_err": worst, "over": "whole table"}
        del out64
        torch.cuda.synchronize()
        print(f"# fp64 walk {ms64:.4f} ms/step; max rel RSS fp32 vs fp64 {worst:.3e}",
              file=sys.stderr, flush=True)

    if not args.no_reduce:
        res["fused_reduce"] = bench_reduce(X, plan, args.steps, stream)
        print(f"# fused reduce: {res['fused_reduce']['top0']['ms_per_step']:.4f} ms/step "
              f"(top-8 {res['fused_reduce']['top8']['ms_per_step']:.4f})", file=sys.stderr,
              flush=True)
    if not args.no_batched:
        res["batched"] = bench_batched(args.steps, stream)
        print(f"# batched: {res['batched']['ms_per_step']:.3f} ms/step graph, "
              f"{res['batched']['sequential_ms']:.3f} ms sequential, cap k={res['batched']['tuned_k_cap']}",
              file=sys.stderr, flush=True)
    if not args.no_adjoint:
        res["adjoint"] = bench_adjoint(args.steps, stream)
        print(f"# adjoint: fwd {res['adjoint']['fwd_ms']:.4f} ms, bwd {res['adjoint']['bwd_ms']:.4f} ms"
              f" (forming R0 and the anchors again: {res['adjoint']['bwd_full_ms']:.4f} ms)",
              file=sys.stderr, flush=True)
        res["adjoint_headline"] = bench_adjoint_headline(X, args.workload, args.steps, stream)
        a3 = res["adjoint_headline"]
        print(f"# adjoint on {args.workload}: fwd {a3['fwd_ms']:.4f} ms, bwd {a3['bwd_ms']:.4f} ms "
              f"(full {a3['bwd_full_ms']:.4f} ms, FP64 {a3['bwd_fp64_ms']:.4f} ms)",
              file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        print(f"# cpu baseline: oracle on {args.cpu_sample} families ...", file=sys.stderr,
              flush=True)
        gs.score_all(X, plan=plan, what="bic", precision="fp32", out=out)
        torch.cuda.synchronize()
        res["cpu_baseline"] = cpu_baseline(X_host, m, args.cpu_sample, out)
    else:
        res["cpu_baseline"] = None
    res["host"] = host_info()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
