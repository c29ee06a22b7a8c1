"""Benchmark of the IVHD loop on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config C3] [--mode det|atomic|both]

One step is one full pass of the loop over the synthetic workload: T
iterations of (random-neighbour draws every R iterations, edge forces,
per-vertex reduction, momentum update) on a kNN graph already built and
resident in HBM.  The headline value is edge-updates/s = M (nn + rn) T K / t
over K timed steps, t from HIP events on the stream the library launches on.

The JSON line also carries
  roofline      the deterministic step kernel's algorithmic bytes per launch
                (32 M + 8 M (nn + rn)) over its average launch time, measured
                with HIP events around back-to-back launches, against 8 TB/s;
                `traffic` = HBM bytes per launch from rocprofv3 counters when
                profiles/ holds figures taken on the current kernel source
  cpu_baseline  the FP64 oracle (plain C, one thread) timed on a bounded
                sample of the same workload shape (rank 0, N = 1 only)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
STEP_SOURCE = os.path.join(ROOT, "paper_2303_05455_amd", "csrc", "step.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_det_C3_traffic.md")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest(path=STEP_SOURCE) -> str:
    return hashlib.sha1(open(path, "rb").read()).hexdigest()[:12]


def stored_traffic():
    """HBM bytes per launch of the det step kernel from the committed
    rocprofv3 counter summary, if it was taken on the current source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m = re.search(r"source_sha1:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != source_digest():
        return None
    return float(t.group(1))


def alg_bytes(M, nn, rn):
    """Algorithmic bytes of one iteration: read y, read+write v, write y
    (32 B per vertex) plus, per edge, its index and its reaction delivered to
    the other end (8 B per edge)."""
    return 32 * M + 8 * M * (nn + rn)


def cpu_baseline(cfg, iters, seed=0):
    import oracle
    import synth
    rng = np.random.default_rng([seed, cfg.cfg_id, 99])
    sizes = synth.cluster_sizes(cfg.M, cfg.K, cfg.sizes, cfg.zipf_s)
    labels = np.repeat(np.arange(cfg.K, dtype=np.int32), sizes)[rng.permutation(cfg.M)]
    nn_idx = synth.random_neighbour_graph(cfg.M, cfg.nn, rng, labels=labels, hub_alpha=1.2)
    Y0 = synth.init_positions(cfg.M, rng)
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.run(Y0, np.zeros_like(Y0, dtype=np.float64), nn_idx, rn=cfg.rn, a=cfg.a, b=cfg.b,
               c=cfg.c, seed=cfg.seed, R=cfg.R, T=iters)
    dt = time.perf_counter() - t0
    return {
        "value": cfg.M * (cfg.nn + cfg.rn) * iters / dt,
        "unit": "edge-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"plain-C FP64 oracle loop, one thread, {iters} of the {cfg.T} iterations at "
                   f"M={cfg.M:,}, nn={cfg.nn}, rn={cfg.rn}, R={cfg.R} on a same-shape synthetic "
                   f"graph ({dt:.1f} s)"),
    }


def calibrate_copy(mib: int):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 4, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--mode", default="both", choices=["det", "atomic", "both"])
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import synth
    from paper_2303_05455_amd import Context, ivhd_knn_build

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = synth.CONFIGS[args.config]
    M, nn, rn, R, T = cfg.M, cfg.nn, cfg.rn, cfg.R, cfg.T

    t0 = time.perf_counter()
    X, labels, Y0 = synth.make_inputs(cfg)
    log(f"inputs {cfg.name}: M={M} N={cfg.N} ({time.perf_counter() - t0:.1f} s)")
    dX = torch.from_numpy(X).to(dev)
    del X
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nn_idx = ivhd_knn_build(dX, nn)
    torch.cuda.synchronize()
    knn_s = time.perf_counter() - t0
    del dX
    indeg = torch.bincount(nn_idx.view(-1).long(), minlength=M)
    max_deg = int(indeg.max().item()) + nn + 2 * rn + 8
    log(f"kNN graph (exact, nn={nn}) built in {knn_s:.2f} s; max nn in-degree {int(indeg.max())}")

    d_y0 = torch.from_numpy(Y0).to(dev)
    res = {}
    modes = ["det", "atomic"] if args.mode == "both" else [args.mode]
    for mode in modes:
        y = d_y0.clone()
        v = torch.zeros_like(y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = Context(nn_idx, y, v, rn=rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed,
                      rn_resample_every=R, mode=mode)
        init_ms = (time.perf_counter() - t0) * 1e3
        ctx.set_graphs(not args.no_graphs)
        for _ in range(args.warmup):
            ctx.step(T)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.step(T)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        E = ctx.stress()
        ctx.close()
        iters = T * args.steps
        res[mode] = {
            "value": M * (nn + rn) * iters / t,
            "ms_per_step": t * 1e3 / args.steps,
            "us_per_iter": t * 1e6 / iters,
            "gbps_alg": alg_bytes(M, nn, rn) * iters / t / 1e9,
            "init_ms": init_ms,
            "final_stress": E,
        }
        log(f"{mode}: {res[mode]['value']:.4g} edge-updates/s, {res[mode]['us_per_iter']:.2f} us/iter, "
            f"{res[mode]['gbps_alg']:.0f} GB/s algorithmic, E={E:.6g}")

    # per-launch time of the deterministic step kernel: back-to-back launches
    # (no draws), HIP events on the library's stream
    roofline = None
    if "det" in res:
        y = d_y0.clone()
        v = torch.zeros_like(y)
        ctx = Context(nn_idx, y, v, rn=rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed,
                      rn_resample_every=0, mode="det")
        launches = 64 * 20
        ctx.step(128)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.step(launches)
        e1.record()
        torch.cuda.synchronize()
        per_launch = e0.elapsed_time(e1) / 1e3 / launches
        ctx.close()
        achieved = alg_bytes(M, nn, rn) / per_launch / 1e9
        traffic = stored_traffic()
        roofline = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
            "kernel": "step_det_kernel", "alg_bytes_per_launch": alg_bytes(M, nn, rn),
            "us_per_launch": per_launch * 1e6,
        }
        log(f"det step kernel: {per_launch * 1e6:.2f} us/launch, {achieved:.0f} GB/s algorithmic "
            f"({achieved / HBM_PEAK_GBPS:.1%} of 8 TB/s)")

    cpu = None
    if not args.no_cpu:
        log(f"timing the FP64 oracle on {args.cpu_iters} iterations ...")
        cpu = cpu_baseline(cfg, args.cpu_iters)
        log(f"oracle: {cpu['value']:.4g} edge-updates/s")

    main_mode = "det" if "det" in res else modes[0]
    r = res[main_mode]
    out = {
        "metric": "edge-updates/sec (M·(nn+rn)·iters/s) at M=1.4M + achieved HBM GB/s",
        "value": r["value"],
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{cfg.name}: IVHD loop, M={M:,} points N={cfg.N} ({cfg.K}-cluster "
                         f"{'Zipf(' + str(cfg.zipf_s) + ')' if cfg.sizes == 'zipf' else 'equal'} "
                         f"Gaussian mixture), exact kNN nn={nn}, rn={rn} redrawn every {R} "
                         f"iterations, {T} iterations per step, {main_mode} reduction"),
            "M": M, "N": cfg.N, "nn": nn, "rn": rn, "R": R, "T": T, "c": cfg.c, "a": cfg.a,
            "b": cfg.b, "mode": main_mode, "graphs": not args.no_graphs,
        },
        "gbps_alg": r["gbps_alg"],
        "us_per_iter": r["us_per_iter"],
        "modes": res,
        "knn_build_s": knn_s,
        "max_degree_bound": max_deg,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
