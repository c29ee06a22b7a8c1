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
                `traffic` = HBM-side bytes per launch from rocprofv3 counters
                when profiles/ holds figures taken on the current kernel source
  cpu_baseline  the FP64 oracle (plain C) timed on a bounded sample of the
                same workload shape, on every host thread and on one
                (N = 1 only)

Other workloads (one JSON line each, not the headline):
  --config C2   the loop at the MNIST shape (70,000 x 784, nn = 5)
  --config C4   the differentiable stress: forward (FP64 stress) and backward
                (gradient kernel) at 1,000,000 points, nn = 5, rn = 1
  --config C5   the parametric encoder: training throughput, embedding of the
                held-out points, and their kNN preservation beside plain IVHD
  --refine      the late-stage refinements (reverse-neighbour mask for the
                last 200 iterations, l1 distance for the last 50) against the
                plain loop, by Q_NX(10) and cf_10 (use with --config C2)
The C1-C3 lines also carry the loop's variants (Nesterov, l1, adaptive b,
Adam) timed on the same workload.
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
BF16_PEAK_TFLOPS = 2500.0
# the det step kernel's source and the constants that shape its launch (block
# size, hub threshold, vertex order): the stored traffic figure belongs to them
STEP_SOURCES = [os.path.join(ROOT, "paper_2303_05455_amd", "csrc", f) for f in ("step.hip", "ivhd_internal.h",
                                                                              "order.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_det_C3_traffic.md")
METRIC = "edge-updates/sec (M·(nn+rn)·iters/s) at M=1.4M + achieved HBM GB/s"
# adaptive-b threshold on |dT| (the kinetic energy change per step), per point:
# at the 1.4M-point shape 1e-4 accepts the first steps from rest at the
# configured b (1e-6 and 1e-5 rejected them and shrank b 4-16x for good)
ADAPT_TAU_PER_POINT = 1e-4
# Adam on the loop: each coordinate moves by about lr per step
ADAM_LR = 1e-3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest(paths=None) -> str:
    h = hashlib.sha1()
    for p in (paths or STEP_SOURCES):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:12]


def stored_traffic():
    """HBM-side bytes per launch of the det step kernel from the committed
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


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def host_threads() -> int:
    """Threads the oracle may use: OMP_NUM_THREADS when set, else the CPUs
    this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(cfg, iters, seed=0):
    """The FP64 oracle loop timed on the host: one thread over ``iters``
    iterations and every host thread (the threaded loop, equal to the
    one-thread loop bit for bit) over 4 * ``iters``."""
    import oracle
    import synth
    rng = np.random.default_rng([seed, cfg.cfg_id, 99])
    nn_idx, _, Y0 = synth.standin_graph(cfg, rng)
    oracle.build(force=False)
    kw = dict(rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed, R=cfg.R)
    V0 = np.zeros_like(Y0, dtype=np.float64)
    t0 = time.perf_counter()
    oracle.run(Y0, V0, nn_idx, T=iters, **kw)
    dt1 = time.perf_counter() - t0
    nt = host_threads()
    iters_n = 4 * iters
    t0 = time.perf_counter()
    oracle.run(Y0, V0, nn_idx, T=iters_n, threads=nt, **kw)
    dtn = time.perf_counter() - t0
    shape = (f"at M={cfg.M:,}, nn={cfg.nn}, rn={cfg.rn}, R={cfg.R} on a same-shape synthetic graph "
             f"(in-cluster targets with Pareto(2.2) popularity, largest in-degree near the exact graph's; the oracle never takes the GPU's kNN graph)")
    return {
        "value": cfg.M * (cfg.nn + cfg.rn) * iters_n / dtn,
        "unit": "edge-updates/s",
        "cores": nt,
        "kind": "oracle",
        "sample": (f"plain-C FP64 oracle loop on {nt} OpenMP threads (per-vertex gather, bitwise equal to "
                   f"the one-thread loop), {iters_n} of the {cfg.T} iterations {shape} ({dtn:.1f} s)"),
        "one_thread": {
            "value": cfg.M * (cfg.nn + cfg.rn) * iters / dt1, "unit": "edge-updates/s", "cores": 1,
            "sample": f"the one-thread edge-by-edge loop, {iters} iterations, same graph ({dt1:.1f} s)",
        },
    }


def gather_ceiling(M, nn, rn, kernel_s, dev, reps=20):
    """A second, labelled bound for the step kernel, which is bound by random
    8-byte position gathers (2 M (nn + rn) per iteration: every edge read from
    both ends): the time of the same number of gathers alone (the library's
    probe kernel, one 8-byte load and store per index), from one eighth of the
    position rows (one XCD's share, resident in its L2) and uniformly from all
    M rows (the footprint of the loop)."""
    import torch
    from paper_2303_05455_amd import ivhd_probe_gather
    G = 2 * M * (nn + rn)
    gen = torch.Generator().manual_seed(7)
    src = torch.rand((M, 2), generator=gen).to(dev)
    out = torch.empty((G, 2), dtype=torch.float32, device=dev)
    res = {"gathers_per_launch": G}
    for name, n_src in (("l2_resident_us", max(1, M // 8)), ("uniform_us", M)):
        idx = torch.randint(0, n_src, (G,), dtype=torch.int32, generator=gen).to(dev)
        ivhd_probe_gather(src, idx, out)
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(reps):
            ivhd_probe_gather(src, idx, out)
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) * 1e3 / reps
        del idx
    res["kernel_us"] = kernel_s * 1e6
    res["kernel_vs_l2_resident"] = res["l2_resident_us"] / res["kernel_us"]
    return res


def atomic_floor(M, rn, dev, reps=20):
    """The atomic mode's first pass delivers each of the M rn reactions of an
    iteration with one 64-bit integer atomic to a random vertex: the time of
    those atomics alone (the library's probe kernel), a labelled bound for
    that pass."""
    import torch
    from paper_2303_05455_amd import ivhd_probe_atomic
    n = M * rn
    gen = torch.Generator().manual_seed(8)
    idx = torch.randint(0, M, (n,), dtype=torch.int32, generator=gen).to(dev)
    acc = torch.zeros(M, dtype=torch.int64, device=dev)
    ivhd_probe_atomic(acc, idx)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        ivhd_probe_atomic(acc, idx)
    e1.record()
    torch.cuda.synchronize()
    return {"atomics_per_iteration": n, "atomics_alone_us": e0.elapsed_time(e1) * 1e3 / reps}


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


def build_graph(cfg, dev):
    import torch
    import synth
    from paper_2303_05455_amd import ivhd_knn_build
    t0 = time.perf_counter()
    X, labels, Y0 = synth.make_inputs(cfg)
    log(f"inputs {cfg.name}: M={cfg.M} N={cfg.N} ({time.perf_counter() - t0:.1f} s)")
    dX = torch.from_numpy(X).to(dev)
    del X
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nn_idx = ivhd_knn_build(dX, cfg.nn)
    torch.cuda.synchronize()
    knn_s = time.perf_counter() - t0
    indeg = torch.bincount(nn_idx.view(-1).long()[nn_idx.view(-1) >= 0], minlength=cfg.M)
    log(f"kNN graph (exact, nn={cfg.nn}) built in {knn_s:.2f} s; max nn in-degree {int(indeg.max())}")
    return dX, labels, Y0, nn_idx, knn_s, int(indeg.max())


def ivf_report(dX, exact, cfg):
    """Approximate kNN graph (inverted file, nlist ~ sqrt(M)) beside the exact
    one: build and search times, recall of the exact neighbours on 20,000
    sampled rows, for two probe counts."""
    import torch
    from paper_2303_05455_amd import ivhd_ivf_train, ivhd_ivf_search
    M = cfg.M
    nlist = 1 << int(round(np.log2(np.sqrt(M))))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C, a = ivhd_ivf_train(dX, nlist, 6)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    me = torch.arange(M, dtype=torch.int32, device=dX.device)
    rows = np.random.default_rng(9).choice(M, min(M, 20000), replace=False)
    ex = exact.cpu().numpy()
    out = {"nlist": nlist, "lloyd_iterations": 6, "train_s": train_s, "search": {}}
    for nprobe in (4, 16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = ivhd_ivf_search(dX, C, a, dX, cfg.nn, nprobe, self_idx=me)
        torch.cuda.synchronize()
        search_s = time.perf_counter() - t0
        g = g.cpu().numpy()
        recall = float(np.mean([len(np.intersect1d(g[i], ex[i])) for i in rows]) / cfg.nn)
        out["search"][str(nprobe)] = {"search_s": search_s, "recall": recall}
        log(f"approximate kNN (nlist {nlist}, nprobe {nprobe}): train {train_s:.2f} s + search "
            f"{search_s:.2f} s, recall {recall:.3f}")
    return out


def run_loop(args, cfg):
    import torch
    from paper_2303_05455_amd import Context
    dev = torch.device("cuda:0")
    M, nn, rn, R, T = cfg.M, cfg.nn, cfg.rn, cfg.R, cfg.T
    dX, labels, Y0, nn_idx, knn_s, max_in = build_graph(cfg, dev)
    knn_ivf = None if args.no_variants else ivf_report(dX, nn_idx, cfg)
    # heavy-ball stability: b * lambda_max < 2 (1 + a), lambda_max <= max degree + 1
    bound = 2 * (1 + cfg.a) / (max_in + nn + 2 * rn + 2)
    if cfg.b > bound:
        log(f"warning: b = {cfg.b} exceeds the stability bound {bound:.2g} of this graph")

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
        e0, e1 = events()
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
        if mode == "atomic" and rn > 0:
            res[mode]["reaction_atomics"] = atomic_floor(M, rn, dev)
            log(f"atomic mode: its {M * rn:,} reaction atomics alone take "
                f"{res[mode]['reaction_atomics']['atomics_alone_us']:.1f} us")

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
        e0, e1 = events()
        e0.record()
        ctx.step(launches)
        e1.record()
        torch.cuda.synchronize()
        per_launch = e0.elapsed_time(e1) / 1e3 / launches
        ctx.close()
        achieved = alg_bytes(M, nn, rn) / per_launch / 1e9
        roofline = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": stored_traffic() if cfg.name == "C3" else None,
            "kernel": "det_kernel", "alg_bytes_per_launch": alg_bytes(M, nn, rn),
            "us_per_launch": per_launch * 1e6,
            "gather_ceiling": gather_ceiling(M, nn, rn, per_launch, dev),
        }
        log(f"det step kernel: {per_launch * 1e6:.2f} us/launch, {achieved:.0f} GB/s algorithmic "
            f"({achieved / HBM_PEAK_GBPS:.1%} of 8 TB/s); the same number of random gathers alone: "
            f"{roofline['gather_ceiling']['l2_resident_us']:.1f} us from one L2's share of the positions, "
            f"{roofline['gather_ceiling']['uniform_us']:.1f} us uniform over all of them")

    # the thesis's variants of the loop on the same workload (det mode).  The
    # look-ahead and the l1 distance lower the stability bound of b (Nesterov:
    # b lambda_max < 2 (1 + a) / (1 + 2 a); l1: up to twice the stiffness), so
    # those two run at b / 2.
    variants = {}
    for name, kw, b in () if args.no_variants else (("nesterov", dict(nesterov=True), cfg.b / 2),
                                                     ("l1", dict(metric="l1"), cfg.b / 2),
                                                     ("adaptive", dict(), cfg.b), ("adaptive_from_10b", dict(), 10 * cfg.b),
                                                     ("adam", dict(), cfg.b)):
        y = d_y0.clone()
        v = torch.zeros_like(y)
        ctx = Context(nn_idx, y, v, rn=rn, a=cfg.a, b=b, c=cfg.c, seed=cfg.seed,
                      rn_resample_every=R, mode="det", **kw)
        if name.startswith("adaptive"):
            ctx.set_adaptive(True, tau=ADAPT_TAU_PER_POINT * M, g1=1.05, g2=0.5)
        if name == "adam":
            ctx.set_adam(True, lr=ADAM_LR)
        ctx.set_graphs(not args.no_graphs)
        ctx.step(T)
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        ctx.step(T)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        variants[name] = {"value": M * (nn + rn) * T / t, "us_per_iter": t * 1e6 / T, "b": b,
                          "final_stress": ctx.stress()}
        if name.startswith("adaptive"):
            variants[name].update(ctx.adaptive())
            variants[name]["tau"] = ADAPT_TAU_PER_POINT * M
        ctx.close()
        log(f"variant {name}: {variants[name]['value']:.4g} edge-updates/s, "
            f"{variants[name]['us_per_iter']:.2f} us/iter")

    # quality of the configured run's layout (T iterations from the start), off the timed region
    quality = None
    if not args.no_variants:
        y = d_y0.clone()
        v = torch.zeros_like(y)
        ctx = Context(nn_idx, y, v, rn=rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed, rn_resample_every=R)
        ctx.step(T)
        ctx.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        quality = layout_quality(dX, y, labels)
        quality["eval_s"] = time.perf_counter() - t0
        log(f"layout after {T} it: Q_NX(10) {quality['q_nx10']:.4f} (random {quality['q_nx10_random']:.2g}), "
            f"cf_2/10/100 {quality['cf2']:.4f}/{quality['cf10']:.4f}/{quality['cf100']:.4f}, "
            f"T(10) {quality['trust10']:.4f} on {quality['rows']} rows ({quality['eval_s']:.2f} s)")
    _NX_CACHE.clear()
    del dX

    cpu = None
    if not args.no_cpu:
        log(f"timing the FP64 oracle on {args.cpu_iters} iterations ...")
        cpu = cpu_baseline(cfg, args.cpu_iters)
        log(f"oracle: {cpu['value']:.4g} edge-updates/s")

    main_mode = "det" if "det" in res else modes[0]
    r = res[main_mode]
    return {
        "metric": METRIC,
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
                         f"Gaussian mixture), exact kNN nn={nn}, rn={rn} "
                         f"{'redrawn every ' + str(R) + ' iterations' if R else 'drawn once'}, "
                         f"{T} iterations per step, {main_mode} reduction"),
            "M": M, "N": cfg.N, "nn": nn, "rn": rn, "R": R, "T": T, "c": cfg.c, "a": cfg.a,
            "b": cfg.b, "mode": main_mode, "graphs": not args.no_graphs, "reorder": True,
        },
        "gbps_alg": r["gbps_alg"],
        "us_per_iter": r["us_per_iter"],
        "modes": res,
        "variants": variants,
        "knn_build_s": knn_s,
        "knn_ivf": knn_ivf,
        "max_nn_in_degree": max_in,
        "quality": quality,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def run_stress(args, cfg):
    """Forward (FP64 stress) and backward (gradient) of the differentiable stress."""
    import torch
    from paper_2303_05455_amd import Context
    from paper_2303_05455_amd import api
    from paper_2303_05455_amd.autograd import IVHDStress, StressEdges
    dev = torch.device("cuda:0")
    M, nn, rn = cfg.M, cfg.nn, cfg.rn
    dX, labels, Y0, nn_idx, knn_s, max_in = build_graph(cfg, dev)
    del dX
    # the random neighbours come from the loop's own draw (epoch 0)
    ctx = Context(nn_idx, torch.from_numpy(Y0).to(dev), rn=rn, c=cfg.c, seed=cfg.seed)
    rn_idx = ctx.rn_edges()
    ctx.close()
    edges = StressEdges(nn_idx, rn_idx, c=cfg.c)
    y = torch.from_numpy(Y0).to(dev).requires_grad_(True)
    E_edges = M * (nn + rn)
    for _ in range(args.warmup + 1):
        loss = IVHDStress.apply(y, edges)
        loss.backward()
    torch.cuda.synchronize()
    reps = max(args.steps, 1) * 20
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        edges.stress64(y.detach())
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / 1e3 / reps
    g = torch.empty_like(y)
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        edges.grad(y.detach(), out=g)
    e1.record()
    torch.cuda.synchronize()
    t_bwd = e0.elapsed_time(e1) / 1e3 / reps
    # what the autograd function runs when the layout requires a gradient:
    # stress and gradient from one pass, then the chain-rule scale
    one = torch.ones(1, dtype=torch.float32, device=dev)
    gs = torch.empty_like(g)
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        edges.stress_grad(y.detach(), out=g)
        api.ivhd_scale_f32(g, one, gs, stream=edges.stream)
    e1.record()
    torch.cuda.synchronize()
    t_fused = e0.elapsed_time(e1) / 1e3 / reps
    fwd_bytes = 8 * M + 4 * E_edges + 8
    bwd_bytes = 16 * M + 8 * E_edges
    log(f"stress forward {t_fwd * 1e6:.1f} us ({fwd_bytes / t_fwd / 1e9:.0f} GB/s), "
        f"backward {t_bwd * 1e6:.1f} us ({bwd_bytes / t_bwd / 1e9:.0f} GB/s), "
        f"forward+backward as the autograd function runs them {t_fused * 1e6:.1f} us")
    return {
        "metric": "differentiable IVHD stress: forward+backward edge evaluations/s at M=1M",
        "value": E_edges / t_fused, "unit": "edges/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": t_fused * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP64 stress accumulation)",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: IVHDStress autograd Function, M={M:,} N={cfg.N}, exact kNN "
                               f"nn={nn}, rn={rn}", "M": M, "nn": nn, "rn": rn},
        "forward_us": t_fwd * 1e6, "backward_us": t_bwd * 1e6, "fused_us": t_fused * 1e6,
        "fused": "stress and gradient from one pass (ivhd_edges_stress_grad) + the upstream scale "
                 "(ivhd_scale_f32), as IVHDStress runs them when y requires a gradient",
        "forward_gbps_alg": fwd_bytes / t_fwd / 1e9, "backward_gbps_alg": bwd_bytes / t_bwd / 1e9,
        "knn_build_s": knn_s, "max_nn_in_degree": max_in,
    }


_NX_CACHE = {}


def layout_quality(dX, y, labels, n_rows=10_000, seed=5):
    """Q_NX(10), cf_k (k = 2, 10, 100) and T(10) of a layout over a sample of
    rows, from the library's evaluation kernels (FP64 rank order); the data
    neighbourhoods of the sample are computed once per data array."""
    from paper_2303_05455_amd.evaluate import quality, sample_rows
    M = dX.shape[0]
    rows = sample_rows(M, n_rows, seed)
    hit = _NX_CACHE.get("x") is dX and _NX_CACHE.get("key") == (n_rows, seed)
    q = quality(dX, y, rows, labels=labels, ks=(2, 10, 100), k_qnx=(10,), k_trust=(10,),
                nx=_NX_CACHE["nx"] if hit else None)
    _NX_CACHE.clear()
    _NX_CACHE.update(x=dX, key=(n_rows, seed), nx=q["nx"])
    return {"rows": q["rows"], "q_nx10": q["q_nx"][10], "q_nx10_random": q["q_nx_random"][10],
            "cf2": q["cf"][2], "cf10": q["cf"][10], "cf100": q["cf"][100], "trust10": q["trust"][10]}


def run_encoder(args, cfg):
    """Parametric IVHD: train the MLP on the stress of its batches, embed the
    held-out points, score them by kNN preservation beside plain IVHD."""
    import torch
    import synth
    from paper_2303_05455_amd import Context, ivhd_knn_build
    from paper_2303_05455_amd.parametric import ParametricIVHD
    dev = torch.device("cuda:0")
    epochs = args.epochs
    dX, labels, _, nn_idx, knn_s, max_in = build_graph(cfg, dev)
    knn_ivf = ivf_report(dX, nn_idx, cfg)
    x16 = ParametricIVHD.to_bf16(dX)
    del dX
    torch.cuda.empty_cache()
    Xh, lab_h, _ = synth.make_inputs(cfg, heldout=True)
    dXh = torch.from_numpy(Xh).to(dev)
    xh16 = ParametricIVHD.to_bf16(dXh)
    enc = ParametricIVHD(cfg.N, (512, 512), batch=8192, nn=cfg.nn, rn=cfg.rn, c=cfg.c, lr=1e-3, seed=cfg.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    enc.fit(x16, nn_idx, epochs=epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = epochs * ((cfg.M + 8191) // 8192)
    rows = 8192 * (1 + cfg.nn + cfg.rn)
    flop_step = rows * 2 * (3 * cfg.N * 512 + 3 * 512 * 512) - rows * 2 * cfg.N * 512  # no input gradient
    log(f"trained {epochs} epochs ({steps} steps) in {t_train:.1f} s: "
        f"{steps / t_train:.1f} steps/s, {flop_step * steps / t_train / 1e12:.0f} TFLOP/s; "
        f"loss {enc.losses[0]:.4g} -> {enc.losses[-1]:.4g}")
    Zh = torch.empty((cfg.M_heldout, 2), dtype=torch.float32, device=dev)
    enc.embed(xh16, Zh)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    enc.embed(xh16, Zh)
    e1.record()
    torch.cuda.synchronize()
    t_embed = e0.elapsed_time(e1) / 1e3
    q_enc = layout_quality(dXh, Zh, lab_h)
    # plain IVHD on the held-out points (its own kNN graph, 2000 iterations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nn_h = ivhd_knn_build(dXh, cfg.nn)
    max_in_h = int(torch.bincount(nn_h.view(-1).long(), minlength=cfg.M_heldout).max())
    bound_h = 2 * (1 + cfg.a) / (max_in_h + cfg.nn + 2 * cfg.rn + 2)
    if cfg.b > bound_h:
        log(f"warning: b = {cfg.b} exceeds the stability bound {bound_h:.2g} of the held-out graph "
            f"(max nn in-degree {max_in_h})")
    y = torch.from_numpy(synth.init_positions(cfg.M_heldout, np.random.default_rng(1))).to(dev)
    ctx = Context(nn_h, y, rn=cfg.rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=1, rn_resample_every=100)
    ctx.step(2000)
    torch.cuda.synchronize()
    t_ivhd = time.perf_counter() - t0
    q_ivhd = layout_quality(dXh, y, lab_h)
    ctx.close()
    # fallback: plain IVHD started from the encoder's layout, 200 iterations
    t0 = time.perf_counter()
    y2 = enc.embed(xh16, refine_iters=200, nn_idx=nn_h, b=cfg.b, seed=1)
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    q_fb = layout_quality(dXh, y2, lab_h)
    q_enc_, cf_enc = q_enc["q_nx10"], q_enc["cf10"]
    q_ivhd_, cf_ivhd = q_ivhd["q_nx10"], q_ivhd["cf10"]
    q_fb_, cf_fb = q_fb["q_nx10"], q_fb["cf10"]
    log(f"held-out {cfg.M_heldout}: encoder Q_NX(10)={q_enc_:.4f} cf_10={cf_enc:.3f} in {t_embed * 1e3:.2f} ms; "
        f"plain IVHD Q_NX(10)={q_ivhd_:.4f} cf_10={cf_ivhd:.3f} in {t_ivhd:.2f} s; IVHD from encoder "
        f"(200 it) Q_NX(10)={q_fb_:.4f} cf_10={cf_fb:.3f}")
    return {
        "metric": "parametric IVHD: held-out embedding points/s (MLP 784-512-512-2, BF16 MFMA)",
        "value": cfg.M_heldout / t_embed, "unit": "points/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": t_train * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (FP32 accumulate)", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: MLP {cfg.N}-512-512-2 trained {epochs} epochs on the stress of "
                               f"batches of 8192 sources (nn={cfg.nn}, rn={cfg.rn}) over M={cfg.M:,}; "
                               f"{cfg.M_heldout:,} held-out points embedded",
                   "M": cfg.M, "N": cfg.N, "epochs": epochs, "batch": 8192},
        "train_s": t_train, "train_steps_per_s": steps / t_train,
        "train_tflops": flop_step * steps / t_train / 1e12,
        "train_mfma_frac": flop_step * steps / t_train / 1e12 / BF16_PEAK_TFLOPS,
        "loss_first_epoch": enc.losses[0], "loss_last_epoch": enc.losses[-1],
        "embed_ms": t_embed * 1e3, "quality_encoder": q_enc, "quality_plain_ivhd_2000it": q_ivhd,
        "quality_ivhd_from_encoder_200it": q_fb,
        "plain_ivhd_s": t_ivhd, "fallback_s": t_fb,
        "knn_build_s": knn_s, "knn_ivf": knn_ivf, "max_nn_in_degree": max_in,
        "heldout_max_nn_in_degree": max_in_h,
    }


def run_refine(args, cfg):
    """Late-stage refinements of the thesis's improvements chapter (the
    reverse-neighbour mask with a helper graph of 4 nn for the last 200
    iterations, the l1 distance for the last 50: late_stage.staged_run)
    against the plain loop with the same iteration count; quality by the
    sample scores, cost as the extra wall time of the refinement stages."""
    import torch
    from paper_2303_05455_amd import Context
    from paper_2303_05455_amd.late_stage import staged_run
    dev = torch.device("cuda:0")
    M, nn, rn, T = cfg.M, cfg.nn, cfg.rn, cfg.T
    dX, labels, Y0, nn_idx, knn_s, max_in = build_graph(cfg, dev)
    kw = dict(rn=rn, a=cfg.a, b=cfg.b, c=cfg.c, seed=cfg.seed, rn_resample_every=cfg.R)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y_base = torch.from_numpy(Y0).to(dev)
    ctx = Context(nn_idx, y_base, torch.zeros_like(y_base), **kw)
    ctx.step(T)
    torch.cuda.synchronize()
    ctx.close()
    t_base = time.perf_counter() - t0
    q_base = layout_quality(dX, y_base, labels)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = torch.from_numpy(Y0).to(dev)
    info = staged_run(nn_idx, y, torch.zeros_like(y), T=T, x=dX, **kw)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    q_ref = layout_quality(dX, y, labels)
    kept = info["kept"]
    log(f"refine {cfg.name}: plain {T} it Q_NX(10)={q_base['q_nx10']:.4f} cf_10={q_base['cf10']:.4f} in "
        f"{t_base:.2f} s; reverse-neighbour mask (keeps {kept:.1%} of nn edges) for the last 200 it, l1 for "
        f"the last 50: Q_NX(10)={q_ref['q_nx10']:.4f} cf_10={q_ref['cf10']:.4f} in {t_ref:.2f} s")
    return {
        "metric": "late-stage refinement: Q_NX(10) and cf_10 vs plain IVHD, same iteration count",
        "value": t_ref, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": t_ref * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: M={M:,} N={cfg.N}, nn={nn}, rn={rn}, {T} iterations; helper "
                               f"kNN graph of {4 * nn}; reverse-neighbour mask for the last 200, l1 "
                               f"distance for the last 50", "M": M, "N": cfg.N, "T": T},
        "quality_plain": q_base, "plain_s": t_base, "quality_refined": q_ref, "refined_s": t_ref,
        "nn_edges_kept": kept, "knn_build_s": knn_s,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--mode", default="both", choices=["det", "atomic", "both"])
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the Nesterov / l1 / adaptive lines")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB")
    ap.add_argument("--no-sub", action="store_true",
                    help="skip the differentiable-stress (C4) and encoder (C5) sub-records of the default run")
    ap.add_argument("--refine", action="store_true",
                    help="late-stage refinements (reverse-neighbour mask, l1) vs the plain loop")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import synth
    cfg = synth.CONFIGS[args.config]
    if args.refine:
        out = run_refine(args, cfg)
    elif cfg.name == "C4":
        out = run_stress(args, cfg)
    elif cfg.name == "C5":
        out = run_encoder(args, cfg)
    else:
        out = run_loop(args, cfg)
        if cfg.name == "C3" and not args.no_sub:
            # the differentiable stress and the parametric encoder at their own
            # shapes, measured in the same run (sub-records; not the headline)
            torch.cuda.empty_cache()
            out["sub"] = {"C4": run_stress(args, synth.CONFIGS["C4"])}
            torch.cuda.empty_cache()
            out["sub"]["C5"] = run_encoder(args, synth.CONFIGS["C5"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
