#!/usr/bin/env python3
"""Benchmark of the layered sparse-DNN forward on one MI355X.

Workload (the metric's configuration): the batched forward at the largest shape
one GPU holds, 65536 neurons x 1920 layers (4.03e9 nonzeros, int32 ids + fp32
weights, 32 GB resident), 32 inputs per neuron (weights 1/16, bias -0.45, clip
32), 15000 Bernoulli(0.2) binary input rows in 20 uneven batches of 250..4000 rows,
all batches in one pass (one persistent launch or one merged graph), fp32, drawn by
the seeded device generator of sdnn_inputs (seed 4).  A step is one sdnn_forward
over all 15000 rows and all 1920 layers, with the network and the inputs resident
in HBM.  The metric is edges/s = rows x nnz(W) / step time.

Prints ONE JSON line.  Besides the required fields it carries:
  roofline      the dominant kernel's algorithmic HBM bytes per launch / its
                average duration (HIP events on the library's own stream),
                against MI355X's 8 TB/s; traffic from committed rocprofv3 counters
  cpu_baseline  the FP64 oracle timed on this host on a bounded row sample
                (all host threads, and one thread on a smaller sample)
  extras        the plain form (batches one after another) of the same workload,
                the tuned and default plans, and, with --extras: the C2 plain
                forward, a full-live C2 layer, S2 (sustained), C3 and S3 batched vs
                plain, S4 (sustained at 65536 neurons), the G5 bwd/fwd ratio
  streams       with --streams C3,S2_20,C4: the stream/graph forms of the batched
                forward (explicit graph, eager and captured over 1-8 streams)
  streamed      with --streamed: parameters in pinned host memory streamed through
                two device slots vs the same kernels over resident parameters
  table         with --table C1,C2,...: per-config edges/s, algorithmic GB/s and
                roofline fraction, plain vs batched, C5 backward / forward
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
K = 32


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", default="C4", choices=["C4", "C2", "C3", "S2", "S3", "S4", "C1", "C5", "G5"],
                    help="workload of the JSON line: C4 (batched, 65536 x 1920; the default) or another "
                         "configuration (for profiling one kernel family)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--engine", default="auto", choices=["auto", "graph", "graph_merged", "persistent", "eager"],
                    help="auto: time graph and persistent in warm-up and keep the faster")
    ap.add_argument("--extras", dest="extras", action="store_true", default=True)
    ap.add_argument("--no-extras", dest="extras", action="store_false")
    ap.add_argument("--cpu", dest="cpu", action="store_true", default=True)
    ap.add_argument("--no-cpu", dest="cpu", action="store_false")
    ap.add_argument("--cpu-rows", type=int, default=15000, help="row sample for the oracle baseline (all threads)")
    ap.add_argument("--cpu-rows1", type=int, default=400, help="row sample for the one-thread oracle baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 5 times (the reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counter scale) and exit")
    ap.add_argument("--streams", default="", metavar="CONFIGS",
                    help="also time the stream/graph forms on these configs (C3,S2_20,C4)")
    ap.add_argument("--streamed", action="store_true", default=False,
                    help="also time the forward with parameters streamed from host memory")
    ap.add_argument("--corun", default="", metavar="COUNTS",
                    help="co-run throughput: run this many copies of the inference program at once "
                         "(e.g. 1,2,4) and report weighted speedup")
    ap.add_argument("--corun-args", default="", help="extra arguments for each co-running program")
    ap.add_argument("--table-forms", default="plain,merged,persistent",
                    help="forms the results table times (a profiled run without cooperative launches: plain,merged)")
    ap.add_argument("--table", default="", metavar="CONFIGS",
                    help="also run the per-config results table (e.g. C1,C2,C3,C4,C5,S2,S3)")
    ap.add_argument("--plain", dest="plain", action="store_true", default=True,
                    help="also time the plain form (batches one after another) of a batched headline")
    ap.add_argument("--no-plain", dest="plain", action="store_false")
    ap.add_argument("--tune", action="store_true", default=True)
    ap.add_argument("--no-tune", dest="tune", action="store_false")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def forward_bytes(prof, N, L):
    """Algorithmic HBM bytes of one forward from its row profile prof[0..L]:
    per layer with R_l > 0 rows: 8NK (ids + weights) + 4N (bias) + 8 R_l N (read
    and write the alive rows) + 4 (R_l + R_{l+1}) (work lists)."""
    tot = 0
    for l in range(L):
        r, r1 = int(prof[l]), int(prof[l + 1])
        if r > 0:
            tot += 8 * N * K + 4 * N + 8 * r * N + 4 * (r + r1)
    return tot


# committed rocprofv3 counter summaries of the persistent chain kernels, per
# headline workload: (summary, kernel source it was taken with)
PROFILES = {"C4": "k_chain_rowu_C4_forward.md", "C2": "k_chain_sched_C2_forward.md"}
# the sources each profiled chain kernel is built from (hashed together); for the
# chunked kernel also its create-time neuron pairing, whose order sets how the
# parts of a row stream drift apart and so how often rows are fetched again
KERNEL_SOURCES = {"C4": ("sdnn_rowc.hip", "sdnn_device.hpp", "sdnn_internal.hpp", "sdnn_rowsched.hip"),
                  "C2": ("sdnn_fwd.hip", "sdnn_device.hpp", "sdnn_internal.hpp")}


def kernel_source_sha256(workload):
    import hashlib
    h = hashlib.sha256()
    for src in KERNEL_SOURCES[workload]:
        h.update(open(os.path.join(ROOT, "paper_2004_10908_amd", "csrc", src), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the persistent chain kernel from its committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the summary is for another
    kernel or the kernel source has changed since those counters were taken."""
    if workload not in PROFILES:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", PROFILES[workload])).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        k, _, v = line.strip().partition(": ")
        if k in ("traffic_bytes_per_launch", "kernel_source_sha256", "kernel"):
            vals[k] = v.strip()
    if len(vals) != 3 or vals["kernel"] != kernel or kernel_source_sha256(workload) != vals["kernel_source_sha256"]:
        return None
    return int(vals["traffic_bytes_per_launch"])


def chain_kernel_name(plan):
    """Name of the persistent chain kernel a plan runs (as rocprofv3 reports it)."""
    T, NT, v = plan["rows_per_tile"], plan["threads"], plan["variant"]
    if v == 2:
        return "sdnn::k_chain_sched<512, 40>"
    if v == 3:
        return f"sdnn::k_chain_wide<{T}, {NT}>"
    if v == 4:
        return "sdnn::k_chain_row"
    if v == 5:
        return "sdnn::k_chain_row_sched"
    if v == 6:
        return f"sdnn::k_chain_rowc<{T}>"
    if v == 7:
        return f"sdnn::k_chain_rowu<{T}>"
    return f"sdnn::k_chain<{T}, {NT}, {'true' if v == 0 else 'false'}>"


def live_edges(prof, N, L):
    return sum(int(prof[l]) for l in range(L)) * N * K


def time_forward(torch, net, y0, out, steps, warmup, batch_off=None, on_start=None):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        net.forward(y0, batch_off=batch_off, out=out)
    torch.cuda.synchronize()
    if on_start is not None:
        on_start()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        net.forward(y0, batch_off=batch_off, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2004_10908_amd as P
    import sdnn_inputs as gen

    if not os.path.exists(P.LIB_PATH):
        from paper_2004_10908_amd import build as b
        b.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "launches": 5}))
        return

    name = args.config
    cfg = gen.CONFIGS[name]
    N, L, B = cfg.n_neurons, cfg.n_layers, cfg.rows
    nnz = cfg.nnz
    t0 = time.time()
    idx, w, b = device_net(torch, gen, cfg, dev)
    y0 = device_inputs(torch, cfg, dev)
    off = [int(v) for v in gen.make_batches(cfg)] if cfg.n_batches > 1 else None
    torch.cuda.synchronize()
    log(f"generated {name} in {time.time() - t0:.1f}s")
    net = P.Net(idx, w, b, max_rows=B)
    default_plan = net.plan
    batched = off is not None
    out = {}
    net.forward(y0, batch_off=off, out=out, profile=True)
    extras = {"default_plan": default_plan}
    if args.tune:
        # the autotuner times every variant of the net's kernel family on the
        # workload's own rows (one full-live layer of the persistent chain kernel)
        rows0 = B
        eng0 = "persistent"
        net.set_exec(eng0)
        extras["default_plan_ms"] = round(time_forward(torch, net, y0, out, 3, 1, batch_off=off), 4)
        t1 = time.time()
        plan = net.tune(rows0, y_sample=y0[:rows0])
        extras["tune_seconds"] = round(time.time() - t1, 2)
        extras["tuned_plan"] = plan
        extras["tuned_plan_ms"] = round(time_forward(torch, net, y0, out, 3, 1, batch_off=off), 4)
        log("default plan", default_plan, extras["default_plan_ms"], "ms; tuned plan", plan,
            extras["tuned_plan_ms"], "ms")

    # engine choice (warm-up): the batched forms (persistent launch, merged graph), or
    # for one batch the graph and the persistent launch
    engines = {}
    cands = (["persistent", "graph_merged"] if batched else ["graph", "persistent"]) \
        if args.engine == "auto" else [args.engine]
    for eng in cands:
        net.set_exec(eng)
        engines[eng] = time_forward(torch, net, y0, out, max(2, args.warmup), 1, batch_off=off)
    engine = min(engines, key=engines.get)
    net.set_exec(engine)
    log("warm-up engine times (ms)", engines, "->", engine)

    # ---------------------------------------------------------------- timed region
    # In persistent mode the library brackets its chain kernel with HIP events on the
    # stream it launches on; those give the dominant kernel's own average duration.
    timed_kernel = engine == "persistent"
    if timed_kernel:
        net.set_timing(True)
    ms = time_forward(torch, net, y0, out, args.steps, args.warmup, batch_off=off,
                      on_start=(lambda: net.kernel_time()) if timed_kernel else None)   # drop warm-up events
    k_ms, k_n = net.kernel_time() if timed_kernel else (0.0, 0)
    if timed_kernel:
        net.set_timing(False)
        k_avg = k_ms / k_n if k_n else ms
    prof = out["layer_rows"].cpu().numpy()
    n_nz = int(out["n_nz"].item())
    value = B * nnz / (ms / 1e3)
    alg = forward_bytes(prof, N, L)
    plan = net.plan
    if timed_kernel:
        kernel = chain_kernel_name(plan)
        alg_launch, dur_ms = alg, k_avg
        kdesc = kernel + " (persistent forward: all layers of all batches, one launch per step)"
    else:
        kernel = None
        alg_launch, dur_ms = alg / L, ms / L
        kdesc = f"layer kernel of plan {plan} (one graph node per layer; step time / layers)"
    achieved = alg_launch / (dur_ms / 1e3) / 1e9
    tb = measured_traffic(name, kernel) if timed_kernel else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(tb / (dur_ms / 1e3) / 1e9, 1) if tb else None,
                "traffic_bytes_per_launch": tb, "kernel": kdesc,
                "alg_bytes_per_launch": alg_launch, "avg_launch_ms": round(dur_ms, 4)}
    log(f"{name} {engine}: {ms:.3f} ms/step, {value:.3e} edges/s, profile head {prof[:5].tolist()}, nz {n_nz}")
    extras.update({"engines_ms": {k: round(v, 4) for k, v in engines.items()}, "plan": plan,
                   "profile_head": prof[:6].tolist(), "live_edges_per_s": live_edges(prof, N, L) / (ms / 1e3),
                   "alg_bytes": alg})
    if batched and args.plain:
        # the plain form of the same workload: the batches one after another through
        # the layer graph
        net.set_exec("graph")
        pms = time_forward(torch, net, y0, out, 2, 1, batch_off=off)
        extras["plain_ms"] = round(pms, 3)
        extras["plain_edges_per_s"] = B * nnz / (pms / 1e3)
        extras["batched_over_plain"] = round(pms / ms, 3)
        log(f"{name} plain (graph, batches in turn): {pms:.3f} ms")
    net.close()
    del idx, w, b, out
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- extras
    if args.extras:
        try:
            extras.update(bench_extras(args, torch, np, P, gen, dev))
        except Exception as e:  # extras never hide the headline
            extras["error"] = repr(e)
            log("extras failed:", repr(e))
    if args.streams:
        extras["streams"] = bench_streams(args, torch, P, gen, dev)
    if args.streamed:
        extras["streamed"] = bench_streamed(args, torch, P, gen, dev)
    if args.table:
        extras["table"] = bench_table(args, torch, P, gen, dev)
    if args.corun:
        extras["corun"] = bench_corun(args)

    cpu = None
    if args.cpu:
        try:
            cpu = cpu_baseline(args, np, gen, cfg, y0, off)
        except Exception as e:
            log("cpu baseline failed:", repr(e))
    del y0
    torch.cuda.empty_cache()

    desc = (f"{name} {'batched' if batched else 'plain'} forward: {N} neurons x {L} layers, k=32, "
            f"{'w=1/16' if cfg.weight == 'const' else cfg.weight + ' weights'}, b={cfg.bias}, clip {cfg.clamp:g}, "
            f"{B} Bernoulli({cfg.density:g}) rows" + (f" in {len(off) - 1} uneven batches" if batched else "")
            + f", seed {cfg.seed}")
    line = {"metric": "edges/s (inputs x nnz(W) / s)", "value": value, "unit": "edges/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
            "config": {"workload": desc, "global_batch": B, "seq_len": None,
                       "parallelism": "single-gpu", "engine": engine},
            "roofline": roofline, "cpu_baseline": cpu, "extras": extras}
    print(json.dumps(line), flush=True)
    # every GPU call is done: unload the library now rather than at interpreter exit
    torch.cuda.synchronize()
    P.sdnn.unload()


def full_live_layer(torch, net, y, reps=10):
    """Time sdnn_layer on every row (no compaction): the steady-state kernel rate."""
    yo = torch.empty_like(y)
    stream = torch.cuda.current_stream()
    net.layer(0, y, yo)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        net.layer(0, y, yo)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def device_net(torch, gen, cfg, dev, n_layers=None):
    L = cfg.n_layers if n_layers is None else n_layers
    idx = torch.empty((L, cfg.n_neurons, K), dtype=torch.int32, device=dev)
    w = torch.empty((L, cfg.n_neurons, K), dtype=torch.float32, device=dev)
    b = torch.empty((L, cfg.n_neurons), dtype=torch.float32, device=dev)
    for l in range(L):
        i_, w_, b_ = gen.make_layer_device(cfg, l, dev)
        idx[l].copy_(i_)
        w[l].copy_(w_)
        b[l].copy_(b_)
    return idx, w, b


def device_inputs(torch, cfg, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(cfg.seed * 7919 + 1)
    if cfg.row_density:
        p = torch.rand((cfg.rows, 1), generator=g, device=dev) * 0.4 + 0.1
    else:
        p = cfg.density
    return (torch.rand((cfg.rows, cfg.n_neurons), generator=g, device=dev) < p).float()


def bench_extras(args, torch, np, P, gen, dev):
    ex = {}
    # C2: the plain forward of 4096 neurons x 480 layers, 60000 rows (the scheduled
    # resident-weight kernel), and a full-live layer of its shape (every row alive):
    # the kernel's steady-state rate
    cfg = gen.CONFIGS["C2"]
    N = cfg.n_neurons
    idx, w, b = device_net(torch, gen, cfg, dev)
    y0 = device_inputs(torch, cfg, dev)
    net = P.Net(idx, w, b, max_rows=cfg.rows)
    o = {}
    net.forward(y0, out=o, profile=True)
    res = {"plan": net.plan}
    for eng in ("graph", "persistent"):
        net.set_exec(eng)
        ms = time_forward(torch, net, y0, o, 5, 2)
        prof = o["layer_rows"].cpu().numpy()
        alg = forward_bytes(prof, N, cfg.n_layers)
        res[eng] = {"ms": round(ms, 4), "edges_per_s": cfg.rows * cfg.nnz / (ms / 1e3),
                    "live_edges_per_s": live_edges(prof, N, cfg.n_layers) / (ms / 1e3),
                    "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
    res["profile_head"] = prof[:5].tolist()
    ms = full_live_layer(torch, net, y0)
    byt = 8 * N * K + 4 * N + 8 * y0.shape[0] * N
    res["full_live_layer"] = {"rows": y0.shape[0], "ms": round(ms, 4), "alg_GBps": round(byt / ms / 1e6, 1),
                              "frac": round(byt / ms / 1e6 / HBM_PEAK_GBS, 4),
                              "edges_per_s": y0.shape[0] * N * K / (ms / 1e3)}
    ex["C2"] = res
    log("C2", res)
    net.close()
    del idx, w, b, y0, o
    torch.cuda.empty_cache()

    # S2: sustained companion (rows stay alive), device-drawn net and inputs
    cfg = gen.CONFIGS["S2"]
    N = cfg.n_neurons
    idx, w, b = device_net(torch, gen, cfg, dev)
    y0 = device_inputs(torch, cfg, dev)
    net = P.Net(idx, w, b, max_rows=cfg.rows)
    net.tune(cfg.rows, y_sample=y0)
    o = {}
    net.forward(y0, out=o, profile=True)
    res = {}
    for eng in ("graph", "persistent"):
        net.set_exec(eng)
        ms = time_forward(torch, net, y0, o, 3, 1)
        prof = o["layer_rows"].cpu().numpy()
        alg = forward_bytes(prof, N, cfg.n_layers)
        res[eng] = {"ms": round(ms, 3), "edges_per_s": cfg.rows * cfg.nnz / (ms / 1e3),
                    "live_edges_per_s": live_edges(prof, N, cfg.n_layers) / (ms / 1e3),
                    "alg_GBps": round(alg / ms / 1e6, 1), "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
    res["alive_profile"] = [int(v) for v in prof[[0, 1, 2, 5, 10, 20, 100, 479, 480]]]
    ex["S2"] = res
    log("S2", res)
    net.close()
    del idx, w, b, y0, o
    torch.cuda.empty_cache()

    # C3 / S3 / S4: batched (one pass over all 20 uneven batches) vs plain (batches one
    # after another); the plan tuned on the first batch against the default one
    for name in ("C3", "S3", "S4"):
        cfg = gen.CONFIGS[name]
        N, L = cfg.n_neurons, cfg.n_layers
        idx, w, b = device_net(torch, gen, cfg, dev)
        y0 = device_inputs(torch, cfg, dev)
        off = [int(v) for v in gen.make_batches(cfg)]
        net = P.Net(idx, w, b, max_rows=cfg.rows)
        o = {}
        net.forward(y0, out=o, profile=True)
        r = {"default_plan": net.plan}
        reps = 1 if name == "S4" else (2 if name == "S3" else 3)
        net.set_exec("persistent")
        r["default_plan_persistent_ms"] = round(time_forward(torch, net, y0, o, reps, 1, batch_off=off), 3)
        r["tuned_plan"] = net.tune(cfg.rows, y_sample=y0)
        prof = o["layer_rows"].cpu().numpy()
        alg = forward_bytes(prof, N, L)
        forms = ("persistent", "graph_merged") if name == "S4" else ("graph", "graph_merged", "persistent")
        for eng in forms:
            net.set_exec(eng)
            ms = time_forward(torch, net, y0, o, reps, 1, batch_off=off)
            r[eng] = {"ms": round(ms, 3), "edges_per_s": cfg.rows * cfg.nnz / (ms / 1e3),
                      "live_edges_per_s": live_edges(prof, N, L) / (ms / 1e3),
                      "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
        r["batched_best"] = max(("graph_merged", "persistent"), key=lambda k: r[k]["edges_per_s"])
        if "graph" in r:
            r["plain"] = "graph (batches one after another)"
            r["batched_over_plain"] = r[r["batched_best"]]["edges_per_s"] / r["graph"]["edges_per_s"]
        r["alive_profile"] = [int(prof[i]) for i in (0, 1, 2, 5, 10, 100, L - 1, L)]
        ex[name] = r
        log(name, r)
        net.close()
        del idx, w, b, y0, o
        torch.cuda.empty_cache()

    # G5: forward + backward (bwd/fwd ratio) on 4096 rows, checkpoints every 16 layers
    cfg = gen.CONFIGS["G5"]
    idx, w, b = device_net(torch, gen, cfg, dev)
    y0 = device_inputs(torch, cfg, dev)
    net = P.Net(idx, w, b, max_rows=cfg.rows, ckpt_every=16, flags=P.sdnn.SDNN_TRAINABLE)
    net.set_exec("graph")
    o = net.forward(y0, ckpt=True)
    dy = torch.randn_like(o["y"]) * 1e-4
    stream = torch.cuda.current_stream()
    for _ in range(2):
        net.forward(y0, ckpt=True, out=o)
        net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 3
    fwd_ms = bwd_ms = 0.0
    for _ in range(reps):
        e[0].record(stream)
        net.forward(y0, ckpt=True, out=o)
        e[1].record(stream)
        net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
        e[2].record(stream)
        torch.cuda.synchronize()
        fwd_ms += e[0].elapsed_time(e[1]) / reps
        bwd_ms += e[1].elapsed_time(e[2]) / reps
    ex["G5"] = {"fwd_ms": round(fwd_ms, 3), "bwd_ms": round(bwd_ms, 3), "bwd_over_fwd": round(bwd_ms / fwd_ms, 3),
                "n_nz": int(o["n_nz"].item()), "fwd_edges_per_s": cfg.rows * cfg.nnz / (fwd_ms / 1e3)}
    log("G5", ex["G5"])
    net.close()
    return ex


def bench_streams(args, torch, P, gen, dev):
    """Graph-construction forms over batches (the paper's stream-count experiment):
    the explicitly built graph (batches in turn, and merged), the persistent launch,
    eager launches round-robin over K streams, and the same launches captured from K
    streams into one graph.  Workspace = the nets' scratch memory."""
    from paper_2004_10908_amd.streams import StreamForward
    named = {"C3": gen.CONFIGS["C3"], "C4": gen.CONFIGS["C4"],
             "S2_20": gen.CONFIGS["S2"].with_(n_batches=20, batch_lo=1500, batch_hi=4500)}
    sres = {}
    for name in args.streams.split(","):
        cfg = named[name]
        idx, w, b = device_net(torch, gen, cfg, dev)
        y0 = device_inputs(torch, cfg, dev)
        off = [int(v) for v in gen.make_batches(cfg)]
        net = P.Net(idx, w, b, max_rows=cfg.rows)
        o = {}
        net.forward(y0, batch_off=off, out=o)
        r = {"batches": len(off) - 1, "rows": cfg.rows, "N": cfg.n_neurons, "layers": cfg.n_layers}
        for eng in ("graph", "graph_merged", "persistent"):
            net.set_exec(eng)
            r[eng] = {"ms": round(time_forward(torch, net, y0, o, 2, 1, batch_off=off), 3),
                      "workspace_MB": round(net.ws_bytes / 2**20, 1)}
        base = o["y"].clone()
        y = torch.empty_like(y0)
        for cap in (False, True):
            for k in ((1, 2, 4) if not cap else (1, 2, 4, 8)):
                # each stream's net holds its own workspace (at 65536 neurons, lane
                # images of 26 GB): skip a stream count whose nets would not fit
                free = torch.cuda.mem_get_info(dev)[0]
                if k * net.ws_bytes > 0.85 * free:
                    r[("captured" if cap else "eager") + f"_{k}"] = {
                        "skipped": f"{k} stream nets need up to {k * net.ws_bytes / 2**30:.0f} GiB, "
                                   f"{free / 2**30:.0f} GiB free"}
                    continue
                sf = StreamForward(idx, w, b, off, k, capture=cap)
                sf.run(y0, y)
                torch.cuda.synchronize()
                same = bool(torch.equal(y, base))
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(2):
                    sf.run(y0, y)
                e1.record()
                torch.cuda.synchronize()
                r[("captured" if cap else "eager") + f"_{k}"] = {"ms": round(e0.elapsed_time(e1) / 2, 3),
                                                                  "workspace_MB": round(sf.workspace_bytes / 2**20, 1),
                                                                  "equal_to_graph": same}
                sf.close()
                del sf
                torch.cuda.empty_cache()                  # (the next stream count's nets need the room)
        sres[name] = r
        log("streams " + name, r)
        net.close()
        del idx, w, b, y0, o, base, y
        torch.cuda.empty_cache()
    return sres


def bench_streamed(args, torch, P, gen, dev):
    """Parameters in pinned host memory streamed through two device slots, against the
    same kernels over resident parameters (layer by layer over all rows)."""
    from paper_2004_10908_amd.streamed import StreamedForward
    cases = (("C2_4096", gen.CONFIGS["C2"].with_(rows=4096)),
             ("C4_1000x64", gen.CONFIGS["C4"].with_(rows=1000, n_layers=64)))
    res = {}
    for name, cfg in cases:
        idx, w, b = device_net(torch, gen, cfg, dev)
        y0 = device_inputs(torch, cfg, dev)
        net = P.Net(idx, w, b, max_rows=cfg.rows, flags=P.sdnn.SDNN_NO_SCHEDULE | P.sdnn.SDNN_NO_COMPACTION)
        ya, yb = torch.empty_like(y0), torch.empty_like(y0)

        def resident():
            src = y0
            for l in range(cfg.n_layers):
                dst = yb if (cfg.n_layers - 1 - l) % 2 == 0 else ya
                net.layer(l, src, dst)
                src = dst

        sf = StreamedForward(idx.cpu().pin_memory(), w.cpu().pin_memory(), b.cpu().pin_memory(), cfg.rows)
        out = torch.empty_like(y0)
        r = {"N": cfg.n_neurons, "layers": cfg.n_layers, "rows": cfg.rows,
             "param_bytes_per_forward": int(idx.numel() * 8 + b.numel() * 4), "slot_bytes": sf.slot_bytes}
        for key, fn in (("resident", resident), ("streamed", lambda: sf.run(y0, out))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(2):
                fn()
            e1.record()
            torch.cuda.synchronize()
            r[key + "_ms"] = round(e0.elapsed_time(e1) / 2, 3)
        r["equal"] = bool(torch.equal(out, yb))
        r["copy_GBps_if_all_exposed"] = round(r["param_bytes_per_forward"] / (r["streamed_ms"] / 1e3) / 1e9, 1)
        res[name] = r
        log("streamed " + name, r)
        sf.close()
        net.close()
        del idx, w, b, y0, ya, yb, out
        torch.cuda.empty_cache()
    return res


def bench_table(args, torch, P, gen, dev):
    """The per-config results table: nominal and live edges/s, algorithmic bytes /
    time and its fraction of the HBM peak, for the plain form (batches one after
    another through the layer graph) and the batched form (the faster of the merged
    graph and the persistent launch); the forward + backward ratio for C5."""
    res = {}
    for name in args.table.split(","):
        cfg = gen.CONFIGS[name]
        N, L = cfg.n_neurons, cfg.n_layers
        idx, w, b = device_net(torch, gen, cfg, dev)
        y0 = device_inputs(torch, cfg, dev)
        trainable = cfg.ckpt_every > 0
        net = P.Net(idx, w, b, max_rows=cfg.rows, ckpt_every=cfg.ckpt_every,
                    flags=P.sdnn.SDNN_TRAINABLE if trainable else 0)
        off = [int(v) for v in gen.make_batches(cfg)] if cfg.n_batches > 1 else None
        o = {}
        net.forward(y0, batch_off=off, out=o, profile=True)
        prof = o["layer_rows"].cpu().numpy()
        alg, live = forward_bytes(prof, N, L), live_edges(prof, N, L)
        steps = 1 if L * N > 480 * 16384 else 3
        r = {"rows": cfg.rows, "N": N, "layers": L, "alive_head": [int(v) for v in prof[:4]],
             "alive_last": int(prof[L]), "alg_bytes": alg, "plan": net.plan}
        forms = [("plain", "graph")] + ([("merged", "graph_merged"), ("persistent", "persistent")] if off else
                                        [("persistent", "persistent")])
        forms = [f for f in forms if f[0] in args.table_forms.split(",")]
        for form, eng in forms:
            net.set_exec(eng)
            ms = time_forward(torch, net, y0, o, steps, 1, batch_off=off)
            r[form] = {"ms": round(ms, 3), "nominal_edges_per_s": cfg.rows * cfg.nnz / (ms / 1e3),
                       "live_edges_per_s": live / (ms / 1e3), "alg_GBps": round(alg / ms / 1e6, 1),
                       "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if off and "merged" in r and "persistent" in r:
            best = min(("merged", "persistent"), key=lambda k: r[k]["ms"])
            r["batched_best"] = best
            r["batched_over_plain"] = round(r["plain"]["ms"] / r[best]["ms"], 3)
        if trainable:
            net.set_exec("graph")
            ob = net.forward(y0, ckpt=True)
            dy = torch.randn_like(ob["y"]) * 1e-4
            for _ in range(2):
                net.forward(y0, ckpt=True, out=ob)
                net.backward(y0, ob["ckpt"], ob["nz_rows"], ob["n_nz"], dy)
            torch.cuda.synchronize()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            net.forward(y0, ckpt=True, out=ob)
            e[1].record()
            net.backward(y0, ob["ckpt"], ob["nz_rows"], ob["n_nz"], dy)
            e[2].record()
            torch.cuda.synchronize()
            r["fwd_ckpt_ms"] = round(e[0].elapsed_time(e[1]), 3)
            r["bwd_ms"] = round(e[1].elapsed_time(e[2]), 3)
            r["bwd_over_fwd"] = round(r["bwd_ms"] / r["fwd_ckpt_ms"], 3)
        res[name] = r
        log("table " + name, r)
        net.close()
        del idx, w, b, y0, o
        torch.cuda.empty_cache()
    return res


def bench_corun(args):
    """The paper's co-run throughput experiment: K copies of the inference program
    (paper_2004_10908_amd.corun: a batched forward of the whole input, then the
    category check of every batch on the host) start together on this machine;
    throughput = weighted speedup, the sum over copies of (time of the program
    alone) / (its time in the co-run)."""
    import subprocess
    import tempfile
    res = {}
    alone = None
    for k in [int(x) for x in args.corun.split(",")]:
        log(f"corun {k}: starting {k} program(s)")
        go = os.path.join(tempfile.mkdtemp(prefix="corun"), "go")
        cmd = [sys.executable, "-u", "-m", "paper_2004_10908_amd.corun", "--go", go] + args.corun_args.split()
        procs = [subprocess.Popen(cmd, cwd=ROOT, stdout=subprocess.PIPE, text=True) for _ in range(k)]
        for p in procs:
            line = p.stdout.readline()
            if line.strip() != "ready":
                raise RuntimeError(f"co-run program did not start: {line!r}")
        open(go, "w").close()
        outs = []
        for p in procs:
            out, _ = p.communicate(timeout=600)
            if p.returncode != 0:
                raise RuntimeError(f"co-run program failed ({p.returncode})")
            outs.append(json.loads(out.strip().splitlines()[-1]))
        times = [sum(o["seconds"]) / len(o["seconds"]) for o in outs]
        if alone is None:
            alone = times[0]
        res[str(k)] = {"seconds": [round(t, 4) for t in times], "weighted_speedup": round(sum(alone / t for t in times), 3),
                       "mismatches": sum(o["mismatches"] for o in outs), "alive_rows": outs[0]["alive_rows"]}
        log(f"corun {k}", res[str(k)])
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, np, gen, cfg, y0, off):
    """The FP64 oracle (plain C, OpenMP over rows) on this host: every host thread on
    a row sample of the same workload, and one thread on a smaller sample.  Its
    layers come from the same device generator as the GPU run's (generated before
    the timed part); it runs layers 0, 1, ... until its own count of alive rows is
    zero, after which the remaining layers receive no rows (every bias is <= 0) and
    add no work, exactly as the GPU's early exit."""
    import oracle
    import torch
    oracle.build()
    dev = y0.device
    rows = min(args.cpu_rows, cfg.rows)
    sample = y0[:rows].cpu().numpy()
    layers = []

    def grow(n):
        while len(layers) < min(n, cfg.n_layers):
            i_, w_, b_ = gen.make_layer_device(cfg, len(layers), dev)
            layers.append((i_.cpu().numpy(), w_.cpu().numpy(), b_.cpu().numpy()))

    threads = oracle.max_threads()
    n_layers = 2
    while True:
        grow(n_layers)
        t0 = time.perf_counter()
        res = oracle.forward(layers, sample, cfg.clamp, threads=threads)
        dt = time.perf_counter() - t0
        if res.alive_after[-1] == 0 or len(layers) == cfg.n_layers:
            break
        n_layers *= 2                               # not extinct yet: more layers, time again
    last = len(layers)
    rows1 = max(1, min(rows, args.cpu_rows1))
    t0 = time.perf_counter()
    oracle.forward(layers, sample[:rows1], cfg.clamp, threads=1)
    dt1 = time.perf_counter() - t0
    ext = (f"every row is dead after layer {last - 1} (the oracle's own count), so layers {last}..{cfg.n_layers - 1} "
           "receive no rows" if res.alive_after[-1] == 0 else "all layers")
    return {"value": rows * cfg.nnz / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {rows} of the {cfg.rows} {cfg.name} rows through layers 0..{last - 1}; {ext} "
                      f"(FP64, {threads} threads, {dt:.1f} s)",
            "seconds": round(dt, 2), "cpu_model": cpu_model(), "alive_after": [int(a) for a in res.alive_after],
            "single_thread": {"value": rows1 * cfg.nnz / dt1, "unit": "edges/s", "rows": rows1,
                              "seconds": round(dt1, 2)}}


if __name__ == "__main__":
    main()
