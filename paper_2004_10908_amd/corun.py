"""One inference program for the co-run throughput experiment.

The paper measures the throughput of several copies of its inference program
running at once on one machine (section "Large Sparse Neural Network Inference":
co-running inference on 1920-layer nets, throughput as weighted speedup).  This
program is one such copy: it draws a sustained net and its inputs (seeded, on the
device), derives the truth categories of every batch from one forward per batch,
then ``--runs`` times runs the whole input as one batched forward (every batch in
one launch sequence, the merged graph), brings the nonzero-row ids back to the
host and checks them batch by batch against the truth categories, and prints one
JSON line with the time of each run.  With ``--go FILE`` it prints "ready" after
its set-up and waits for FILE to exist before the timed runs, so that a driver can
start several copies together.

The forward runs as the merged graph of ordinary kernels, not as the persistent
cooperative kernel: the persistent kernel's grid barrier assumes that its whole
grid is resident, which another process's kernels on the same GPU do not
guarantee.

    python -m paper_2004_10908_amd.corun --neurons 4096 --layers 1920 --rows 20000
"""
from __future__ import annotations

import argparse
import json
import os
import time


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--neurons", type=int, default=4096)
    ap.add_argument("--layers", type=int, default=1920)
    ap.add_argument("--rows", type=int, default=20000)
    ap.add_argument("--batches", type=int, default=20)
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--bias", type=float, default=-0.35)
    ap.add_argument("--runs", type=int, default=3)
    ap.add_argument("--go", default="", help="wait for this file before the timed runs")
    return ap.parse_args(argv)


def main(argv=None):
    args = parse(argv)
    import numpy as np
    import torch

    import sdnn_inputs as gen
    from . import sdnn as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # a sustained net (per-row input density U(0.1, 0.5)): rows stay alive through the layers
    cfg = gen.NetConfig("corun", args.neurons, args.layers, args.rows, args.seed, bias=args.bias,
                        row_density=True, n_batches=args.batches, batch_lo=max(1, args.rows // (4 * args.batches)),
                        batch_hi=max(2, 4 * args.rows // args.batches))
    N, L, R = cfg.n_neurons, cfg.n_layers, cfg.rows
    idx = torch.empty((L, N, 32), dtype=torch.int32, device=dev)
    w = torch.empty((L, N, 32), dtype=torch.float32, device=dev)
    b = torch.empty((L, N), dtype=torch.float32, device=dev)
    for l in range(L):
        i_, w_, b_ = gen.make_layer_device(cfg, l, dev)
        idx[l].copy_(i_)
        w[l].copy_(w_)
        b[l].copy_(b_)
    g = torch.Generator(device=dev)
    g.manual_seed(cfg.seed * 7919 + 1)
    p = torch.rand((R, 1), generator=g, device=dev) * 0.4 + 0.1
    y0 = (torch.rand((R, N), generator=g, device=dev) < p).float()
    off = [int(x) for x in gen.make_batches(cfg)]
    nb = len(off) - 1
    big = max(off[i + 1] - off[i] for i in range(nb))
    # truth categories: the nonzero rows of one forward per batch
    single = S.Net(idx, w, b, max_rows=big, exec_mode="graph")
    truth = []
    for bi in range(nb):
        r0, r1 = off[bi], off[bi + 1]
        if r1 == r0:
            truth.append(np.zeros(0, np.int64))
            continue
        o = single.forward(y0[r0:r1].contiguous())
        n = int(o["n_nz"].item())
        truth.append(o["nz_rows"][:n].cpu().numpy().astype(np.int64) + r0)
    single.close()
    net = S.Net(idx, w, b, max_rows=R, exec_mode="graph_merged")
    out = net.forward(y0, batch_off=off)      # warm-up (instantiates the merged graph)
    torch.cuda.synchronize()
    if args.go:
        print("ready", flush=True)
        while not os.path.exists(args.go):
            time.sleep(0.01)
    secs, bad = [], 0
    for _ in range(args.runs):
        t0 = time.perf_counter()
        net.forward(y0, batch_off=off, out=out)
        n = int(out["n_nz"].item())               # synchronizes the stream
        got = out["nz_rows"][:n].cpu().numpy().astype(np.int64)
        # the golden-reference check: nonzero rows of each batch against its truth categories
        for bi in range(nb):
            mine = got[(got >= off[bi]) & (got < off[bi + 1])]
            bad += int(len(np.setxor1d(mine, truth[bi])))
        secs.append(time.perf_counter() - t0)
    res = {"seconds": secs, "mismatches": bad, "batches": nb, "rows": R, "neurons": N, "layers": L,
           "alive_rows": int(sum(len(t) for t in truth))}
    net.close()
    torch.cuda.synchronize()
    S.unload()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
