"""Chunked one-row-tile kernel (16384 < N <= 65536, N a multiple of 2048; plan
variant 6, rows staged in 2 or 4 chunks, paired neurons, a create-time bank order
per chunk) and its uniform-weight two-part form (variant 7: two parts per
workgroup, the default where every layer has one weight value and N % 4096 == 0):
every layer of their chains checked element by element against the oracle through
the chain's own activations, with several rows per row stream, and the same for the
wide-layer kernel on the same net; the engines bitwise equal to each other and
variant 7 equal to variant 6 output for output; a clamp the sums reach, a positive
bias (no compaction), empty and one-row calls; the autotuner leaving every output
unchanged."""
import numpy as np
import pytest
import torch

import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, check_layer_sync, forward_layers, host_layers, upload

pytestmark = pytest.mark.gpu

WIDE = (32, 1024, 3)


def default_variant(N, uniform=True):
    return 7 if uniform and (N // 2048) % 2 == 0 else 6


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


# N: 18432 (2 chunks, 9 parts: 3 row streams per XCD), 32768 (2 chunks of 16384, 16
# parts), 34816 (4 chunks of 8704, 17 parts: one stream per XCD, idle workgroups),
# 65536 (4 chunks of 16384, 32 parts, the C4 / S4 width).  Rows: several per stream.
@pytest.mark.parametrize("N,layers,rows,cfgname", [(18432, 4, 300, "S3"), (32768, 3, 200, "S4"),
                                                   (34816, 3, 150, "S4"), (65536, 4, 120, "S4"),
                                                   (65536, 3, 96, "C4")])
def test_rowc_chain_layer_sync(P, N, layers, rows, cfgname):
    cfg = gen.CONFIGS[cfgname].with_(n_neurons=N, n_layers=layers, rows=rows, seed=5 * N + rows)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    chunks = 2 if N <= 32768 else 4
    v0 = default_variant(N)
    assert net.plan["variant"] == v0 and net.plan["rows_per_tile"] == chunks, net.plan   # the default
    off = [0, rows // 5, rows // 5, rows // 5 + 1, rows]
    base = None
    for v in sorted({v0, 6}, reverse=True):
        net.set_plan(chunks, 1024, v)
        for m in ("persistent", "graph", "graph_merged", "eager"):
            o, nz, ys = forward_layers(net, y0, batch_off=off, mode=m)
            if base is None:
                prof = o["layer_rows"].cpu().numpy()
                print(f"N={N} rows={rows} variant {v} profile {prof.tolist()}", flush=True)
                check_chain(lay, cfg.clamp, ys, prof, nz, y0h)
                dead = np.setdiff1d(np.arange(rows), nz)
                assert (o["y"].cpu().numpy()[dead] == 0).all(), "dead rows must be exactly zero"
                base = (o["y"].clone(), ys)
            else:
                # the other engines, and variant 6 against 7: the same slots in the same
                # order with the same weight (padding adds w * 0 in 7 and 0 * y in 6)
                assert torch.equal(o["y"], base[0]), (v, m)
                assert all(np.array_equal(a, c) for a, c in zip(ys, base[1])), (v, m)
    # the wide-layer kernel on the same net (ascending order): also within the bounds
    net.set_plan(*WIDE)
    o, nz, ys = forward_layers(net, y0, batch_off=off, mode="persistent")
    check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
    net.close()


@pytest.mark.parametrize("weight", ["he", "const"])
def test_rowc_layer_sync_clamp_positive_bias_and_no_compaction(P, weight):
    """Layer by layer with a clamp the sums reach and a positive bias (compaction off:
    every row in every layer, the alive flags with no work list), on both chunk counts;
    He weights take variant 6 (the two-part form is refused), one weight value takes
    variant 7."""
    for N in (20480, 40960):
        layers, rows, clamp = 3, 200, 1.5
        cfg = gen.tiny_config(N, layers, rows, seed=N + 19, weight=weight, bias=0.05, clamp=clamp, row_density=True)
        idx, w, b = upload(cfg)
        lay = host_layers(idx, w, b)
        y0h = gen.make_inputs(cfg)
        net = P.Net(idx, w, b, max_rows=rows, clamp=clamp)
        assert net.plan["variant"] == default_variant(N, weight == "const"), net.plan
        if weight == "he":
            with pytest.raises(Exception):
                net.set_plan(2 if N <= 32768 else 4, 1024, 7)
        y = torch.from_numpy(y0h).to(DEV) * 1.5
        for l in range(layers):
            yn = net.layer(l, y)
            torch.cuda.synchronize()
            check_layer_sync(y.cpu().numpy(), yn.cpu().numpy(), lay[l], clamp)
            y = yn
        net.close()
        net = P.Net(idx, w, b, max_rows=rows, clamp=clamp, ckpt_every=1)
        for m in ("persistent", "graph"):
            o, nz, ys = forward_layers(net, torch.from_numpy(y0h).to(DEV), mode=m)
            check_chain(lay, clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h, compact=False)
        net.close()


def test_rowc_empty_and_single_row(P):
    N = 65536
    cfg = gen.CONFIGS["S4"].with_(n_neurons=N, n_layers=3, rows=5, seed=31)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    net = P.Net(idx, w, b, max_rows=5, ckpt_every=1)
    assert net.plan["variant"] == 7, net.plan
    for v in (7, 6):
        net.set_plan(4, 1024, v)
        for rows in (1, 0, 5):
            y0 = torch.from_numpy(y0h[:rows]).to(DEV)
            for m in ("persistent", "graph"):
                o, nz, ys = forward_layers(net, y0, mode=m)
                if rows:
                    check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h[:rows])
                else:
                    assert len(nz) == 0
    net.close()


def test_rowc_family_autotune_on_the_workload(P):
    """At 65536 neurons with one weight value the two-part kernel is alone in its
    family: tuning on the workload's rows keeps it and leaves every output bitwise
    unchanged."""
    N, rows = 65536, 256
    cfg = gen.CONFIGS["S4"].with_(n_neurons=N, n_layers=2, rows=rows, seed=37)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows)
    a = net.forward(y0, batch_off=[0, 100, rows])
    torch.cuda.synchronize()
    plan = net.tune(rows, y_sample=y0)
    print("tuned plan", plan, flush=True)
    assert plan["tuned_us"] > 0 and plan["variant"] == 7
    c = net.forward(y0, batch_off=[0, 100, rows])
    torch.cuda.synchronize()
    assert torch.equal(a["y"], c["y"])
    net.close()


def test_two_part_needs_one_weight_in_every_layer(P):
    """One weight value in every layer but one (a single weight of the last layer
    changed): the two-part form is refused, variant 6 serves the net, and its chain
    still matches the oracle; with the weight restored the two-part form is the
    default again and gives the same outputs."""
    N, layers, rows = 20480, 3, 120
    cfg = gen.CONFIGS["S4"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=97)
    idx, w, b = upload(cfg)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    w_odd = w.clone()
    w_odd[layers - 1, 123, 7] *= 1.5
    lay = host_layers(idx, w_odd, b)
    net = P.Net(idx, w_odd, b, max_rows=rows, ckpt_every=1)
    assert net.plan["variant"] == 6, net.plan
    with pytest.raises(Exception):
        net.set_plan(2, 1024, 7)
    o, nz, ys = forward_layers(net, y0, mode="persistent")
    check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
    net.close()
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    assert net.plan["variant"] == 7, net.plan
    a = forward_layers(net, y0, mode="persistent")[0]["y"].clone()
    net.set_plan(2, 1024, 6)
    c = forward_layers(net, y0, mode="persistent")[0]["y"]
    assert torch.equal(a, c)
    net.close()
