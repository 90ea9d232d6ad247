"""One-row-tile resident-weight kernel (2048 < N <= 16384; plan variant 5 with the
bank-scheduled slot order, the default, and variant 4 in ascending order): every
layer of its chain checked element by element against the oracle through the
chain's own activations, with several rows per tile stream, partial parts and
partial row copies; variant 4 bitwise equal to the LDS-staged kernel, which sums
in the same order; dead rows cleared; the engines equal to each other."""
import numpy as np
import pytest
import torch

import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, check_layer_sync, forward_layers, host_layers, upload

pytestmark = pytest.mark.gpu

ROW = (1, 1024, 4)


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


# N: 2052 (two parts, the second of 4 neurons), 6000 (three parts, a partial last
# part), 10000 (a partial last 1 KB row copy), 16384 (eight full parts, the C3 / S3
# width).  Rows: several tiles per tile stream (256 / G streams of one row each).
@pytest.mark.parametrize("N,layers,rows,cfgname", [(2052, 6, 700, "S2"), (6000, 6, 500, "S2"),
                                                   (10000, 5, 450, "S3"), (16384, 8, 1100, "S3"),
                                                   (16384, 4, 300, "C3")])
def test_row_chain_layer_sync(P, N, layers, rows, cfgname):
    cfg = gen.CONFIGS[cfgname].with_(n_neurons=N, n_layers=layers, rows=rows, seed=3 * N + rows)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    assert net.plan["variant"] == 5, net.plan        # the default for these widths
    off = [0, rows // 5, rows // 5, rows // 5 + 1, rows]
    for plan in ((1, 1024, 5), (1, 1024, 4)):
        net.set_plan(*plan)
        base = None
        for m in ("persistent", "graph", "graph_merged", "eager"):
            o, nz, ys = forward_layers(net, y0, batch_off=off, mode=m)
            if base is None:
                prof = o["layer_rows"].cpu().numpy()
                print(f"plan {plan} N={N} rows={rows} profile {prof.tolist()}", flush=True)
                check_chain(lay, cfg.clamp, ys, prof, nz, y0h)
                dead = np.setdiff1d(np.arange(rows), nz)
                assert (o["y"].cpu().numpy()[dead] == 0).all(), "dead rows must be exactly zero"
                base = (o["y"].clone(), ys)
            else:
                assert torch.equal(o["y"], base[0]), (plan, m)
                assert all(np.array_equal(a, c) for a, c in zip(ys, base[1])), (plan, m)
    # the LDS-staged streamed-weight kernel sums in ascending order like variant 4: bitwise equal
    net.set_plan(2, 1024, 0)
    o, nz, ys = forward_layers(net, y0, batch_off=off, mode="graph")
    assert torch.equal(o["y"], base[0])
    net.close()


def test_row_layer_sync_clamp_positive_bias_and_no_compaction(P):
    """Layer by layer with a clamp the sums reach and a positive bias (compaction
    off: every row in every layer, the alive flags with no work list)."""
    N, layers, rows, clamp = 7000, 3, 300, 1.5
    cfg = gen.tiny_config(N, layers, rows, seed=17, weight="he", bias=0.05, clamp=clamp, row_density=True)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    net = P.Net(idx, w, b, max_rows=rows, clamp=clamp)
    assert net.plan["variant"] == 5, net.plan
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


def test_row_empty_and_single_row(P):
    N = 16384
    cfg = gen.CONFIGS["S3"].with_(n_neurons=N, n_layers=3, rows=5, seed=23)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    net = P.Net(idx, w, b, max_rows=5, ckpt_every=1)
    for rows in (1, 0, 5):
        y0 = torch.from_numpy(y0h[:rows]).to(DEV)
        for m in ("persistent", "graph"):
            o, nz, ys = forward_layers(net, y0, mode=m)
            if rows:
                check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h[:rows])
            else:
                assert len(nz) == 0
    net.close()


def test_row_family_autotune_on_the_workload(P):
    """At 16384 neurons the tuner chooses within a family of kernels that sum in the
    same order: the one-row-tile kernel in ascending order, the LDS-staged and the
    wide-layer kernels (or the bank-scheduled one-row-tile kernel alone).  Timing
    them on the workload's rows picks a plan and leaves every output bitwise
    unchanged."""
    N, rows = 16384, 600
    cfg = gen.CONFIGS["S3"].with_(n_neurons=N, n_layers=3, rows=rows, seed=29)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows)
    for plan0 in ((1, 1024, 5), (1, 1024, 4)):
        net.set_plan(*plan0)
        a = net.forward(y0, batch_off=[0, 250, rows])
        torch.cuda.synchronize()
        plan = net.tune(rows, y_sample=y0)
        print("tuned plan", plan0, "->", plan, flush=True)
        assert plan["tuned_us"] > 0
        assert (plan["variant"] == 5) == (plan0[2] == 5)
        c = net.forward(y0, batch_off=[0, 250, rows])
        torch.cuda.synchronize()
        assert torch.equal(a["y"], c["y"])
    net.close()
