"""Wide-layer kernels (rows packed T per tile as [N][T], one T*4-byte gather per
slot): parity with the oracle on shapes the scheduled kernel cannot take, and
every variant bitwise equal to the others and to the LDS-staged kernel, which
sums in the same order."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, check_layer_sync, forward_layers, host_layers, run_forward, upload

pytestmark = pytest.mark.gpu

MODES = ["eager", "graph", "persistent", "graph_merged", "auto"]   # auto: persistent on the wide kernels
WIDE = [(T, NT, 3) for T in (8, 16, 32) for NT in (256, 512)] + [(16, 1024, 3), (32, 1024, 3)]


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


# N = 6000: no 8-row LDS tile fits and the last neuron chunk is partial;
# 16384 and 65536: the widths of the two batched configurations.  Row counts leave
# a partial last tile for every T.
@pytest.mark.parametrize("N,layers,rows", [(6000, 6, 300), (16384, 4, 77), (65536, 3, 41)])
def test_wide_forward_matches_oracle(P, N, layers, rows):
    cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=N + rows)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    if N > 16384:
        # a row exceeds one 64 KB LDS buffer: chunked one-row tiles, two parts per
        # workgroup (one weight value, 32 parts)
        assert net.plan["variant"] == 7, net.plan
    else:
        assert net.plan["variant"] == 5, net.plan    # one-row tiles with resident weights
    net.set_plan(32, 1024, 3)
    base = None
    for m in MODES:
        o, nz, ys = forward_layers(net, y0, mode=m)
        if base is None:
            check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
            base = o["y"].clone()
        else:
            assert torch.equal(o["y"], base), m
    net.close()


# Several tiles per workgroup (one-row-tile kernel at 16384 neurons, and the wide
# kernel on the same net) and per XCD tile stream (chunked one-row-tile kernel and
# wide kernel at 65536 neurons), every layer of the chain checked element by element
# through its own activations.
@pytest.mark.parametrize("N,layers,rows,plan", [(16384, 8, 2400, None), (16384, 6, 2400, (32, 1024, 3)),
                                                (65536, 6, 1200, None), (65536, 4, 1200, (32, 1024, 3))])
def test_wide_chain_layer_sync_multi_tile(P, N, layers, rows, plan):
    cfg = gen.CONFIGS["S3"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=N + rows + layers)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    if plan is not None:
        net.set_plan(*plan)
    base = None
    for m in ("persistent", "graph_merged"):
        o, nz, ys = forward_layers(net, y0, batch_off=[0, rows // 3, rows // 3 + 1, rows], mode=m)
        if base is None:
            prof = o["layer_rows"].cpu().numpy()
            check_chain(lay, cfg.clamp, ys, prof, nz, y0h)
            assert prof[layers - 1] > 0, prof
            base = ys
        else:
            assert all(np.array_equal(a, c) for a, c in zip(ys, base)), m
    net.close()


def test_wide_variants_bitwise_equal(P):
    """Every (T, NT) of the wide kernels, in the graph chain over uneven, empty and
    one-row batches and in the persistent chain, against the 4-row LDS-staged kernel."""
    N, layers, rows = 6000, 5, 333
    cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=91)
    idx, w, b = upload(cfg)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    off = [0, 40, 40, 41, 200, rows]
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    base = None
    for T, NT, v in [(4, 512, 0), (1, 1024, 4)] + WIDE:
        plan = net.set_plan(T, NT, v)
        assert (plan["rows_per_tile"], plan["threads"], plan["variant"]) == (T, NT, v)
        for m in ("graph", "persistent"):
            o, nz, ys = forward_layers(net, y0, batch_off=off, mode=m)
            if base is None:
                check_chain(host_layers(idx, w, b), cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
                base = (o["y"].clone(), list(nz))
            else:
                assert torch.equal(o["y"], base[0]), (T, NT, v, m)
                assert list(nz) == base[1], (T, NT, v, m)
    net.close()


@pytest.mark.parametrize("T,NT,v", WIDE + [(1, 1024, 4), (1, 1024, 5)])
def test_wide_layer_sync_clamp_and_positive_bias(P, T, NT, v):
    """Layer by layer with a clamp the sums reach and a positive bias (compaction
    off), then the whole forward in every mode."""
    N, layers, rows, clamp = 7000, 3, 45, 1.5
    cfg = gen.tiny_config(N, layers, rows, seed=T * 1000 + NT + v, weight="he", bias=0.05, clamp=clamp,
                          row_density=True)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=rows, clamp=clamp)
    net.set_plan(T, NT, v)
    y0h = gen.make_inputs(cfg)
    y = torch.from_numpy(y0h).to(DEV) * 1.5
    lay = host_layers(idx, w, b)
    for l in range(layers):
        yn = net.layer(l, y)
        torch.cuda.synchronize()
        check_layer_sync(y.cpu().numpy(), yn.cpu().numpy(), lay[l], clamp)
        y = yn
    net.close()
    net = P.Net(idx, w, b, max_rows=rows, clamp=clamp, ckpt_every=1)
    net.set_plan(T, NT, v)
    for m in MODES:
        o, nz, ys = forward_layers(net, torch.from_numpy(y0h).to(DEV), mode=m)
        check_chain(lay, clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h, compact=False)
    net.close()


def test_set_plan_errors(P):
    cfg = gen.CONFIGS["S2"].with_(n_neurons=6000, n_layers=2, rows=20, seed=5)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=20)
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.set_plan(12, 256, 3)                 # no such tile
    with pytest.raises(P.SdnnError, match="EUNSUPPORTED"):
        net.set_plan(4, 512, 2)                  # no schedule for this shape
    with pytest.raises(P.SdnnError, match="EUNSUPPORTED"):
        net.set_plan(16, 512, 0)                 # 16 rows of 6000 floats exceed the LDS
    net.close()
    cfg = gen.CONFIGS["S2"].with_(n_neurons=4096, n_layers=2, rows=20, seed=6)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=20)
    assert net.plan["variant"] == 2
    with pytest.raises(P.SdnnError, match="EUNSUPPORTED"):
        net.set_plan(16, 256, 3)                 # no packed buffer in this net's workspace
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.layer(0, torch.zeros(21, 4096, device=DEV))   # more rows than max_rows
    net.close()
