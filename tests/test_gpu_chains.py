"""Long persistent chains: hundreds of grid barriers in one cooperative launch, with
each layer's arguments read again from the kernel-argument segment and every
layer's rows produced by workgroups on other XCDs (the barrier's release / acquire
is what makes them visible).  Every layer of the chain is checked element by element
against the oracle through the chain's own activations, and the persistent launch
is bitwise equal to the explicit graph (layer by layer, and in its row profile),
for the resident-weight kernel families."""
import numpy as np
import pytest
import torch

import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, forward_layers, host_layers, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


def _chain_vs_graph(P, cfg, variant, plan=None, batch_off=None):
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=cfg.rows, ckpt_every=1)
    if plan is not None:
        net.set_plan(*plan)
    assert net.plan["variant"] == variant, net.plan
    base = None
    for m in ("persistent", "graph"):
        o, nz, ys = forward_layers(net, y0, batch_off=batch_off, mode=m)
        prof = o["layer_rows"].cpu().numpy()
        if base is None:
            check_chain(lay, cfg.clamp, ys, prof, nz, y0h)
            print(f"{cfg.name}: alive after layers 0, L/2, L: {prof[1]}, {prof[cfg.n_layers // 2]}, "
                  f"{prof[cfg.n_layers]}", flush=True)
            assert prof[cfg.n_layers] > 0, "rows must stay alive to the last layer"
            base = (ys, prof)
        else:
            assert np.array_equal(prof, base[1]), m
            assert all(np.array_equal(a, c) for a, c in zip(ys, base[0])), m
    net.close()


def test_long_chain_scheduled(P):
    # the scheduled kernel (plan variant 2) over 160 layers of a sustained net: 160 grid
    # barriers, four parts per tile (N = 4096), rows dying at different layers
    cfg = gen.CONFIGS["S2"].with_(n_layers=160, rows=400, seed=71)
    _chain_vs_graph(P, cfg, 2, batch_off=[0, 150, 151, 300, 400])


def test_long_chain_one_row_tile(P):
    # the one-row-tile kernel in its bank-scheduled order (variant 5) over 64 layers
    cfg = gen.CONFIGS["S3"].with_(n_neurons=8192, n_layers=64, rows=240, seed=73)
    _chain_vs_graph(P, cfg, 5)


def test_long_chain_chunked(P):
    # the chunked one-row-tile kernel (variant 6, two chunks) over 32 layers
    cfg = gen.CONFIGS["S3"].with_(n_neurons=18432, n_layers=32, rows=160, seed=79)
    _chain_vs_graph(P, cfg, 6)


def test_long_chain_two_part(P):
    # the uniform-weight two-part chunked kernel (variant 7, two chunks, 12 parts of
    # 2048 in 6 workgroup parts) over 32 layers
    cfg = gen.CONFIGS["S3"].with_(n_neurons=24576, n_layers=32, rows=160, seed=83)
    _chain_vs_graph(P, cfg, 7)
