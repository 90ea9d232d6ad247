"""Forward with the parameters in pinned host memory, streamed through two device
slots: equal, bit for bit, to the same kernels over resident parameters, and to the
oracle's result."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_end_to_end, check_layer_sync, host_layers, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


@pytest.mark.parametrize("N,layers,rows,slots", [(1024, 9, 333, 2), (2048, 6, 130, 3), (1024, 1, 50, 2)])
def test_streamed_equals_resident(P, N, layers, rows, slots):
    from paper_2004_10908_amd.streamed import StreamedForward
    cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=N + layers)
    idx, w, b = upload(cfg)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    lay = host_layers(idx, w, b)
    # resident parameters, same kernel family, layer by layer over all rows, each layer
    # checked against the oracle fed the same inputs
    net = P.Net(idx, w, b, max_rows=rows, flags=P.sdnn.SDNN_NO_SCHEDULE | P.sdnn.SDNN_NO_COMPACTION)
    assert net.plan["variant"] != 2
    y = y0
    ties = set()
    for l in range(layers):
        yn = net.layer(l, y)
        torch.cuda.synchronize()
        ties |= check_layer_sync(y.cpu().numpy(), yn.cpu().numpy(), lay[l], cfg.clamp)
        y = yn
    base = y.clone()
    ref = oracle.forward(lay, y0h, cfg.clamp)
    net.close()
    sf = StreamedForward(idx.cpu().pin_memory(), w.cpu().pin_memory(), b.cpu().pin_memory(), rows, slots=slots)
    out = torch.full_like(y0, float("nan"))
    for rep in range(2):                      # the second run reuses slots and events
        out.fill_(float("nan"))
        sf.run(y0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, base), rep
    nz = torch.nonzero((out != 0).any(dim=1)).flatten().cpu().numpy().astype(np.int32)
    check_end_to_end(out.cpu().numpy(), nz, ref, ties)
    sf.close()


def test_streamed_rejects_unpinned_and_positive_bias(P):
    from paper_2004_10908_amd.streamed import StreamedForward
    cfg = gen.tiny_config(256, 2, 8, seed=3)
    idx, w, b = upload(cfg)
    with pytest.raises(ValueError):
        StreamedForward(idx.cpu(), w.cpu(), b.cpu(), 8)
    with pytest.raises(ValueError):
        StreamedForward(idx.cpu().pin_memory(), w.cpu().pin_memory(), (b.cpu() + 1.0).pin_memory(), 8)
