"""Batches over several streams, issued directly or captured as one graph: the same
outputs as the single-stream forward, bit for bit, and the oracle's row set."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, forward_layers, host_layers, run_forward, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


# N = 2048: scheduled kernels; N = 1000: the streamed-weight kernels
@pytest.mark.parametrize("N,layers,rows", [(2048, 12, 1200), (1000, 9, 700)])
def test_streams_equal_single_stream(P, N, layers, rows):
    from paper_2004_10908_amd.streams import StreamForward
    cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=N + layers)
    idx, w, b = upload(cfg)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    off = [0, 150, 151, 151, 480, 700 if rows > 700 else rows - 1, rows - 1, rows]   # uneven, empty, 1-row
    off = sorted(min(v, rows) for v in off)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=1)
    o, nz, ys = forward_layers(net, y0, batch_off=off, mode="graph")
    check_chain(host_layers(idx, w, b), cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
    base = o["y"].clone()
    net.close()
    for k in (1, 2, 3):
        sf = StreamForward(idx, w, b, off, k)
        y = torch.full_like(y0, float("nan"))
        sf.run(y0, y)
        torch.cuda.synchronize()
        assert torch.equal(y, base), k
        assert np.array_equal(sf.nz_rows().cpu().numpy(), np.asarray(nz, np.int64)), k
        sf.close()


def test_captured_streams_replay_equal(P):
    """A captured multi-stream forward replayed several times, with other work between
    the replays, reproduces the single-stream result every time."""
    from paper_2004_10908_amd.streams import StreamForward
    cfg = gen.CONFIGS["S2"].with_(n_neurons=1024, n_layers=10, rows=900, seed=77)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    off = [0, 100, 350, 351, 600, 900]
    net = P.Net(idx, w, b, max_rows=cfg.rows)
    o, nz = run_forward(net, y0, batch_off=off, mode="graph")
    base = o["y"].clone()
    for k in (2, 4):
        sf = StreamForward(idx, w, b, off, k, capture=True)
        y = torch.zeros_like(y0)
        for rep in range(3):
            y.fill_(float("nan"))
            sf.run(y0, y)
            torch.cuda.synchronize()
            assert torch.equal(y, base), (k, rep)
            assert torch.equal(sf.nz_rows().cpu(), torch.from_numpy(np.asarray(nz)).long()), (k, rep)
            # eager work of the program between replays
            run_forward(net, y0, batch_off=off, mode="eager")
            torch.cuda.synchronize()
        sf.close()
    net.close()
