"""GPU parity of the forward pass (C ABI via the ctypes binding) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import (DEV, check_chain, check_end_to_end, check_layer_sync, forward_layers, host_layers,
                            run_forward, upload)

pytestmark = pytest.mark.gpu

MODES = ["eager", "graph", "persistent", "graph_merged"]


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


def _net(P, idx, w, b, rows, **kw):
    return P.Net(idx, w, b, max_rows=rows, **kw)


@pytest.mark.parametrize("N,rows,weight,bias,clamp", [
    (32, 1, "he", 0.1, 32.0), (64, 7, "he", -0.05, 1.5), (96, 37, "uniform", -0.3, 32.0),
    (1000, 129, "he", 0.0, 2.0), (4096, 19, "const", -0.35, 32.0),
    # two parts and a last 64-id block of 16 ids (partial block copies and transposes)
    (1040, 23, "he", -0.1, 32.0)])
def test_layer_sync_small_nets(P, N, rows, weight, bias, clamp):
    cfg = gen.tiny_config(N, 4, rows, seed=N + rows, weight=weight, bias=bias, clamp=clamp, row_density=True)
    idx, w, b = upload(cfg)
    net = _net(P, idx, w, b, rows, clamp=clamp)
    y = torch.from_numpy(gen.make_inputs(cfg)).to(DEV) * 1.5
    lay = host_layers(idx, w, b)
    for l in range(cfg.n_layers):
        yn = net.layer(l, y)
        torch.cuda.synchronize()
        check_layer_sync(y.cpu().numpy(), yn.cpu().numpy(), lay[l], clamp)
        y = yn


def test_c1_all_modes_match_oracle_and_each_other(P):
    cfg = gen.CONFIGS["C1"]
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    outs = {}
    for flags in (0, P.sdnn.SDNN_NO_COMPACTION):
        net = _net(P, idx, w, b, cfg.rows, flags=flags, ckpt_every=1)
        for m in MODES:
            o, nz, ys = forward_layers(net, y0, mode=m)
            check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h, compact=flags == 0)
            outs[(flags, m)] = o["y"].clone()
        net.close()
    base = outs[(0, "graph")]
    for k, v in outs.items():
        assert torch.equal(v, base), k


def test_sustained_companion_small(P):
    """Row densities U(0.1, 0.5) keep rows alive through every layer."""
    cfg = gen.CONFIGS["S2"].with_(n_neurons=1024, n_layers=40, rows=333)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    net = _net(P, idx, w, b, cfg.rows, ckpt_every=1)
    y0 = torch.from_numpy(y0h).to(DEV)
    for m in ("graph", "persistent"):
        o, nz, ys = forward_layers(net, y0, mode=m)
        assert len(nz) > 50
        check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)


def test_batched_forms_equal_plain(P):
    cfg = gen.CONFIGS["S2"].with_(n_neurons=2048, n_layers=24, rows=1500)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    off = [0, 0, 311, 312, 900, 900, 1499, 1500]        # uneven, with empty and 1-row batches
    net = _net(P, idx, w, b, cfg.rows, ckpt_every=1)
    base = None
    for m in MODES:
        o, nz, ys = forward_layers(net, y0, batch_off=off, mode=m)
        if base is None:
            check_chain(lay, cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h)
            base = o["y"].clone()
            base_ys = ys
        assert torch.equal(o["y"], base), m
        assert all(np.array_equal(a, c) for a, c in zip(ys, base_ys)), m
    o, nz = run_forward(net, y0, batch_off=None, mode="graph")
    assert torch.equal(o["y"], base)


# Multi-tile pipelines: every one of the scheduled kernel's 256 / G tile streams runs
# several 4-row tiles (next-tile copies, buffer toggle, the deferred liveness words,
# the lockstep), checked element by element on every layer through the chain's own
# activations.  He weights with a negative bias make rows die at different layers with
# mixed-sign sums (a row alive overall can have an all-zero slice of one part).
@pytest.mark.parametrize("N,rows,layers,weight,bias", [
    (1024, 4000, 10, "he", -0.05),       # G = 1: 256 streams, ~4 tiles each
    (2048, 2600, 10, "he", -0.05),       # G = 2: 128 streams, ~5 tiles each
    (4096, 4000, 16, "he", -0.05),       # G = 4: 64 streams, ~16 tiles each
    (4096, 3000, 24, "const", -0.35),    # the C2 net with per-row densities (S2), rows saturate at 32
])
def test_chain_layer_sync_multi_tile(P, N, rows, layers, weight, bias):
    if weight == "const":
        cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=layers, rows=rows, seed=N + rows)
    else:
        cfg = gen.tiny_config(N, layers, rows, seed=N + rows, weight=weight, bias=bias, row_density=True)
    idx, w, b = upload(cfg)
    lay = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = _net(P, idx, w, b, rows, ckpt_every=1)
    assert net.plan["variant"] == 2, net.plan
    base = None
    for m in ("persistent", "graph"):
        o, nz, ys = forward_layers(net, y0, mode=m)
        prof = o["layer_rows"].cpu().numpy()
        if base is None:
            ties = check_chain(lay, cfg.clamp, ys, prof, nz, y0h)
            print(f"N={N} rows={rows}: alive per layer {prof.tolist()}, tie-flip rows {ties}")
            assert prof[layers // 2] > 0          # rows still alive half-way: the deep layers are exercised
            base = ys
        else:
            assert all(np.array_equal(a, c) for a, c in zip(ys, base)), m
    net.close()


def test_positive_bias_turns_compaction_off_and_matches(P):
    cfg = gen.tiny_config(256, 6, 40, seed=3, weight="he", bias=0.02, row_density=True)
    idx, w, b = upload(cfg)
    b[2, 5] = 0.5
    y0h = gen.make_inputs(cfg)
    y0h[3] = 0.0
    net = _net(P, idx, w, b, cfg.rows, ckpt_every=1)
    o, nz, ys = forward_layers(net, torch.from_numpy(y0h).to(DEV), mode="graph")
    check_chain(host_layers(idx, w, b), cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y0h, compact=False)
    assert (o["layer_rows"].cpu().numpy()[:cfg.n_layers] == cfg.rows).all()   # no compaction


def test_empty_and_single_row_calls(P):
    cfg = gen.tiny_config(128, 3, 5, seed=9, weight="he", bias=-0.01)
    idx, w, b = upload(cfg)
    net = _net(P, idx, w, b, 5, ckpt_every=1)
    y0 = torch.zeros(0, 128, device=DEV)
    o = net.forward(y0, profile=True)
    torch.cuda.synchronize()
    assert int(o["n_nz"].item()) == 0 and (o["layer_rows"].cpu().numpy() == 0).all()
    y1h = gen.make_inputs(cfg.with_(rows=1))
    for m in MODES:
        o, nz, ys = forward_layers(net, torch.from_numpy(y1h).to(DEV), mode=m)
        check_chain(host_layers(idx, w, b), cfg.clamp, ys, o["layer_rows"].cpu().numpy(), nz, y1h)


def test_argument_errors(P):
    cfg = gen.tiny_config(128, 3, 8, seed=2)
    idx, w, b = upload(cfg)
    net = _net(P, idx, w, b, 8)
    y0 = torch.ones(8, 128, device=DEV)
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.forward(torch.ones(9, 128, device=DEV))                      # rows > max_rows
    buf = torch.zeros(16 * 128, device=DEV)
    o = {"y": buf[: 8 * 128].view(8, 128), "nz_rows": torch.empty(8, dtype=torch.int32, device=DEV),
         "n_nz": torch.empty(1, dtype=torch.int32, device=DEV), "ckpt": None, "layer_rows": None}
    with pytest.raises(P.SdnnError, match="overlap"):
        P.sdnn_forward(net.h, buf[4 * 128: 12 * 128].view(8, 128), 8, None, 1, o["y"], o["nz_rows"], o["n_nz"])
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.forward(y0, batch_off=[0, 5, 4, 8])                           # decreasing offsets
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.forward(y0, batch_off=[1, 8])
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.forward(y0, ckpt=True)                                         # net has no checkpoint stride
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.set_exec(9)
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.layer(3, y0)
    d = P.make_desc(128, 3, 8)
    small = torch.empty(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(P.SdnnError, match="ENOMEM"):
        P.sdnn_create(d, idx, w, b, small)
    ws = torch.empty(P.sdnn_workspace_size(d) + 512, dtype=torch.uint8, device=DEV)
    with pytest.raises(P.SdnnError, match="aligned"):
        P.sdnn_create(d, idx, w, b, ws[8:], P.sdnn_workspace_size(d))


def test_debug_checks_reject_bad_patterns(P):
    cfg = gen.tiny_config(128, 2, 4, seed=4)
    idx, w, b = upload(cfg)
    P.Net(idx, w, b, max_rows=4, flags=P.sdnn.SDNN_DEBUG_CHECKS).close()
    bad = idx.clone()
    bad[1, 7, 3] = 128                                                      # out of range
    with pytest.raises(P.SdnnError, match="out of range"):
        P.Net(bad, w, b, max_rows=4, flags=P.sdnn.SDNN_DEBUG_CHECKS)
    bad = idx.clone()
    bad[0, 2, 5] = bad[0, 2, 4]                                             # duplicate id
    with pytest.raises(P.SdnnError, match="ascending"):
        P.Net(bad, w, b, max_rows=4, flags=P.sdnn.SDNN_DEBUG_CHECKS)


def test_autotune_keeps_results(P):
    cfg = gen.CONFIGS["S2"].with_(n_neurons=1024, n_layers=6, rows=600)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = P.Net(idx, w, b, max_rows=600)
    a, _ = run_forward(net, y0, mode="graph")
    plan = net.tune(600)
    assert plan["tuned_us"] > 0
    c, _ = run_forward(net, y0, mode="graph")
    assert torch.equal(a["y"], c["y"])
    plan = net.tune(600, y_sample=y0)                  # on the workload's own rows
    assert plan["tuned_us"] > 0
    c, _ = run_forward(net, y0, mode="graph")
    assert torch.equal(a["y"], c["y"])
    with pytest.raises(P.SdnnError, match="EINVAL"):
        P.sdnn.sdnn_tune(net.h, 601, torch.zeros(601, 1024, device=DEV))


@pytest.mark.slow
def test_c2_full_size(P):
    """60000 x 4096 x 480: the whole net runs; the oracle checks the first layers
    over every row (every row is dead by layer 2) and layer-0 values on a sample."""
    cfg = gen.CONFIGS["C2"]
    idx, w, b = upload(cfg, exact_layers=3)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=cfg.rows)
    o, nz = run_forward(net, y0, mode="graph")
    prof = o["layer_rows"].cpu().numpy()
    ref = oracle.forward(host_layers(idx, w, b, 0, 3), y0h, cfg.clamp)
    assert ref.alive_after[-1] == 0
    assert list(prof[1:4]) == ref.alive_after and (prof[4:] == 0).all()
    assert len(nz) == 0 and not torch.any(o["y"])
    o2, _ = run_forward(net, y0, mode="persistent")
    assert torch.equal(o2["y"], o["y"]) and torch.equal(o2["layer_rows"], o["layer_rows"])
    sample = np.linspace(0, cfg.rows - 1, 97).astype(np.int64)
    ys = y0[torch.from_numpy(sample).to(DEV)]
    check_layer_sync(ys.cpu().numpy(), net.layer(0, ys).cpu().numpy(), host_layers(idx, w, b, 0, 1)[0], cfg.clamp)


@pytest.mark.slow
@pytest.mark.parametrize("name", ["C3", "C4"])
def test_batched_full_size_sampled(P, name):
    """Full-size batched configs: all 20 uneven batches in one pass; the oracle
    follows sampled rows of every batch through the first three layers."""
    cfg = gen.CONFIGS[name]
    idx, w, b = upload(cfg, exact_layers=3)
    off = gen.make_batches(cfg)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    del y0h
    net = P.Net(idx, w, b, max_rows=cfg.rows)
    o, nz = run_forward(net, y0, batch_off=list(off), mode="persistent")
    prof = o["layer_rows"].cpu().numpy()
    assert len(nz) == 0 and not torch.any(o["y"])
    assert prof[0] == cfg.rows and (prof[4:] == 0).all()
    o2, _ = run_forward(net, y0, batch_off=list(off), mode="graph_merged")
    assert torch.equal(o2["layer_rows"], o["layer_rows"])
    rows = np.concatenate([np.linspace(off[i], off[i + 1] - 1, 3).astype(np.int64) for i in range(len(off) - 1)])
    ys = y0[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    ref = oracle.forward(host_layers(idx, w, b, 0, 3), ys, cfg.clamp)
    assert ref.alive_after[-1] == 0
    y1 = net.layer(0, y0[torch.from_numpy(rows).to(DEV)])
    check_layer_sync(ys, y1.cpu().numpy(), host_layers(idx, w, b, 0, 1)[0], cfg.clamp)


def test_determinism_run_to_run(P):
    cfg = gen.CONFIGS["S2"].with_(n_neurons=4096, n_layers=12, rows=700)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = P.Net(idx, w, b, max_rows=700)
    a, _ = run_forward(net, y0, mode="persistent")
    ya = a["y"].clone()
    b2, _ = run_forward(net, y0, mode="persistent")
    assert torch.equal(ya, b2["y"])


def test_kernel_timing_api(P):
    """sdnn_set_timing / sdnn_kernel_time: one event pair per persistent launch, the
    sum restarts after each read, the kernel time fits inside the wall time of the
    calls, and other engines record nothing."""
    import time
    cfg = gen.CONFIGS["S2"].with_(n_neurons=1024, n_layers=12, rows=2000, seed=31)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = _net(P, idx, w, b, cfg.rows)
    o = {}
    net.set_exec("persistent")
    net.forward(y0, out=o)
    net.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        net.forward(y0, out=o)
    ms, n = net.kernel_time()             # waits for the recorded events
    wall_ms = (time.perf_counter() - t0) * 1e3
    assert n == 3 and 0.0 < ms <= wall_ms
    assert net.kernel_time() == (0.0, 0)  # a new sum
    net.set_exec("graph")
    net.forward(y0, out=o)
    assert net.kernel_time() == (0.0, 0)  # only the persistent kernel is timed
    net.set_timing(False)
    net.set_exec("persistent")
    net.forward(y0, out=o)
    torch.cuda.synchronize()
    assert net.kernel_time()[1] == 0
    net.close()


@pytest.mark.parametrize("N,rows", [(1024, 600), (65536, 40)])
def test_device_error_is_reported_by_the_next_call(P, N, rows):
    """An error word raised on the device (injected from the host here, as a timed-out
    barrier would raise it): every grid barrier of the persistent chain gives up, the
    kernels return normally, the finalize pass publishes the word, and the next call
    returns SDNN_EDEVICE without launching anything; a recreated net works."""
    cfg = gen.CONFIGS["S2"].with_(n_neurons=N, n_layers=6, rows=rows, seed=5)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    net = _net(P, idx, w, b, rows)
    ref, _ = run_forward(net, y0, mode="persistent")
    ref_y = ref["y"].clone()
    net.check_device()
    net.inject_device_error(1)
    o = net.forward(y0, out=ref)                  # runs; every barrier gives up
    torch.cuda.synchronize()
    with pytest.raises(P.SdnnError, match="EDEVICE"):
        net.forward(y0, out=ref)
    with pytest.raises(P.SdnnError, match="EDEVICE"):
        net.layer(0, y0)
    with pytest.raises(P.SdnnError, match="EDEVICE"):
        net.check_device()
    with pytest.raises(P.SdnnError, match="EINVAL"):
        net.inject_device_error(0)
    net.close()
    net = _net(P, idx, w, b, rows)
    o, _ = run_forward(net, y0, mode="persistent")
    net.check_device()
    assert torch.equal(o["y"], ref_y)
    net.close()
