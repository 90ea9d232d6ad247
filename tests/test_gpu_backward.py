"""GPU parity of the backward pass against the oracle, checkpoint invariance,
determinism and the autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_chain, forward_layers, host_layers, normwise, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2004_10908_amd as p
    assert torch.cuda.is_available()
    p.lib()
    return p


def gpu_fwd_bwd(P, net, y0, dy_fn):
    o = net.forward(y0, ckpt=True)
    dy = dy_fn(o["y"])
    dw, db, dy0 = net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
    torch.cuda.synchronize()
    return o, dy, dw, db, dy0


def oracle_grads(layers, y0h, dy_h, clamp):
    ref = oracle.forward(layers, y0h, clamp, keep=True)
    dws, dbs, dy0 = oracle.backward(layers, ref.ys, dy_h, clamp)
    return ref, dws, dbs, dy0


def layer_sync_bounds(idx, w, clamp, y_in, y_out, dy, groups=256):
    """Exact fp64 layer backward on the fp32 inputs and the summation-error bounds
    of an fp32 evaluation: gamma_{R+P} sum|G||Y| (dW), gamma_{R+P} sum|G| (db) with P <= 256 partials,
    gamma_{deg+1} sum|w||G| (dY)."""
    R = y_in.shape[0]
    dw, db, dyi = oracle.layer_backward(idx, w, clamp, y_in, y_out, dy)
    aw, ab, ay = oracle.layer_backward(idx, np.abs(w), clamp, np.abs(y_in), y_out, np.abs(dy))
    gR = oracle.gamma(R + groups)
    gK = oracle.gamma(int(np.bincount(idx.ravel(), minlength=idx.shape[0]).max()) + 1)
    return (dw, gR * aw), (db, gR * ab), (dyi, gK * ay)


@pytest.mark.parametrize("N,rows,layer_kind,clamp", [(64, 13, "he", 1.5), (1024, 77, "he", 2.0),
                                                     (4096, 64, "he", 32.0), (4096, 200, "uniform", 32.0),
                                                     # partial last 64-id block (N % 64 = 16, 32)
                                                     (1040, 45, "he", 32.0), (96, 21, "uniform", 2.0)])
def test_layer_backward_synchronized(P, N, rows, layer_kind, clamp):
    """One layer: the GPU's dW, db, dY from given fp32 Y_l, Y_{l+1}, dY_{l+1} are within the
    summation-error bound of the exact (fp64) result on the same inputs."""
    cfg = gen.tiny_config(N, 3, rows, seed=N + rows, weight=layer_kind, bias=0.0 if layer_kind == "he" else -0.3,
                          clamp=clamp, row_density=True)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=rows, clamp=clamp, ckpt_every=1, flags=P.sdnn.SDNN_TRAINABLE)
    layers = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    ref = oracle.forward(layers, y0h, clamp, keep=True, compact=False)
    rng = np.random.default_rng(N)
    for l in range(cfg.n_layers):
        yin = ref.ys[l].astype(np.float32)
        yout = net.layer(l, torch.from_numpy(yin).to(DEV))
        dy = rng.normal(size=(rows, N)).astype(np.float32)
        gdw, gdb, gdy = net.layer_backward(l, torch.from_numpy(yin).to(DEV), yout, torch.from_numpy(dy).to(DEV))
        torch.cuda.synchronize()
        (rdw, edw), (rdb, edb), (rdy, edy) = layer_sync_bounds(layers[l][0], layers[l][1], clamp, yin,
                                                               yout.cpu().numpy(), dy)
        for name, g, r, e in (("dW", gdw, rdw, edw), ("db", gdb, rdb, edb), ("dY", gdy, rdy, edy)):
            d = np.abs(g.cpu().numpy().astype(np.float64) - r)
            assert (d <= e + 1e-30).all(), f"layer {l} {name}: worst excess {(d - e).max()}"


def replayed_gradients(P, cfg, y0h, dy_fn, idx, w, b):
    """The library's forward + backward (checkpoints every cfg.ckpt_every layers) against
    the oracle's backward replayed on the GPU's own activations Y_0 .. Y_L (taken from a
    second net over the same parameters with a checkpoint at every layer, whose forward
    is bitwise the same), so that both sides use the same masks 0 < y < c even where an
    fp32 evaluation lands on the other side of a kink than the exact one.  Per layer,
    ||dW - dW_ref|| <= 1e-4 ||dW_ref|| and the same for db and dY_0.  Returns the worst
    ratios."""
    layers = host_layers(idx, w, b)
    y0 = torch.from_numpy(y0h).to(DEV)
    net = P.Net(idx, w, b, max_rows=cfg.rows, clamp=cfg.clamp, ckpt_every=cfg.ckpt_every,
                flags=P.sdnn.SDNN_TRAINABLE)
    o = net.forward(y0, ckpt=True)
    dy = dy_fn(o["y"])
    dw, db, dy0 = net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
    torch.cuda.synchronize()
    net_a = P.Net(idx, w, b, max_rows=cfg.rows, clamp=cfg.clamp, ckpt_every=1)
    oa, nz, ys = forward_layers(net_a, y0, mode="graph")
    net_a.close()
    assert torch.equal(oa["y"], o["y"]), "the checkpointing net's forward differs from the per-layer one"
    S, L, rows = cfg.ckpt_every, cfg.n_layers, cfg.rows
    ck = o["ckpt"]
    for m in range(1, (L + S - 1) // S):
        slot = ck[(m - 1) * rows * cfg.n_neurons: m * rows * cfg.n_neurons].view(rows, cfg.n_neurons).cpu().numpy()
        alive = (ys[m * S] != 0).any(axis=1)
        assert np.array_equal(slot[alive], ys[m * S][alive]), f"checkpoint {m} differs from Y_{m * S}"
    check_chain(layers, cfg.clamp, ys, oa["layer_rows"].cpu().numpy(), nz, y0h, compact=float(b.max()) <= 0)
    dy_h = dy.cpu().numpy()
    dws, dbs, rdy0 = oracle.backward(layers, ys, dy_h, cfg.clamp)
    worst = {"dW": 0.0, "db": 0.0}
    for l in range(L):
        worst["dW"] = max(worst["dW"], normwise(dw[l].cpu().numpy(), dws[l], f"dW[{l}]"))
        worst["db"] = max(worst["db"], normwise(db[l].cpu().numpy(), dbs[l], f"db[{l}]"))
    worst["dY0"] = normwise(dy0.cpu().numpy(), rdy0, "dY0")
    net.close()
    return worst, o, dy


@pytest.mark.parametrize("N,L,rows,S,clamp,bias", [(64, 5, 13, 2, 1.5, 0.05), (256, 7, 40, 3, 32.0, 0.0),
                                                   (1024, 9, 33, 4, 2.0, -0.02),
                                                   # several tiles per tile stream in every backward kernel
                                                   (2048, 8, 1500, 3, 32.0, 0.0)])
def test_backward_small_nets(P, N, L, rows, S, clamp, bias):
    cfg = gen.tiny_config(N, L, rows, seed=N + L, weight="he", bias=bias, clamp=clamp, row_density=True,
                          ckpt_every=S)
    idx, w, b = upload(cfg)
    y0h = gen.make_inputs(cfg) * np.float32(1.25)
    V = torch.from_numpy(np.random.default_rng(1).normal(size=(rows, N)).astype(np.float32)).to(DEV)
    worst, _, _ = replayed_gradients(P, cfg, y0h, lambda y: V, idx, w, b)
    print(f"N={N} L={L} rows={rows}: worst normwise {worst}")


def test_g5_live_gradients_vs_oracle(P):
    """He weights, bias 0: about half the units are in (0, 32) in every one of the
    120 layers.  MSE against a teacher with perturbed weights; the loss gradient is the
    library's (from the GPU's outputs), the same fp32 values enter the oracle's replay."""
    cfg = gen.CONFIGS["G5"].with_(rows=1024)
    idx, w, b = upload(cfg)
    layers = host_layers(idx, w, b)
    y0h = gen.make_inputs(cfg)
    teacher = [(i, gen.teacher_weights(cfg, ww, l), bb) for l, (i, ww, bb) in enumerate(layers)]
    T = oracle.teacher_outputs(teacher, y0h, cfg.clamp)
    Td = torch.from_numpy(T).to(DEV)
    losses = []

    def dy_fn(y):
        loss, dy = P.mse(y, Td)
        losses.append((loss, y))
        return dy
    worst, o, dy = replayed_gradients(P, cfg, y0h, dy_fn, idx, w, b)
    print(f"G5 (1024 rows, 120 layers): worst per-layer normwise relative errors {worst}")
    assert worst["dW"] < 1e-4 and worst["db"] < 1e-4
    # the library's loss kernel on the GPU's own outputs
    loss, y = losses[0]
    rl, rd = oracle.mse(y.cpu().numpy(), T)
    assert abs(float(loss.item()) - rl) <= 1e-5 * rl + 1e-12
    np.testing.assert_allclose(dy.cpu().numpy(), rd, rtol=1e-5, atol=1e-12)
    assert int(o["n_nz"].item()) == cfg.rows      # every row stays alive


def test_checkpointing_does_not_change_gradients(P):
    cfg = gen.CONFIGS["G5"].with_(n_neurons=1024, n_layers=20, rows=64)
    idx, w, b = upload(cfg)
    y0 = torch.from_numpy(gen.make_inputs(cfg)).to(DEV)
    V = torch.randn(64, 1024, device=DEV, generator=torch.Generator(device=DEV).manual_seed(3))
    res = []
    for S in (20, 6, 1):
        net = P.Net(idx, w, b, max_rows=64, ckpt_every=S, flags=P.sdnn.SDNN_TRAINABLE)
        _, _, dw, db, dy0 = gpu_fwd_bwd(P, net, y0, lambda y: V)
        res.append((dw, db, dy0))
        net.close()
    for r in res[1:]:
        assert all(torch.equal(a, c) for a, c in zip(res[0], r))
    net = P.Net(idx, w, b, max_rows=64, ckpt_every=6, flags=P.sdnn.SDNN_TRAINABLE)
    _, _, dw2, db2, dy02 = gpu_fwd_bwd(P, net, y0, lambda y: V)
    assert torch.equal(dw2, res[0][0]) and torch.equal(db2, res[0][1])       # run-to-run


@pytest.mark.slow
def test_c5_literal_gradients_are_exactly_zero(P):
    cfg = gen.CONFIGS["C5"]
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=cfg.rows, ckpt_every=16, flags=P.sdnn.SDNN_TRAINABLE)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    T = torch.zeros_like(y0)
    o = net.forward(y0, ckpt=True)
    loss, dy = P.mse(o["y"], T)
    dw, db, dy0 = net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
    torch.cuda.synchronize()
    assert int(o["n_nz"].item()) == 0 and float(loss.item()) == 0.0
    assert not torch.any(dw) and not torch.any(db) and not torch.any(dy0)
    sample = gen.make_inputs(cfg, 0, 200)
    ref = oracle.forward(host_layers(idx, w, b, 0, 3), sample, cfg.clamp)
    assert ref.alive_after[-1] == 0


def test_autograd_function_and_finite_differences(P):
    from paper_2004_10908_amd.torch_fn import sparse_dnn
    cfg = gen.tiny_config(64, 4, 6, seed=5, weight="he", bias=0.05, clamp=1.5, row_density=True)
    idx, w, b = upload(cfg)
    w.requires_grad_(True)
    b.requires_grad_(True)
    net = P.Net(idx, w.detach(), b.detach(), max_rows=6, clamp=1.5, ckpt_every=2, flags=P.sdnn.SDNN_TRAINABLE)
    y0 = (torch.from_numpy(gen.make_inputs(cfg)).to(DEV) * 1.3).requires_grad_(True)
    V = torch.randn(6, 64, device=DEV, generator=torch.Generator(device=DEV).manual_seed(0))
    y, nz, n = sparse_dnn(y0, net, w, b)
    (y * V).sum().backward()
    gw, gb, gy = w.grad.clone(), b.grad.clone(), y0.grad.clone()
    # finite differences of the GPU forward on a few weights (piecewise linear, masks kept)
    wd = net.w
    checked = 0
    for (l, j, k) in [(0, 3, 1), (1, 10, 7), (2, 20, 30), (3, 40, 0), (3, 63, 31), (1, 0, 0)]:
        old = float(wd[l, j, k])
        h = 1e-2
        vals = []
        masks = []
        for s in (+1, -1):
            wd[l, j, k] = old + s * h
            o = net.forward(y0.detach())
            vals.append(float((o["y"].double() * V.double()).sum()))
            masks.append(((o["y"] > 0) & (o["y"] < 1.5)).clone())
        wd[l, j, k] = old
        if not torch.equal(masks[0], masks[1]):
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - float(gw[l, j, k])) <= 2e-3 * max(1.0, abs(fd)), (l, j, k, fd, float(gw[l, j, k]))
        checked += 1
    assert checked >= 3
    assert gy.shape == y0.shape and torch.isfinite(gb).all()


def test_mse_kernel(P):
    rng = np.random.default_rng(0)
    y = rng.normal(size=(37, 129)).astype(np.float32)
    t = rng.normal(size=(37, 129)).astype(np.float32)
    loss, dy = P.mse(torch.from_numpy(y).to(DEV), torch.from_numpy(t).to(DEV))
    rl, rdy = oracle.mse(y, t)
    assert abs(float(loss.item()) - rl) <= 1e-5 * rl
    np.testing.assert_allclose(dy.cpu().numpy(), rdy, rtol=1e-5, atol=1e-9)
