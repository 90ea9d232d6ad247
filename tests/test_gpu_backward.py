"""GPU parity of the backward pass against the oracle, checkpoint invariance,
determinism and the autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
import sdnn_inputs as gen
from tests.sdnn_gpu import DEV, check_grad, host_layers, upload

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


def summand_scales(layers, ys, dy_h, clamp):
    """S_g = sum_r |G[r,j]| |Y_l[r, idx[j,k]]| and sum_r |G[r,j]| per layer (fp64)."""
    g = np.asarray(dy_h, np.float64)
    sw, sb = [None] * len(layers), [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        idx, w, _ = layers[l]
        G = g * ((ys[l + 1] > 0) & (ys[l + 1] < clamp))
        aG = np.abs(G)
        sw[l] = np.einsum("rj,rjk->jk", aG, np.abs(ys[l])[:, idx])
        sb[l] = aG.sum(axis=0)
        _, _, g = oracle.layer_backward(idx, w, clamp, ys[l], ys[l + 1], g)
    return sw, sb


@pytest.mark.parametrize("N,L,rows,S,clamp,bias", [(64, 5, 13, 2, 1.5, 0.05), (256, 7, 40, 3, 32.0, 0.0),
                                                   (1024, 9, 33, 4, 2.0, -0.02)])
def test_backward_small_nets(P, N, L, rows, S, clamp, bias):
    cfg = gen.tiny_config(N, L, rows, seed=N + L, weight="he", bias=bias, clamp=clamp, row_density=True)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=rows, clamp=clamp, ckpt_every=S, flags=P.sdnn.SDNN_TRAINABLE)
    y0h = gen.make_inputs(cfg) * np.float32(1.25)
    y0 = torch.from_numpy(y0h).to(DEV)
    rng = np.random.default_rng(1)
    V = rng.normal(size=(rows, N)).astype(np.float32)
    o, dy, dw, db, dy0 = gpu_fwd_bwd(P, net, y0, lambda y: torch.from_numpy(V).to(DEV))
    layers = host_layers(idx, w, b)
    ref, dws, dbs, rdy0 = oracle_grads(layers, y0h, V.astype(np.float64), clamp)
    sw, sb = summand_scales(layers, ref.ys, V, clamp)
    for l in range(L):
        check_grad(dw[l].cpu().numpy(), dws[l], sw[l], rows, f"dW[{l}]")
        check_grad(db[l].cpu().numpy(), dbs[l], sb[l], rows, f"db[{l}]")
    assert np.abs(dy0.cpu().numpy() - rdy0).max() <= 1e-4 * max(1.0, np.abs(rdy0).max())


def _g5(P, rows, S):
    cfg = gen.CONFIGS["G5"].with_(rows=rows)
    idx, w, b = upload(cfg)
    net = P.Net(idx, w, b, max_rows=rows, ckpt_every=S, flags=P.sdnn.SDNN_TRAINABLE)
    return cfg, idx, w, b, net


@pytest.mark.slow
def test_g5_live_gradients_vs_oracle(P):
    """He weights, bias 0: about half the units are in (0, 32) in every layer."""
    rows = 96
    cfg, idx, w, b, net = _g5(P, rows, 16)
    y0h = gen.make_inputs(cfg)
    y0 = torch.from_numpy(y0h).to(DEV)
    layers = host_layers(idx, w, b)
    teacher = [(i, gen.teacher_weights(cfg, ww, l), bb) for l, (i, ww, bb) in enumerate(layers)]
    T = oracle.teacher_outputs(teacher, y0h, cfg.clamp)
    Tt = torch.from_numpy(T).to(DEV)
    o = net.forward(y0, ckpt=True)
    loss, dy = P.mse(o["y"], Tt)
    dw, db, dy0 = net.backward(y0, o["ckpt"], o["nz_rows"], o["n_nz"], dy)
    torch.cuda.synchronize()
    ref = oracle.forward(layers, y0h, cfg.clamp, keep=True)
    # forward masks agree (no tie flips), so the backward compares like with like
    yl = o["y"].cpu().numpy()
    assert ((yl > 0) & (yl < 32) == (ref.y > 0) & (ref.y < 32)).all()
    rloss, rdy = oracle.mse(ref.y, T)
    assert abs(float(loss.item()) - rloss) <= 1e-5 * rloss + 1e-12
    dws, dbs, rdy0 = oracle.backward(layers, ref.ys, rdy, cfg.clamp)
    sw, sb = summand_scales(layers, ref.ys, rdy, cfg.clamp)
    for l in range(cfg.n_layers):
        check_grad(dw[l].cpu().numpy(), dws[l], sw[l], rows, f"dW[{l}]")
        check_grad(db[l].cpu().numpy(), dbs[l], sb[l], rows, f"db[{l}]")


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
    y, nz, n = sparse_dnn(y0, net)
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
