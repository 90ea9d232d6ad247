"""Pins of the FP64 oracle against things other than itself.

The paper prints no numbers for the layer rule, so every pin here comes from
mathematics: a dense brute-force product, nets computed by hand, the closed
form of the first layer on binary inputs, invariants of the rule, and finite
differences / a dense chain rule for the backward pass.
"""
import math

import numpy as np
import pytest

import sdnn_inputs as gen


# ---------------------------------------------------------------- helpers (independent of oracle/)
def dense_matrix(idx, w):
    """Dense [N_in][N_out] matrix of one layer: column j holds w[j][k] at row idx[j][k]."""
    N = idx.shape[0]
    M = np.zeros((N, N), np.float64)
    for j in range(N):
        M[idx[j], j] = w[j].astype(np.float64)
    return M


def dense_forward(layers, y0, clamp):
    ys = [np.asarray(y0, np.float64)]
    for idx, w, b in layers:
        z = ys[-1] @ dense_matrix(idx, w) + b.astype(np.float64)
        ys.append(np.minimum(clamp, np.maximum(0.0, z)))
    return ys


def random_net(N, K, L, seed, clamp_scale=1.0, pos_bias=False):
    rng = np.random.default_rng(seed)
    layers = []
    for _ in range(L):
        idx = np.stack([np.sort(rng.choice(N, K, replace=False)) for _ in range(N)]).astype(np.int32)
        w = rng.normal(0, 1.0 / math.sqrt(K), (N, K)).astype(np.float32) * np.float32(clamp_scale)
        b = rng.normal(0, 0.2, N).astype(np.float32)
        if not pos_bias:
            b = -np.abs(b)
        layers.append((idx, w, b))
    return layers


# ---------------------------------------------------------------- forward pins
@pytest.mark.parametrize("N,K,L,rows,clamp,pos_bias", [
    (8, 2, 3, 5, 32.0, True), (40, 8, 5, 17, 1.5, False), (64, 32, 4, 33, 1.0, True), (256, 32, 8, 20, 32.0, False)])
def test_forward_matches_dense_bruteforce(orc, N, K, L, rows, clamp, pos_bias):
    layers = random_net(N, K, L, seed=N * 7 + L, pos_bias=pos_bias)
    rng = np.random.default_rng(N)
    y0 = (rng.random((rows, N)) < 0.4).astype(np.float32) * rng.uniform(0.5, 2.0, (rows, N)).astype(np.float32)
    y0[0] = 0.0                                      # one all-zero input row
    ref = dense_forward(layers, y0, clamp)
    for compact in (True, False):
        res = orc.forward(layers, y0, clamp, compact=compact, keep=True)
        for l in range(L + 1):
            np.testing.assert_allclose(res.ys[l], ref[l], rtol=1e-12, atol=1e-12)
        assert np.array_equal(res.alive, (ref[-1] != 0).any(axis=1))


# A 4-neuron, 2-layer net worked by hand.  K = 2, clamp c = 4.
HAND_L0 = (np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32),
           np.array([[0.5, 0.25], [1, -1], [2, 0.5], [0.125, 4]], np.float32),
           np.array([-0.25, 0, -1, 0.5], np.float32))
HAND_L1 = (np.array([[0, 3], [1, 2], [0, 1], [2, 3]], np.int32),
           np.array([[1, 1], [0.5, 0.5], [-1, 2], [0.25, -0.5]], np.float32),
           np.array([0, -0.5, 0, -0.25], np.float32))
HAND_Y0 = np.array([[1, 2, 0, 4], [0, 0, 0, 0], [3, 0, 1, 0]], np.float32)
# row 0: n0 = .5*1+.25*2-.25 = .75; n1 = 2-0 = 2; n2 = 0+.5*4-1 = 1; n3 = .125+16+.5 -> clip 4
# row 1 (all-zero input): only the positive bias of n3 survives: .5
# row 2: n0 = 1.5-.25 = 1.25; n1 = 0-1 -> 0; n2 = 2-1 = 1; n3 = .375+.5 = .875
HAND_Y1 = np.array([[0.75, 2, 1, 4], [0, 0, 0, 0.5], [1.25, 0, 1, 0.875]])
# row 0: n0 = .75+4 -> clip 4; n1 = 1+.5-.5 = 1; n2 = -.75+4 = 3.25; n3 = .25-2-.25 -> 0
# row 1: n0 = .5; n1 = -.5 -> 0; n2 = 0; n3 = -.25-.25 -> 0
# row 2: n0 = 1.25+.875 = 2.125; n1 = 0+.5-.5 = 0; n2 = -1.25 -> 0; n3 = .25-.4375-.25 -> 0
HAND_Y2 = np.array([[4, 1, 3.25, 0], [0.5, 0, 0, 0], [2.125, 0, 0, 0]])
# backward of L = sum(Y2):
# mask(Y2) = 0<y<4 -> G1 = [[0,1,1,0],[1,0,0,0],[1,0,0,0]]  (the clipped 4 gets no gradient)
HAND_DB1 = np.array([2, 1, 1, 0])
HAND_DW1 = np.array([[1.25, 1.375], [2, 1], [0.75, 2], [0, 0]])
# dY1 = G1 W1^T: row 0 = [-1, 2.5, .5, 0]; rows 1, 2 = [1, 0, 0, 1]; masked by 0<Y1<4:
HAND_DB0 = np.array([0, 2.5, 0.5, 2])
HAND_DW0 = np.array([[2, -2], [5, 0], [0, 2], [3, 0]])
HAND_DY0 = np.array([[-0.5, 2.25, -1.5, 0.25], [0.125, 0, 0, 4], [0.625, 0.25, 0, 4]])


def test_hand_computed_net(orc):
    res = orc.forward([HAND_L0, HAND_L1], HAND_Y0, clamp=4.0, keep=True)
    assert np.array_equal(res.ys[1], HAND_Y1)
    assert np.array_equal(res.ys[2], HAND_Y2)
    assert list(res.nz_rows) == [0, 1, 2]
    dws, dbs, dy0 = orc.backward([HAND_L0, HAND_L1], res.ys, np.ones((3, 4)), clamp=4.0)
    assert np.array_equal(dbs[1], HAND_DB1) and np.array_equal(dws[1], HAND_DW1)
    assert np.array_equal(dbs[0], HAND_DB0) and np.array_equal(dws[0], HAND_DW0)
    assert np.array_equal(dy0, HAND_DY0)


def test_first_layer_closed_form_on_binary_inputs(orc):
    """Binary inputs and w = 1/16: z = (number of active inputs)/16 + b exactly."""
    cfg = gen.CONFIGS["C1"]
    idx, w, b = gen.make_layer(cfg, 0)
    y0 = gen.make_inputs(cfg)
    counts = y0.astype(np.int64)[:, idx].sum(axis=2)          # [B][N] integer counts
    expect = np.minimum(32.0, np.maximum(0.0, counts / 16.0 + float(b[0])))
    y1, alive, z, s = orc.layer_forward(idx, w, b, 32.0, y0, want_zs=True)
    assert np.array_equal(y1, expect)
    assert np.array_equal(z, counts / 16.0 + float(b[0]))


def binom_tail(n, p, c):
    return sum(math.comb(n, i) * p ** i * (1 - p) ** (n - i) for i in range(c, n + 1))


@pytest.mark.parametrize("bias,cmin,density", [(-0.3, 5, 0.795616), (-0.35, 6, 0.639809),
                                               (-0.4, 7, 0.464526), (-0.45, 8, 0.301763)])
def test_first_layer_density_matches_binomial(orc, bias, cmin, density):
    """Fraction of nonzero first-layer outputs = P(Bin(32, 0.2) >= c_min)."""
    assert abs(binom_tail(32, 0.2, cmin) - density) < 1e-6
    assert (cmin - 1) / 16 + bias <= 0 < cmin / 16 + bias
    cfg = gen.CONFIGS["C1"].with_(bias=bias, rows=600)
    idx, w, b = gen.make_layer(cfg, 0)
    y1, _, _, _ = orc.layer_forward(idx, w, b, 32.0, gen.make_inputs(cfg))
    assert abs(float((y1 != 0).mean()) - density) < 0.004


def test_saturated_row_is_a_fixed_point(orc):
    """A row of all c stays all c when 32 * sum_k w * c... i.e. 32*(1/16)*32 + b >= 32."""
    cfg = gen.CONFIGS["C1"].with_(rows=3)
    y0 = np.zeros((3, 1024), np.float32)
    y0[1] = 32.0
    res = orc.forward((l[1:] for l in gen.iter_layers(cfg, 0, 10)), y0)
    assert (res.y[1] == 32.0).all() and (res.y[0] == 0).all() and (res.y[2] == 0).all()
    assert list(res.nz_rows) == [1]


def test_compaction_is_exact_and_rows_are_independent(orc):
    cfg = gen.CONFIGS["C1"].with_(rows=200, row_density=True)
    layers = [l[1:] for l in gen.iter_layers(cfg, 0, 12)]
    y0 = gen.make_inputs(cfg)
    a = orc.forward(layers, y0, compact=True)
    b = orc.forward(layers, y0, compact=False)
    assert np.array_equal(a.y, b.y) and a.alive_after == b.alive_after
    sub = np.arange(3, 200, 7)
    c = orc.forward(layers, y0[sub], compact=True)
    assert np.array_equal(c.y, a.y[sub])


def test_positive_bias_revives_dead_rows(orc):
    """With a positive bias an all-zero row maps to h(b), so compaction must not drop it."""
    N = 64
    layers = random_net(N, 8, 3, seed=5, pos_bias=False)
    idx, w, b = layers[1]
    b = b.copy()
    b[3] = 0.25
    layers[1] = (idx, w, b)
    y0 = np.zeros((4, N), np.float32)
    y0[2, :10] = 1.0
    ref = dense_forward(layers, y0, 32.0)
    res = orc.forward(layers, y0, compact=True, keep=True)
    for l in range(4):
        np.testing.assert_allclose(res.ys[l], ref[l], rtol=1e-12, atol=1e-14)
    assert res.ys[2][0, 3] != 0.0   # a row dead after layer 0 is revived by layer 1's bias


@pytest.mark.parametrize("name,rows,layers", [("C1", 1000, 6), ("C2", 300, 4), ("C3", 60, 3), ("C4", 12, 3),
                                              ("C5", 300, 4)])
def test_literal_workloads_go_extinct(orc, name, rows, layers):
    """Characterisation: with these biases and weights every row dies within 3 layers."""
    cfg = gen.CONFIGS[name].with_(rows=rows)
    res = orc.forward((l[1:] for l in gen.iter_layers(cfg, 0, layers)), gen.make_inputs(cfg))
    assert res.alive_after[0] > 0
    assert res.alive_after[min(2, layers - 1)] == 0 and not res.alive.any()


def test_tie_flags_cover_fp32_flips(orc):
    """Every 0/nonzero disagreement between an fp32 evaluation and the fp64 oracle is flagged."""
    cfg = gen.CONFIGS["S2"].with_(rows=200, n_neurons=1024)
    l0, l1 = [l[1:] for l in gen.iter_layers(cfg, 0, 2)]
    y1, _, _, _ = orc.layer_forward(*l0, 32.0, gen.make_inputs(cfg))
    y2, _, z, s = orc.layer_forward(*l1, 32.0, y1, want_zs=True)
    idx, w, b = l1
    y1f = y1.astype(np.float32)
    acc = np.zeros(y2.shape, np.float32)
    for k in range(32):                                   # sequential fp32 sum, slot order
        acc = (acc + w[:, k][None, :] * y1f[:, idx[:, k]]).astype(np.float32)
    zf = (acc + b[None, :]).astype(np.float32)
    yf = np.minimum(np.float32(32), np.maximum(np.float32(0), zf))
    flip = (yf != 0) != (y2 != 0)
    amb = orc.ambiguous(z, s, 32.0)
    assert not (flip & ~amb).any()
    # and the fp32 values agree with the oracle within the conditioning-scaled bound
    assert (np.abs(yf - y2) <= np.maximum(1e-5 * np.abs(y2), orc.gamma(33) * s)).all()


# ---------------------------------------------------------------- backward pins
def dense_backward(layers, ys, dy, clamp):
    g = np.asarray(dy, np.float64)
    dws, dbs = [None] * len(layers), [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        idx, w, _ = layers[l]
        M = dense_matrix(idx, w)
        G = g * ((ys[l + 1] > 0) & (ys[l + 1] < clamp))
        D = ys[l].T @ G                                   # dense dL/dM
        dws[l] = np.take_along_axis(D.T, idx.astype(np.int64), axis=1)
        dbs[l] = G.sum(axis=0)
        g = G @ M.T
    return dws, dbs, g


@pytest.mark.parametrize("N,K,L,rows,clamp", [(8, 2, 2, 4, 1.5), (48, 8, 4, 9, 1.0), (128, 32, 3, 16, 32.0)])
def test_backward_matches_dense_chain_rule(orc, N, K, L, rows, clamp):
    layers = random_net(N, K, L, seed=N + L, pos_bias=True)
    rng = np.random.default_rng(3)
    y0 = rng.uniform(0, 2, (rows, N)).astype(np.float32)
    res = orc.forward(layers, y0, clamp, keep=True)
    dy = rng.normal(size=(rows, N))
    dws, dbs, dy0 = orc.backward(layers, res.ys, dy, clamp)
    rdws, rdbs, rdy0 = dense_backward(layers, res.ys, dy, clamp)
    for l in range(L):
        np.testing.assert_allclose(dws[l], rdws[l], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(dbs[l], rdbs[l], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(dy0, rdy0, rtol=1e-11, atol=1e-12)


def _masks(ys, clamp):
    return [((y > 0) & (y < clamp)) | (y >= clamp) * 2 for y in ys[1:]]


def test_backward_matches_finite_differences(orc):
    """Central differences on weights and biases, skipping steps that change a mask."""
    N, K, L, rows, clamp = 16, 4, 3, 5, 1.5
    layers = random_net(N, K, L, seed=11, pos_bias=True)
    rng = np.random.default_rng(12)
    y0 = rng.uniform(0, 2, (rows, N)).astype(np.float32)
    V = rng.normal(size=(rows, N))
    base = orc.forward(layers, y0, clamp, keep=True)
    dws, dbs, _ = orc.backward(layers, base.ys, V, clamp)
    m0 = _masks(base.ys, clamp)

    def loss_with(l, which, j, k, val):
        idx, w, b = layers[l]
        w2, b2 = w.copy(), b.copy()
        if which == "w":
            w2[j, k] = val
        else:
            b2[j] = val
        lay = list(layers)
        lay[l] = (idx, w2, b2)
        r = orc.forward(lay, y0, clamp, keep=True)
        same = all(np.array_equal(a, c) for a, c in zip(_masks(r.ys, clamp), m0))
        return float((r.y * V).sum()), same

    checked = 0
    for l in range(L):
        idx, w, b = layers[l]
        for (which, j, k) in [("w", j, k) for j in range(0, N, 3) for k in range(K)] + [("b", j, 0) for j in range(N)]:
            th = float(w[j, k]) if which == "w" else float(b[j])
            hp = np.float32(th + 1e-3 * max(1.0, abs(th)))
            hm = np.float32(th - 1e-3 * max(1.0, abs(th)))
            fp, okp = loss_with(l, which, j, k, hp)
            fm, okm = loss_with(l, which, j, k, hm)
            if not (okp and okm):
                continue
            fd = (fp - fm) / (float(hp) - float(hm))
            an = dws[l][j, k] if which == "w" else dbs[l][j]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, which, j, k, fd, an)
            checked += 1
    assert checked > 100


def test_backward_linear_regime_closed_form(orc):
    """Positive weights, positive biases and a huge clamp keep every mask at 1: the net is
    affine, Y_L = Y_0 M_0 ... M_{L-1} + const, and the gradients are products of the M_l."""
    N, K, L, rows = 24, 6, 3, 7
    rng = np.random.default_rng(21)
    layers = []
    for _ in range(L):
        idx = np.stack([np.sort(rng.choice(N, K, replace=False)) for _ in range(N)]).astype(np.int32)
        layers.append((idx, rng.uniform(0.1, 0.3, (N, K)).astype(np.float32), rng.uniform(0.1, 0.2, N).astype(np.float32)))
    y0 = rng.uniform(0.1, 1.0, (rows, N)).astype(np.float32)
    clamp = 1e9
    res = orc.forward(layers, y0, clamp, keep=True)
    V = rng.normal(size=(rows, N))
    dws, dbs, dy0 = orc.backward(layers, res.ys, V, clamp)
    Ms = [dense_matrix(i, w) for i, w, _ in layers]
    tail = [np.eye(N)]
    for l in range(L - 1, -1, -1):
        tail.insert(0, Ms[l] @ tail[0])                    # tail[l] = M_l ... M_{L-1}
    np.testing.assert_allclose(dy0, V @ tail[0].T, rtol=1e-11)
    for l in range(L):
        upstream = V @ tail[l + 1].T                        # dL/dY_{l+1}
        np.testing.assert_allclose(dbs[l], upstream.sum(axis=0), rtol=1e-11)
        D = res.ys[l].T @ upstream
        np.testing.assert_allclose(dws[l], np.take_along_axis(D.T, layers[l][0].astype(np.int64), axis=1), rtol=1e-11)


def test_mse_gradient(orc):
    rng = np.random.default_rng(1)
    y, t = rng.normal(size=(5, 6)), rng.normal(size=(5, 6))
    loss, g = orc.mse(y, t)
    assert abs(loss - ((y - t) ** 2).sum() / 30) < 1e-14
    eps = 1e-6
    y2 = y.copy(); y2[2, 3] += eps
    assert abs((orc.mse(y2, t)[0] - loss) / eps - g[2, 3]) < 1e-6


# ---------------------------------------------------------------- forward error bound
def fp32_chain(layers, y0, clamp, reverse=False):
    """An independent fp32 evaluation (separate multiply and add, slot order or reversed)."""
    y = np.asarray(y0, np.float32)
    for idx, w, b in layers:
        acc = np.zeros((y.shape[0], idx.shape[0]), np.float32)
        ks = range(idx.shape[1] - 1, -1, -1) if reverse else range(idx.shape[1])
        for k in ks:
            acc = (acc + (w[:, k][None, :] * y[:, idx[:, k]]).astype(np.float32)).astype(np.float32)
        z = (acc + b[None, :]).astype(np.float32)
        y = np.minimum(np.float32(clamp), np.maximum(np.float32(0), z)).astype(np.float32)
    return y


@pytest.mark.parametrize("name,N,L,rows", [("S2", 1024, 12, 120), ("G5", 512, 10, 64), ("C5", 512, 4, 80)])
def test_fp32_evaluations_stay_within_the_propagated_bound(orc, name, N, L, rows):
    cfg = gen.CONFIGS[name].with_(n_neurons=N, n_layers=L, rows=rows, row_density=(name == "S2"))
    layers = [l[1:] for l in gen.iter_layers(cfg)]
    y0 = gen.make_inputs(cfg)
    ref = orc.forward(layers, y0, cfg.clamp, bound=True)
    for rev in (False, True):
        y32 = fp32_chain(layers, y0, cfg.clamp, reverse=rev).astype(np.float64)
        assert (np.abs(y32 - ref.y) <= ref.bound).all()
    assert (ref.bound > 0).any()


def test_fixed_relative_tolerance_is_unreachable_in_fp32_for_unsaturated_rows(orc):
    """Each layer of the challenge nets has gain sum_k |w| = 32/16 = 2, so rounding
    errors of any fp32 evaluation grow ~2^L on rows that never saturate: a fixed 1e-5
    end-to-end relative check rejects a correct fp32 chain, the propagated bound does not."""
    cfg = gen.CONFIGS["S2"].with_(n_neurons=1024, n_layers=12, rows=200)
    layers = [l[1:] for l in gen.iter_layers(cfg)]
    y0 = gen.make_inputs(cfg)
    ref = orc.forward(layers, y0, cfg.clamp, bound=True)
    y32 = fp32_chain(layers, y0, cfg.clamp).astype(np.float64)
    scale = np.maximum(np.abs(ref.y), np.abs(ref.y).max(axis=1, keepdims=True))
    assert (np.abs(y32 - ref.y) > 1e-5 * scale).any()
    assert (np.abs(y32 - ref.y) <= np.maximum(1e-5 * scale, ref.bound)).all()
    assert all(w.sum(axis=1).max() == 2.0 for _, w, _ in layers)


def _crafted_neuron(bias: float):
    """One neuron of 32 inputs all equal to 1: slot 0 weight 1, slots 1..31 weight 2^-24.
    Summed in slot order in fp32, every 1 + 2^-24 is a tie that rounds back to 1 (to
    even), so the fp32 sum loses 31 u (u = 2^-24) against the exact 1 + 31 u: the
    summation-error bound gamma_33 S is reached to within 33 / 31."""
    N, K = 32, 32
    idx = np.tile(np.arange(K, dtype=np.int32), (N, 1))
    w = np.full((N, K), 2.0 ** -24, np.float32)
    w[:, 0] = 1.0
    b = np.full(N, bias, np.float32)
    y = np.ones((1, N), np.float32)
    acc = np.float32(0.0)
    for k in range(K):
        acc = np.float32(acc + np.float32(w[0, k] * y[0, idx[0, k]]))
    z32 = np.float32(acc + b[0])
    return (idx, w, b), y, float(z32)


def test_tie_margin_and_layer_bound_are_tight(orc):
    """The fp32 rounding margin gamma_33 S used by the tie flags, the layer-synchronized
    tolerance and the one-layer error bound is not loose: on a crafted neuron a plain
    fp32 evaluation in slot order comes within a small factor of it, so a margin 2x or
    10x too wide (or a gamma with too many terms) fails here, while fp32 results never
    leave it (the other pins)."""
    U = 2.0 ** -24
    # no bias: the rounding error of the sum reaches 31 u against the bound gamma_33 (1 + 31 u)
    layer, y, z32 = _crafted_neuron(0.0)
    ref, _, z, s = orc.layer_forward(*layer, 32.0, y, want_zs=True)
    err = abs(z32 - z[0, 0])
    assert err == 31 * U
    bound = orc.layer_bound(*layer, y)[0, 0]
    assert err <= bound <= 1.07 * err
    assert orc.gamma(33) * s[0, 0] == bound
    # bias -1 cancels the sum: the exact output 31 u is positive, the fp32 one is 0, a flip
    # the tie flag must cover with a margin within 2.2x of |z| (S counts the bias too)
    layer, y, z32 = _crafted_neuron(-1.0)
    ref, _, z, s = orc.layer_forward(*layer, 32.0, y, want_zs=True)
    assert z32 == 0.0 and z[0, 0] == 31 * U and ref[0, 0] > 0
    amb = orc.ambiguous(z, s, 32.0)
    assert amb[0, 0]
    assert orc.gamma(33) * s[0, 0] <= 2.2 * abs(z[0, 0])
    # the clamp side: c = 1 + 16 u, exact z = 1 + 31 u clamps to c, the fp32 sum 1 does not
    layer, y, z32 = _crafted_neuron(0.0)
    c = float(np.float32(1.0 + 16 * U))
    ref, _, z, s = orc.layer_forward(*layer, c, y, want_zs=True)
    assert ref[0, 0] == c and z32 < c
    assert orc.ambiguous(z, s, c)[0, 0]
    assert orc.gamma(33) * s[0, 0] <= 2.3 * abs(z[0, 0] - c)
    # far from both kinks nothing is flagged
    layer, y, _ = _crafted_neuron(-0.5)
    _, _, z, s = orc.layer_forward(*layer, 32.0, y, want_zs=True)
    assert not orc.ambiguous(z, s, 32.0).any()
