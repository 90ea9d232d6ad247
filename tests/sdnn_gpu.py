"""Helpers shared by the GPU tests: put seeded nets on the device and compare the
library's results with the oracle under the tie-aware protocol.

Protocol (readings of the paper's unstated precision contract, written here as the
checks that apply them):
* layer-synchronized: feed the GPU's Y_l to the oracle's layer; every output must
  satisfy |y_gpu - y_ref| <= max(1e-5 |y_ref|, gamma_33 S) and may differ in being
  zero / nonzero only where the oracle flags the output tie-ambiguous;
* end-to-end: the set of nonzero final rows must be identical, and on those rows
  |y_gpu - y_ref| <= 1e-5 max(|y_ref|, max_j |y_ref[r, :]|) (row-scaled);
* gradients, per layer: ||d||_2 <= 1e-4 ||g_ref||_2 and elementwise
  |d| <= max(1e-4 |g_ref|, gamma_R S_g) with S_g the sum of |summands|.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
import sdnn_inputs as gen

DEV = "cuda"


def upload(cfg, n_layers=None, exact_layers=None, device=DEV):
    """Stacked (idx, w, b) device tensors.  Layers < exact_layers come from the
    oracle's seeded generator; deeper ones from the device generator."""
    L = cfg.n_layers if n_layers is None else n_layers
    exact = L if exact_layers is None else min(L, exact_layers)
    N, K = cfg.n_neurons, cfg.k
    idx = torch.empty((L, N, K), dtype=torch.int32, device=device)
    w = torch.empty((L, N, K), dtype=torch.float32, device=device)
    b = torch.empty((L, N), dtype=torch.float32, device=device)
    for l in range(L):
        if l < exact:
            i_, w_, b_ = gen.make_layer(cfg, l)
            idx[l].copy_(torch.from_numpy(i_))
            w[l].copy_(torch.from_numpy(w_))
            b[l].copy_(torch.from_numpy(b_))
        else:
            i_, w_, b_ = gen.make_layer_device(cfg, l, device)
            idx[l].copy_(i_)
            w[l].copy_(w_)
            b[l].copy_(b_)
    return idx, w, b


def host_layers(idx, w, b, first=0, last=None):
    last = idx.shape[0] if last is None else last
    return [(idx[l].cpu().numpy(), w[l].cpu().numpy(), b[l].cpu().numpy()) for l in range(first, last)]


def check_layer_sync(y_in, y_gpu, layer, clamp):
    """Layer-synchronized comparison; returns (max scaled error, flips)."""
    idx, w, b = layer
    ref, _, z, s = oracle.layer_forward(idx, w, b, clamp, y_in, want_zs=True)
    y = np.asarray(y_gpu, np.float64)
    tol = np.maximum(1e-5 * np.abs(ref), oracle.gamma(33) * s)
    amb = oracle.ambiguous(z, s, clamp)
    flip = (y != 0) != (ref != 0)
    assert not (flip & ~amb).any(), f"zero/nonzero disagreement at a non-ambiguous output: {np.argwhere(flip & ~amb)[:5]}"
    bad = (np.abs(y - ref) > tol) & ~amb
    assert not bad.any(), f"{int(bad.sum())} outputs outside tolerance, worst {np.abs(y - ref)[bad].max()}"
    return int(flip.sum())


def check_end_to_end(y_gpu, nz_gpu, ref):
    """End-to-end comparison against an oracle ForwardResult.

    With ``ref.bound`` (the propagated fp32 error bound) an output may differ from
    the oracle by max(1e-5 * row scale, bound), and a row may be alive on one side
    only if all its outputs are within the bound of the oracle's.  Without it the
    plain row-scaled 1e-5 check applies and the row sets must match exactly.
    """
    nz_ref = ref.nz_rows
    y = np.asarray(y_gpu, np.float64)
    nz_gpu = np.asarray(nz_gpu)
    assert (np.diff(nz_gpu) > 0).all(), "nonzero-row ids must be ascending"
    scale = np.maximum(np.abs(ref.y), np.abs(ref.y).max(axis=1, keepdims=True))
    tol = 1e-5 * scale if ref.bound is None else np.maximum(1e-5 * scale, ref.bound)
    err = np.abs(y - ref.y)
    if ref.bound is None:
        assert np.array_equal(nz_gpu, nz_ref), "nonzero-row sets differ"
    else:
        diff = np.setxor1d(nz_gpu, nz_ref)
        assert (err[diff] <= ref.bound[diff]).all(), f"rows {diff[:5]} differ in liveness beyond the bound"
    gpu_dead = np.setdiff1d(np.arange(y.shape[0]), nz_gpu)
    assert (y[gpu_dead] == 0).all(), "rows reported dead must be exactly zero"
    bad = err > tol
    assert not bad.any(), f"{int(bad.sum())} outputs outside tolerance; worst excess {(err - tol)[bad].max()}"


def check_grad(g_gpu, g_ref, bound, what, normwise=True):
    """|g - g_ref| <= max(1e-4 |g_ref|, bound) elementwise, and (optionally) the
    normwise 1e-4 check, which only holds where the chain is well conditioned."""
    g = np.asarray(g_gpu, np.float64)
    d = g - g_ref
    if normwise:
        nref = np.linalg.norm(g_ref)
        assert np.linalg.norm(d) <= 1e-4 * nref + 1e-30, f"{what}: normwise {np.linalg.norm(d)} vs {nref}"
    tol = np.maximum(1e-4 * np.abs(g_ref), bound)
    bad = np.abs(d) > tol
    assert not bad.any(), f"{what}: {int(bad.sum())} elements outside tolerance, worst excess {(np.abs(d) - tol)[bad].max()}"


def backward_bounds(layers, ys, eys, dy_last, clamp, rows_groups=256):
    """First-order error bounds of an fp32 backward pass (masks taken as the oracle's).

    ys/eys: exact activations and their forward error bounds per layer; dy_last is
    the (exact, shared) dL/dY_L.  Uses the oracle's layer backward on magnitudes:
    for dW the rounded terms are (|G| + E_G)(|Y| + E_Y), for dY they are |w|(|G| + E_G).
    Returns per-layer (dW ref, E_dW, db ref, E_db) and (dY_0 ref, E_dY0).
    """
    L = len(layers)
    R = ys[0].shape[0]
    gR = oracle.gamma(R + rows_groups)
    D = np.asarray(dy_last, np.float64)
    ED = np.zeros_like(D)
    out = [None] * L
    for l in range(L - 1, -1, -1):
        idx, w, _ = layers[l]
        aw = np.abs(w)
        Y, EY, Yo = ys[l], eys[l], ys[l + 1]
        dw, db, dyi = oracle.layer_backward(idx, w, clamp, Y, Yo, D)
        dwA, dbA, dyA = oracle.layer_backward(idx, aw, clamp, np.abs(Y) + EY, Yo, np.abs(D) + ED)
        dwB, dbB, dyB = oracle.layer_backward(idx, aw, clamp, np.abs(Y), Yo, np.abs(D))
        gK = oracle.gamma(int(np.bincount(idx.ravel(), minlength=idx.shape[0]).max()) + 1)
        out[l] = (dw, (dwA - dwB) + gR * dwA, db, (dbA - dbB) + gR * dbA)
        ED = (dyA - dyB) + gK * dyA
        D = dyi
    return out, D, ED


def run_forward(net, y0, batch_off=None, mode="auto", ckpt=False):
    net.set_exec(mode)
    o = net.forward(y0, batch_off=batch_off, ckpt=ckpt, profile=True)
    torch.cuda.synchronize()
    n = int(o["n_nz"].item())
    return o, o["nz_rows"][:n].cpu().numpy()
