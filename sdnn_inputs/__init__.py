"""Seeded synthetic inputs for the layered sparse DNN.

This module is shared by the FP64 oracle (``oracle/``) and by the GPU library's
tests and benchmark.  It holds no arithmetic of the method itself: it only draws
the connectivity pattern, the weights, the biases, the binary input matrices, the
uneven batch split and the teacher perturbation, each from a documented seed.

The real workload (the sparse-DNN graph challenge data the paper runs: an input
matrix, 1920 sparse layers, bias values and truth categories; paper, section
"Large Sparse Neural Network Inference") is not available.  These draws stand in
for it with the same shapes and value distributions:

* every output neuron j of layer l has K=32 distinct input neurons, drawn
  uniformly with ``numpy.random.default_rng([seed, l])``; a neuron whose draw
  holds a duplicate is redrawn; each neuron's list is sorted ascending (small
  test nets with n < 8k draw each neuron without replacement instead);
* weights are the constant fp32(1/16), or U(0.03, 0.09) / N(0, 2/32) drawn from
  the same per-layer generator after the pattern;
* inputs are Bernoulli(p) binary fp32 matrices from
  ``default_rng([seed, 10**6])`` (``random((B, N)) < p``, generated in row order),
  or with a per-row density p_r ~ U(0.1, 0.5) from ``default_rng([seed, 3*10**6])``;
* batches: 20 uneven consecutive row ranges, sizes drawn from
  ``default_rng([seed, 7])`` by a Dirichlet split with a floor and a cap;
* teacher weights: the student's weights plus N(0, sigma) per nonzero from
  ``default_rng([seed, 2*10**6 + l])``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Iterator, List, Optional, Tuple

import numpy as np

K_DEFAULT = 32
INPUT_STREAM = 10 ** 6
TEACHER_STREAM = 2 * 10 ** 6
ROWDENSITY_STREAM = 3 * 10 ** 6
BATCH_STREAM = 7


@dataclass(frozen=True)
class NetConfig:
    """Shape and value recipe of one synthetic network + input set."""
    name: str
    n_neurons: int
    n_layers: int
    rows: int
    seed: int
    weight: str = "const"          # "const" (1/16) | "uniform" (U(0.03,0.09)) | "he" (N(0, 2/32))
    bias: float = -0.3
    clamp: float = 32.0
    density: float = 0.2           # Bernoulli p of the binary inputs
    row_density: bool = False      # per-row p_r ~ U(0.1, 0.5) instead of a fixed p
    k: int = K_DEFAULT
    n_batches: int = 1
    batch_lo: int = 0
    batch_hi: int = 0
    teacher_sigma: float = 0.0     # > 0: a teacher net exists (MSE target)
    ckpt_every: int = 0            # > 0: trained with checkpointing every ckpt_every layers

    def with_(self, **kw) -> "NetConfig":
        return replace(self, **kw)

    @property
    def nnz(self) -> int:
        return self.n_neurons * self.k * self.n_layers


# The five literal workloads and their sustained / live-gradient companions.
CONFIGS = {
    "C1": NetConfig("C1", 1024, 120, 1000, 1, bias=-0.3),
    "C2": NetConfig("C2", 4096, 480, 60000, 2, bias=-0.35),
    "C3": NetConfig("C3", 16384, 480, 60000, 3, bias=-0.4, n_batches=20, batch_lo=500, batch_hi=8000),
    "C4": NetConfig("C4", 65536, 1920, 15000, 4, bias=-0.45, n_batches=20, batch_lo=250, batch_hi=4000),
    "C5": NetConfig("C5", 4096, 120, 4096, 5, weight="uniform", bias=-0.3, teacher_sigma=0.005, ckpt_every=16),
    "S2": NetConfig("S2", 4096, 480, 60000, 12, bias=-0.35, row_density=True),
    "S3": NetConfig("S3", 16384, 480, 60000, 13, bias=-0.4, row_density=True, n_batches=20, batch_lo=500, batch_hi=8000),
    "S4": NetConfig("S4", 65536, 1920, 15000, 14, bias=-0.45, row_density=True, n_batches=20, batch_lo=250, batch_hi=4000),
    "G5": NetConfig("G5", 4096, 120, 4096, 15, weight="he", bias=0.0, teacher_sigma=0.005, ckpt_every=16),
}


def layer_pattern(seed: int, layer: int, n: int, k: int = K_DEFAULT) -> Tuple[np.ndarray, np.random.Generator]:
    """Connectivity of one layer: int32 [n][k], each row k distinct ascending input ids.

    Returns the per-layer generator too, positioned after the pattern draws, so the
    weight draw that follows is reproducible.
    """
    if k > n:
        raise ValueError("k distinct inputs need k <= n")
    rng = np.random.default_rng([seed, layer])
    if n < 8 * k:
        # small test nets: redrawing until distinct would rarely succeed; draw each
        # neuron's inputs without replacement instead
        idx = np.stack([rng.choice(n, size=k, replace=False) for _ in range(n)]).astype(np.int64)
        idx.sort(axis=1)
        return idx.astype(np.int32), rng
    idx = rng.integers(0, n, size=(n, k), dtype=np.int64)
    while True:
        s = np.sort(idx, axis=1)
        dup = (s[:, 1:] == s[:, :-1]).any(axis=1)
        nd = int(dup.sum())
        if nd == 0:
            break
        idx[dup] = rng.integers(0, n, size=(nd, k), dtype=np.int64)
    idx.sort(axis=1)
    return idx.astype(np.int32), rng


def layer_weights(kind: str, rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    if kind == "const":
        return np.full((n, k), np.float32(1.0 / 16.0), dtype=np.float32)
    if kind == "uniform":
        return rng.uniform(0.03, 0.09, size=(n, k)).astype(np.float32)
    if kind == "he":
        return rng.normal(0.0, np.sqrt(2.0 / k), size=(n, k)).astype(np.float32)
    raise ValueError(f"unknown weight kind {kind!r}")


def make_layer(cfg: NetConfig, layer: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(idx int32 [N][K], w fp32 [N][K], bias fp32 [N]) of one layer."""
    idx, rng = layer_pattern(cfg.seed, layer, cfg.n_neurons, cfg.k)
    w = layer_weights(cfg.weight, rng, cfg.n_neurons, cfg.k)
    b = np.full(cfg.n_neurons, np.float32(cfg.bias), dtype=np.float32)
    return idx, w, b


def iter_layers(cfg: NetConfig, first: int = 0, last: Optional[int] = None) -> Iterator[Tuple[int, np.ndarray, np.ndarray, np.ndarray]]:
    last = cfg.n_layers if last is None else last
    for l in range(first, last):
        yield (l,) + make_layer(cfg, l)


def make_net(cfg: NetConfig, n_layers: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Whole net as stacked arrays: idx int32 [L][N][K], w fp32 [L][N][K], bias fp32 [L][N]."""
    L = cfg.n_layers if n_layers is None else n_layers
    N, K = cfg.n_neurons, cfg.k
    idx = np.empty((L, N, K), np.int32)
    w = np.empty((L, N, K), np.float32)
    b = np.empty((L, N), np.float32)
    for l in range(L):
        idx[l], w[l], b[l] = make_layer(cfg, l)
    return idx, w, b


def teacher_weights(cfg: NetConfig, w: np.ndarray, layer: int) -> np.ndarray:
    """Teacher weights of one layer: student's plus N(0, sigma) on every nonzero."""
    rng = np.random.default_rng([cfg.seed, TEACHER_STREAM + layer])
    return (w.astype(np.float64) + rng.normal(0.0, cfg.teacher_sigma, size=w.shape)).astype(np.float32)


def make_inputs(cfg: NetConfig, row_begin: int = 0, row_end: Optional[int] = None, chunk: int = 4096) -> np.ndarray:
    """Binary fp32 input rows [row_begin, row_end) of the [rows][N] input matrix.

    Rows are drawn in row order from one stream, so any row range is reproducible
    on its own (the stream is advanced past the rows before row_begin).
    """
    row_end = cfg.rows if row_end is None else row_end
    N = cfg.n_neurons
    rng = np.random.default_rng([cfg.seed, INPUT_STREAM])
    if cfg.row_density:
        p_all = np.random.default_rng([cfg.seed, ROWDENSITY_STREAM]).uniform(0.1, 0.5, size=cfg.rows)
    out = np.empty((row_end - row_begin, N), np.float32)
    r = 0
    while r < row_end:
        n = min(chunk, row_end - r)
        u = rng.random((n, N))
        lo, hi = max(r, row_begin), min(r + n, row_end)
        if lo < hi:
            uu = u[lo - r:hi - r]
            p = p_all[lo:hi, None] if cfg.row_density else cfg.density
            out[lo - row_begin:hi - row_begin] = (uu < p)
        r += n
    return out


def make_batches(cfg: NetConfig) -> np.ndarray:
    """int64 [n_batches + 1] offsets of consecutive uneven batches covering all rows."""
    nb, total = cfg.n_batches, cfg.rows
    if nb <= 1:
        return np.array([0, total], np.int64)
    lo, hi = cfg.batch_lo, cfg.batch_hi
    if nb * lo > total or nb * hi < total:
        raise ValueError("batch bounds cannot cover the rows")
    rng = np.random.default_rng([cfg.seed, BATCH_STREAM])
    spare = total - nb * lo
    for _ in range(10000):
        wgt = rng.dirichlet(np.ones(nb))
        frac = wgt * spare
        s = lo + np.floor(frac).astype(np.int64)
        rem = total - int(s.sum())
        order = np.argsort(-(frac - np.floor(frac)), kind="stable")
        s[order[:rem]] += 1
        if s.max() <= hi:
            break
    else:
        raise RuntimeError("no admissible batch split found")
    return np.concatenate([[0], np.cumsum(s)]).astype(np.int64)


def make_layer_device(cfg: NetConfig, layer: int, device, k: Optional[int] = None):
    """A layer with the same distributions, drawn by torch's device generator.

    A second, faster stream (seeded with ``seed * 1000003 + layer``) for the deep
    parts of large nets; it does not reproduce ``make_layer``'s values.
    Returns (idx int32 [N][K], w fp32 [N][K], bias fp32 [N]) on ``device``.
    """
    import torch
    N, K = cfg.n_neurons, cfg.k if k is None else k
    g = torch.Generator(device=device)
    g.manual_seed(cfg.seed * 1000003 + layer)
    idx = torch.randint(0, N, (N, K), generator=g, device=device, dtype=torch.int64)
    while True:
        idx, _ = torch.sort(idx, dim=1)
        dup = (idx[:, 1:] == idx[:, :-1]).any(dim=1)
        nd = int(dup.sum())
        if nd == 0:
            break
        idx[dup] = torch.randint(0, N, (nd, K), generator=g, device=device, dtype=torch.int64)
    if cfg.weight == "const":
        w = torch.full((N, K), 1.0 / 16.0, dtype=torch.float32, device=device)
    elif cfg.weight == "uniform":
        w = torch.rand((N, K), generator=g, device=device, dtype=torch.float32) * 0.06 + 0.03
    else:
        w = torch.randn((N, K), generator=g, device=device, dtype=torch.float32) * float(np.sqrt(2.0 / K))
    b = torch.full((N,), float(np.float32(cfg.bias)), dtype=torch.float32, device=device)
    return idx.to(torch.int32), w, b


def tiny_config(n: int, layers: int, rows: int, seed: int, k: int = K_DEFAULT, **kw) -> NetConfig:
    """A small net for unit tests (any n >= k)."""
    return NetConfig(f"tiny{n}x{layers}", n, layers, rows, seed, k=k, **kw)


__all__ = ["NetConfig", "CONFIGS", "layer_pattern", "layer_weights", "make_layer", "iter_layers", "make_net",
           "make_layer_device",
           "teacher_weights", "make_inputs", "make_batches", "tiny_config", "K_DEFAULT"]
