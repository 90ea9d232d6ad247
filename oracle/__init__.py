"""FP64 oracle of the layered sparse DNN -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and the
two share no code: the arithmetic lives in ``sdnn_oracle.c`` (plain C, double
precision, OpenMP over rows) and this module only strings layers together,
in the order the method applies them:

* forward (the paper's inference workload, section "Large Sparse Neural Network
  Inference"): Y_{l+1} = min(c, max(0, Y_l W_l + b_l)) for l = 0..L-1.  A row
  whose activations are all zero stays all zero while every bias is <= 0, so
  such rows may be skipped ("compaction"); with a positive bias the dead rows are
  brought back, which keeps the result equal to the plain definition.
* backward: the chain rule through the same layers (mask 0 < y < c), given the
  gradient of the loss w.r.t. the last activations.
* the mean-squared-error loss against a teacher's outputs and its gradient.

Tie awareness: for each output the C code also returns the pre-activation z and
the scale S = sum_k |w y| + |b|.  An output is "tie-ambiguous" when |z| or
|z - c| is within gamma_33 * S (gamma_n = n u / (1 - n u), u = 2^-24): an fp32
evaluation of the same sum, in any order, may land on either side of the kink.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "sdnn_oracle.c")
LIB_PATH = os.path.join(_HERE, "libsdnn_oracle.so")

U_FP32 = 2.0 ** -24


def gamma(n: int, u: float = U_FP32) -> float:
    """Higham's gamma_n = n u / (1 - n u): the relative error bound of an n-term fp sum."""
    return n * u / (1.0 - n * u)


def build(force: bool = False) -> str:
    """Compile the C oracle into a shared library next to its source."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_layer_forward.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_double,
                                        P, P, P, P, P, ctypes.c_int]
        L.orc_layer_forward.restype = None
        L.orc_layer_backward.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_double,
                                         P, P, P, P, P, P, ctypes.c_int]
        L.orc_layer_backward.restype = None
        L.orc_layer_bound.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_double, P, P,
                                      P, ctypes.c_int]
        L.orc_layer_bound.restype = None
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _use_library(path: Optional[str]) -> None:
    """Point the driver at another build of the C file (tests plant mistakes this way)."""
    global _lib, LIB_PATH
    _lib = None
    LIB_PATH = path if path is not None else os.path.join(_HERE, "libsdnn_oracle.so")


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check_layer(idx: np.ndarray, w: np.ndarray, b: Optional[np.ndarray]):
    idx = np.ascontiguousarray(idx, np.int32)
    w = np.ascontiguousarray(w, np.float32)
    if idx.ndim != 2 or idx.shape != w.shape:
        raise ValueError("idx and w must both be [N][K]")
    N = idx.shape[0]
    if idx.size and (idx.min() < 0 or idx.max() >= N):
        raise ValueError("input neuron ids out of range")
    if b is not None:
        b = np.ascontiguousarray(b, np.float32)
        if b.shape != (N,):
            raise ValueError("bias must be [N]")
    return idx, w, b


def layer_forward(idx, w, b, clamp: float, y_in: np.ndarray, want_zs: bool = False, threads: int = 0):
    """One layer on all rows of ``y_in`` ([R][N], converted to double).

    Returns (y_out [R][N] double, alive bool [R], z or None, S or None).
    """
    idx, w, b = _check_layer(idx, w, b)
    N, K = idx.shape
    y_in = np.ascontiguousarray(y_in, np.float64)
    if y_in.ndim != 2 or y_in.shape[1] != N:
        raise ValueError("y_in must be [R][N]")
    R = y_in.shape[0]
    y_out = np.empty((R, N), np.float64)
    alive = np.empty(R, np.uint8)
    z = np.empty((R, N), np.float64) if want_zs else None
    s = np.empty((R, N), np.float64) if want_zs else None
    if R:
        lib().orc_layer_forward(R, N, K, _p(idx), _p(w), _p(b), float(clamp), _p(y_in), _p(y_out), _p(z), _p(s),
                                _p(alive), int(threads))
    return y_out, alive.astype(bool), z, s


def layer_backward(idx, w, clamp: float, y_in, y_out, dy_out, want_dy_in: bool = True, threads: int = 0):
    """One backward layer.  Returns (dW [N][K], db [N], dY_in [R][N] or None), all double."""
    idx, w, _ = _check_layer(idx, w, None)
    N, K = idx.shape
    y_in = np.ascontiguousarray(y_in, np.float64)
    y_out = np.ascontiguousarray(y_out, np.float64)
    dy_out = np.ascontiguousarray(dy_out, np.float64)
    R = y_in.shape[0]
    if y_out.shape != (R, N) or dy_out.shape != (R, N) or y_in.shape != (R, N):
        raise ValueError("y_in, y_out and dy_out must all be [R][N]")
    dw = np.zeros((N, K), np.float64)
    db = np.zeros(N, np.float64)
    dy_in = np.zeros((R, N), np.float64) if want_dy_in else None
    if R:
        lib().orc_layer_backward(R, N, K, _p(idx), _p(w), float(clamp), _p(y_in), _p(y_out), _p(dy_out),
                                 _p(dw), _p(db), _p(dy_in), int(threads))
    return dw, db, dy_in


def layer_bound(idx, w, b, y_in, e_in=None, threads: int = 0) -> np.ndarray:
    """Forward error bound of any fp32 evaluation of one layer (see sdnn_oracle.c)."""
    idx, w, b = _check_layer(idx, w, b)
    N, K = idx.shape
    y_in = np.ascontiguousarray(y_in, np.float64)
    R = y_in.shape[0]
    if e_in is not None:
        e_in = np.ascontiguousarray(e_in, np.float64)
        if e_in.shape != y_in.shape:
            raise ValueError("e_in must match y_in")
    e_out = np.empty((R, N), np.float64)
    if R:
        lib().orc_layer_bound(R, N, K, _p(idx), _p(w), _p(b), gamma(33), _p(y_in), _p(e_in), _p(e_out), int(threads))
    return e_out


def ambiguous(z: np.ndarray, s: np.ndarray, clamp: float) -> np.ndarray:
    """Boolean mask of tie-ambiguous outputs (see the module docstring)."""
    tol = gamma(33) * s
    return (np.abs(z) <= tol) | (np.abs(z - clamp) <= tol)


@dataclass
class ForwardResult:
    y: np.ndarray                         # [B][N] double, final activations (dead rows 0)
    alive: np.ndarray                     # bool [B], rows with a nonzero final activation
    alive_after: List[int]                # |rows alive after layer l|, l = 0..L-1
    ambiguous: List[int] = field(default_factory=list)   # tie-ambiguous outputs per layer (if asked)
    ys: Optional[List[np.ndarray]] = None  # Y_0..Y_L, each [B][N] double (if asked)
    bound: Optional[np.ndarray] = None    # [B][N] forward error bound of any fp32 evaluation (if asked)
    bounds: Optional[List[np.ndarray]] = None  # E_0..E_L per layer (if keep and bound)

    @property
    def nz_rows(self) -> np.ndarray:
        return np.flatnonzero(self.alive).astype(np.int32)


def forward(layers: Iterable[Tuple[np.ndarray, np.ndarray, np.ndarray]], y0: np.ndarray, clamp: float = 32.0,
            compact: bool = True, keep: bool = False, ties: bool = False, bound: bool = False,
            threads: int = 0) -> ForwardResult:
    """Run the layer chain over all rows of ``y0`` ([B][N]).

    ``layers`` yields (idx [N][K], w [N][K], b [N]) in layer order (a generator is fine,
    so a large net can be drawn one layer at a time).  With ``compact`` rows that are
    all zero are skipped while every bias met so far is <= 0.  With ``bound`` the
    forward error bound of any fp32 evaluation of the chain is propagated too
    (over every row: a row an fp32 evaluation keeps alive may be dead here).
    """
    y = np.array(y0, dtype=np.float64, copy=True)
    B = y.shape[0]
    err = np.zeros_like(y) if bound else None
    errs = [err.copy()] if (bound and keep) else None
    act = np.ones(B, bool) if not compact else (y != 0).any(axis=1)
    alive_after: List[int] = []
    amb: List[int] = []
    ys = [y.copy()] if keep else None
    for (idx, w, b) in layers:
        b = np.asarray(b, np.float32)
        if compact and b.size and float(b.max()) > 0.0:
            act = np.ones(B, bool)        # a positive bias revives all-zero rows: treat every row
        rows = np.flatnonzero(act)
        if bound:
            err = layer_bound(idx, w, b, y, err, threads=threads)
        y_rows, a_rows, z, s = layer_forward(idx, w, b, clamp, y[rows], want_zs=ties, threads=threads)
        if ties:
            amb.append(int(ambiguous(z, s, clamp).sum()))
        ynew = np.zeros_like(y)
        ynew[rows] = y_rows
        y = ynew
        alive_now = np.zeros(B, bool)
        alive_now[rows] = a_rows
        alive_after.append(int(alive_now.sum()))
        act = alive_now if compact else np.ones(B, bool)
        if keep:
            ys.append(y.copy())
            if errs is not None:
                errs.append(err.copy())
    alive = (y != 0).any(axis=1)
    return ForwardResult(y=y, alive=alive, alive_after=alive_after, ambiguous=amb, ys=ys, bound=err, bounds=errs)


def backward(layers: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]], ys: Sequence[np.ndarray],
             dy_last: np.ndarray, clamp: float = 32.0, threads: int = 0):
    """Gradients of the loss given dL/dY_L, through every layer in reverse order.

    ``ys`` are the forward activations Y_0..Y_L (as returned by ``forward(keep=True)``).
    Returns (dW list [L] of [N][K], db list [L] of [N], dY_0 [B][N]), all double.
    """
    L = len(layers)
    if len(ys) != L + 1:
        raise ValueError("need Y_0..Y_L")
    dws: List[Optional[np.ndarray]] = [None] * L
    dbs: List[Optional[np.ndarray]] = [None] * L
    g = np.asarray(dy_last, np.float64)
    for l in range(L - 1, -1, -1):
        idx, w, _b = layers[l]
        dw, db, g = layer_backward(idx, w, clamp, ys[l], ys[l + 1], g, want_dy_in=True, threads=threads)
        dws[l], dbs[l] = dw, db
    return dws, dbs, g


def mse(y: np.ndarray, t: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean squared error over all B*N entries and its gradient 2 (y - t) / (B N)."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def teacher_outputs(layers_teacher, y0, clamp: float = 32.0, threads: int = 0) -> np.ndarray:
    """The teacher net's final activations, rounded to fp32 (frozen MSE target)."""
    return forward(layers_teacher, y0, clamp, compact=True, threads=threads).y.astype(np.float32)


__all__ = ["build", "lib", "gamma", "layer_forward", "layer_backward", "layer_bound", "ambiguous", "forward", "backward",
           "ForwardResult", "mse", "teacher_outputs", "max_threads", "U_FP32"]
