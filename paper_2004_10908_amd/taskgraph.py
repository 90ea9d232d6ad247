"""ctypes binding of include/sdnn_taskgraph.h (argument marshalling only).

``Executor`` owns a task-graph executor of the library (CPU and GPU worker
threads with work stealing); ``pipeline_run`` runs the inference task graph
(decode a batch on the CPU, run it on the GPU, check its categories on the CPU)
on it.  Every task body runs in the library's C++ code.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from .sdnn import SdnnError, _ptr, lib

SDNN_TG_CPU, SDNN_TG_GPU = 0, 1

_P, _I32, _I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
PROTOTYPES = [
    ("sdnn_tg_executor_create", _I32, [_I32, _I32, ctypes.POINTER(_P)]),
    ("sdnn_tg_executor_destroy", None, [_P]),
    ("sdnn_tg_executor_stats", _I32, [_P, _P]),
    ("sdnn_tg_run_diamond_chain", _I32, [_P, _I32, _I32, _I32, ctypes.POINTER(_I64)]),
    ("sdnn_tg_run_condition_loop", _I32, [_P, _I32, ctypes.POINTER(_I32)]),
    ("sdnn_tg_pipeline_run", _I32, [_P, _P, _I32, _I32, _I64, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                    ctypes.POINTER(ctypes.c_double)]),
    ("sdnn_tg_last_error", ctypes.c_char_p, []),
]


def tglib():
    L = lib()
    if not getattr(L, "_tg_bound", False):
        for name, res, args in PROTOTYPES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        L._tg_bound = True
    return L


class TaskGraphError(SdnnError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = tglib().sdnn_tg_last_error().decode(errors="replace")
        RuntimeError.__init__(self, f"{where}: status {status}: {msg}")


def _chk(st: int, where: str) -> None:
    if st != 0:
        raise TaskGraphError(st, where)


class Executor:
    """n_cpu CPU workers and n_gpu GPU workers (each with its own HIP stream)."""

    def __init__(self, n_cpu: int, n_gpu: int = 0):
        h = _P()
        _chk(tglib().sdnn_tg_executor_create(n_cpu, n_gpu, ctypes.byref(h)), "sdnn_tg_executor_create")
        self.h = h
        self.n_cpu, self.n_gpu = n_cpu, n_gpu

    def stats(self) -> dict:
        s = np.zeros(4, np.int64)
        _chk(tglib().sdnn_tg_executor_stats(self.h, s.ctypes.data_as(_P)), "sdnn_tg_executor_stats")
        return {"executed": int(s[0]), "steals": int(s[1]), "failed_steals": int(s[2]), "sleeps": int(s[3])}

    def run_diamond_chain(self, width: int, depth: int, gpu_every: int = 0) -> int:
        out = _I64()
        _chk(tglib().sdnn_tg_run_diamond_chain(self.h, width, depth, gpu_every, ctypes.byref(out)),
             "sdnn_tg_run_diamond_chain")
        return out.value

    def run_condition_loop(self, iterations: int) -> int:
        out = _I32()
        _chk(tglib().sdnn_tg_run_condition_loop(self.h, iterations, ctypes.byref(out)), "sdnn_tg_run_condition_loop")
        return out.value

    def close(self) -> None:
        if self.h is not None:
            tglib().sdnn_tg_executor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def csr_of_binary(y: np.ndarray):
    """(row pointer int64 [R+1], column ids int32) of the nonzeros of a [R][N] array:
    the sparse input format the pipeline decodes."""
    rows, cols = np.nonzero(y)
    ptr = np.zeros(y.shape[0] + 1, np.int64)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr), cols.astype(np.int32)


def categories_csr(rows_per_batch: Sequence[np.ndarray]):
    """(offsets int64 [nb+1], global row ids int32) of per-batch truth categories."""
    off = np.zeros(len(rows_per_batch) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows_per_batch])
    ids = np.concatenate([np.asarray(r, np.int32) for r in rows_per_batch]) if len(rows_per_batch) else \
        np.zeros(0, np.int32)
    return off, ids


def pipeline_run(ex: Executor, nets, n_neurons: int, batch_off, in_ptr, in_cols, truth_off, truth_rows,
                 y0: torch.Tensor, y: torch.Tensor, nz: torch.Tensor, n_nz: torch.Tensor):
    """Run the inference task graph; returns (mismatches per batch, seconds)."""
    bo = np.ascontiguousarray(batch_off, np.int64)
    ip = np.ascontiguousarray(in_ptr, np.int64)
    ic = np.ascontiguousarray(in_cols, np.int32)
    to = np.ascontiguousarray(truth_off, np.int64)
    tr = np.ascontiguousarray(truth_rows, np.int32)
    if tr.size == 0:
        tr = np.zeros(1, np.int32)
    nb = len(bo) - 1
    mism = np.zeros(nb, np.int64)
    handles = (_P * len(nets))(*[n.h for n in nets])
    sec = ctypes.c_double(0.0)
    _chk(tglib().sdnn_tg_pipeline_run(ex.h, ctypes.cast(handles, _P), len(nets), n_neurons, int(bo[-1]),
                                      bo.ctypes.data_as(_P), nb, ip.ctypes.data_as(_P), ic.ctypes.data_as(_P),
                                      to.ctypes.data_as(_P), tr.ctypes.data_as(_P), _ptr(y0), _ptr(y), _ptr(nz),
                                      _ptr(n_nz), mism.ctypes.data_as(_P), ctypes.byref(sec)),
         "sdnn_tg_pipeline_run")
    return mism, sec.value


__all__ = ["Executor", "pipeline_run", "csr_of_binary", "categories_csr", "SDNN_TG_CPU", "SDNN_TG_GPU",
           "TaskGraphError", "PROTOTYPES"]
