"""ctypes binding of the C ABI in include/sdnn.h (argument marshalling only).

Every function named ``sdnn_*`` here calls the C entry point of the same name in
``libsdnn.so`` with raw device pointers taken from torch tensors; all work runs
in the library's HIP kernels.  Loading fails loudly when the library has not
been built (there is no fallback path).

``Net`` is a small owner object: it allocates the workspace as a torch tensor on
the current device, keeps the borrowed parameter tensors alive and destroys the
C handle when it is garbage collected.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdnn.so")

SDNN_OK, SDNN_EINVAL, SDNN_ENOMEM, SDNN_EHIP, SDNN_EUNSUPPORTED, SDNN_EDEVICE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SDNN_OK", -1: "SDNN_EINVAL", -2: "SDNN_ENOMEM", -3: "SDNN_EHIP", -4: "SDNN_EUNSUPPORTED",
                -5: "SDNN_EDEVICE"}
SDNN_TRAINABLE, SDNN_NO_COMPACTION, SDNN_DEBUG_CHECKS, SDNN_AUTOTUNE, SDNN_NO_SCHEDULE = 0x1, 0x2, 0x4, 0x8, 0x10
SDNN_EXEC_AUTO, SDNN_EXEC_EAGER, SDNN_EXEC_GRAPH, SDNN_EXEC_PERSISTENT, SDNN_EXEC_GRAPH_MERGED = 0, 1, 2, 3, 4
EXEC_NAMES = {"auto": 0, "eager": 1, "graph": 2, "persistent": 3, "graph_merged": 4}


class sdnn_desc(ctypes.Structure):
    _fields_ = [("n_neurons", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("k", ctypes.c_int32),
                ("clamp", ctypes.c_float), ("ckpt_every", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_rows", ctypes.c_int64)]


class sdnn_plan(ctypes.Structure):
    _fields_ = [("rows_per_tile", ctypes.c_int32), ("threads", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("tuned_us", ctypes.c_float)]


# (name, restype, argtypes) of every exported entry point
_P, _I32, _I64, _F, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
PROTOTYPES = [
    ("sdnn_workspace_size", _I32, [ctypes.POINTER(sdnn_desc), ctypes.POINTER(_SZ)]),
    ("sdnn_ckpt_size", _I32, [ctypes.POINTER(sdnn_desc), _I64, ctypes.POINTER(_SZ)]),
    ("sdnn_create", _I32, [ctypes.POINTER(sdnn_desc), _P, _P, _P, _P, _SZ, _P, ctypes.POINTER(_P)]),
    ("sdnn_set_exec", _I32, [_P, _I32]),
    ("sdnn_get_plan", _I32, [_P, ctypes.POINTER(sdnn_plan)]),
    ("sdnn_set_plan", _I32, [_P, ctypes.POINTER(sdnn_plan)]),
    ("sdnn_set_timing", _I32, [_P, _I32]),
    ("sdnn_kernel_time", _I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)]),
    ("sdnn_tune", _I32, [_P, _P, _I64, _P]),
    ("sdnn_forward", _I32, [_P, _P, _I64, _P, _I32, _P, _P, _P, _P, _P, _P]),
    ("sdnn_layer", _I32, [_P, _I32, _P, _I64, _P, _P]),
    ("sdnn_backward", _I32, [_P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("sdnn_layer_backward", _I32, [_P, _I32, _P, _P, _P, _I64, _P, _P, _P, _P]),
    ("sdnn_mse", _I32, [_P, _P, _I64, _P, _P, _P]),
    ("sdnn_mse_noalloc", _I32, [_P, _P, _I64, _P, _P, _P]),
    ("sdnn_schedule_host", _I32, [_P, _I32, _I32, _I32, _P, _P, _P]),
    ("sdnn_row_schedule_host", _I64, [_P, _I32, _I32, _P]),
    ("sdnn_check_device", _I32, [_P, _P]),
    ("sdnn_inject_device_error", _I32, [_P, _I32, _P]),
    ("sdnn_destroy", None, [_P]),
    ("sdnn_last_error", ctypes.c_char_p, []),
    ("sdnn_version", ctypes.c_char_p, []),
]

_lib: Optional[ctypes.CDLL] = None
_live_nets = weakref.WeakSet()      # nets not yet closed (unload() closes them first)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2004_10908_amd.build` "
                               "(or __graft_entry__.build()); there is no non-HIP fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in PROTOTYPES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def unload() -> None:
    """Close every open net and unload libsdnn.so (dlclose), so that its HIP code
    objects are unregistered now, while the HIP runtime (and a profiler attached to
    the process) is still alive, instead of during interpreter exit.  The library
    is loaded again by the next call that needs it."""
    global _lib
    for net in list(_live_nets):
        net.close()
    if _lib is not None:
        import _ctypes
        handle = _lib._handle
        _lib = None
        _ctypes.dlclose(handle)


class SdnnError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().sdnn_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _chk(status: int, where: str) -> None:
    if status != SDNN_OK:
        raise SdnnError(status, where)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_desc(n_neurons: int, n_layers: int, max_rows: int, clamp: float = 32.0, k: int = 32, ckpt_every: int = 0,
              flags: int = 0) -> sdnn_desc:
    return sdnn_desc(n_neurons, n_layers, k, clamp, ckpt_every, flags, max_rows)


# --------------------------------------------------------------------------- thin wrappers (same names as the C ABI)
def sdnn_workspace_size(desc: sdnn_desc) -> int:
    n = _SZ()
    _chk(lib().sdnn_workspace_size(ctypes.byref(desc), ctypes.byref(n)), "sdnn_workspace_size")
    return n.value


def sdnn_ckpt_size(desc: sdnn_desc, rows: int) -> int:
    n = _SZ()
    _chk(lib().sdnn_ckpt_size(ctypes.byref(desc), rows, ctypes.byref(n)), "sdnn_ckpt_size")
    return n.value


def sdnn_create(desc, idx, w, bias, workspace, ws_bytes=None, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    ws_bytes = workspace.numel() * workspace.element_size() if ws_bytes is None else ws_bytes
    _chk(lib().sdnn_create(ctypes.byref(desc), _ptr(idx), _ptr(w), _ptr(bias), _ptr(workspace), ws_bytes,
                           _stream(stream), ctypes.byref(h)), "sdnn_create")
    return h


def sdnn_set_exec(h, mode: int) -> None:
    _chk(lib().sdnn_set_exec(h, mode), "sdnn_set_exec")


def sdnn_get_plan(h) -> dict:
    p = sdnn_plan()
    _chk(lib().sdnn_get_plan(h, ctypes.byref(p)), "sdnn_get_plan")
    return {"rows_per_tile": p.rows_per_tile, "threads": p.threads, "grid": p.grid, "variant": p.variant,
            "tuned_us": p.tuned_us}


def sdnn_set_timing(h, enable: bool) -> None:
    _chk(lib().sdnn_set_timing(h, 1 if enable else 0), "sdnn_set_timing")


def sdnn_kernel_time(h):
    """(summed milliseconds, launches) of the timed persistent chain kernels since the last call."""
    ms, n = ctypes.c_double(0.0), _I32(0)
    _chk(lib().sdnn_kernel_time(h, ctypes.byref(ms), ctypes.byref(n)), "sdnn_kernel_time")
    return ms.value, n.value


def sdnn_set_plan(h, rows_per_tile: int, threads: int, variant: int) -> None:
    p = sdnn_plan(rows_per_tile=rows_per_tile, threads=threads, grid=0, variant=variant, tuned_us=0.0)
    _chk(lib().sdnn_set_plan(h, ctypes.byref(p)), "sdnn_set_plan")


def sdnn_tune(h, rows: int, y_sample=None, stream=None) -> None:
    _chk(lib().sdnn_tune(h, _ptr(y_sample), rows, _stream(stream)), "sdnn_tune")


def sdnn_forward(h, y0, rows, batch_off, n_batches, y_out, nz_rows, n_nz, ckpt=None, layer_rows=None,
                 stream=None) -> None:
    off_arr = None
    if batch_off is not None:
        off_arr = (ctypes.c_int64 * len(batch_off))(*[int(v) for v in batch_off])
    _chk(lib().sdnn_forward(h, _ptr(y0), rows, off_arr, n_batches, _ptr(y_out), _ptr(nz_rows), _ptr(n_nz),
                            _ptr(ckpt), _ptr(layer_rows), _stream(stream)), "sdnn_forward")


def sdnn_layer(h, layer, y_in, rows, y_out, stream=None) -> None:
    _chk(lib().sdnn_layer(h, layer, _ptr(y_in), rows, _ptr(y_out), _stream(stream)), "sdnn_layer")


def sdnn_backward(h, y0, rows, ckpt, nz_rows, n_nz, dy_out, dw, dbias, dy0=None, stream=None) -> None:
    _chk(lib().sdnn_backward(h, _ptr(y0), rows, _ptr(ckpt), _ptr(nz_rows), _ptr(n_nz), _ptr(dy_out), _ptr(dw),
                             _ptr(dbias), _ptr(dy0), _stream(stream)), "sdnn_backward")


def sdnn_layer_backward(h, layer, y_in, y_out, dy_out, rows, dw, dbias, dy_in=None, stream=None) -> None:
    _chk(lib().sdnn_layer_backward(h, layer, _ptr(y_in), _ptr(y_out), _ptr(dy_out), rows, _ptr(dw), _ptr(dbias),
                                   _ptr(dy_in), _stream(stream)), "sdnn_layer_backward")


def sdnn_mse(y, t, n, dy=None, loss=None, stream=None) -> None:
    _chk(lib().sdnn_mse(_ptr(y), _ptr(t), n, _ptr(dy), _ptr(loss), _stream(stream)), "sdnn_mse")


def sdnn_mse_noalloc(y, t, n, dy=None, loss=None, stream=None) -> None:
    _chk(lib().sdnn_mse_noalloc(_ptr(y), _ptr(t), n, _ptr(dy), _ptr(loss), _stream(stream)), "sdnn_mse_noalloc")


def sdnn_row_schedule_host(idx):
    """Bank-scheduled slot orders of the one-row-tile kernel for an int32 numpy array
    idx [L][N][k] -> (cost in LDS passes, perm uint8 [L][N][k])."""
    import numpy as np
    idx = np.ascontiguousarray(idx, np.int32)
    L, N, _ = idx.shape
    perm = np.zeros(idx.shape, np.uint8)
    cost = lib().sdnn_row_schedule_host(idx.ctypes.data_as(_P), N, L, perm.ctypes.data_as(_P))
    if cost < 0:
        raise SdnnError(int(cost), "sdnn_row_schedule_host")
    return int(cost), perm


def sdnn_schedule_host(idx, dmax: int = 44):
    """Host slot schedule for an int32 numpy array idx [L][N][k] -> (worst, ent, lane_neuron, steps)."""
    import numpy as np
    idx = np.ascontiguousarray(idx, np.int32)
    L, N, _ = idx.shape
    nblk = (N + 63) // 64
    ent = np.zeros((L, nblk * 64, dmax), np.uint32)
    ln = np.zeros((L, nblk * 64), np.int32)
    st = np.zeros((L, nblk), np.int32)
    worst = lib().sdnn_schedule_host(idx.ctypes.data_as(_P), N, L, dmax, ent.ctypes.data_as(_P),
                                     ln.ctypes.data_as(_P), st.ctypes.data_as(_P))
    if worst < 0:
        raise SdnnError(worst, "sdnn_schedule_host")
    return worst, ent, ln, st


def sdnn_check_device(h, stream=None) -> None:
    _chk(lib().sdnn_check_device(h, _stream(stream)), "sdnn_check_device")


def sdnn_inject_device_error(h, code: int, stream=None) -> None:
    _chk(lib().sdnn_inject_device_error(h, code, _stream(stream)), "sdnn_inject_device_error")


def sdnn_destroy(h) -> None:
    lib().sdnn_destroy(h)


def sdnn_version() -> str:
    return lib().sdnn_version().decode()


# --------------------------------------------------------------------------- owner object
class Net:
    """A created network: borrowed parameters + workspace + C handle."""

    def __init__(self, idx: torch.Tensor, w: torch.Tensor, bias: torch.Tensor, max_rows: int, clamp: float = 32.0,
                 ckpt_every: int = 0, flags: int = 0, exec_mode: str = "auto", stream=None):
        if idx.dim() != 3 or w.shape != idx.shape or bias.shape != idx.shape[:2]:
            raise ValueError("idx/w must be [L][N][k] and bias [L][N]")
        if not (idx.is_cuda and w.is_cuda and bias.is_cuda):
            raise ValueError("parameters must be device tensors")
        if idx.dtype != torch.int32 or w.dtype != torch.float32 or bias.dtype != torch.float32:
            raise ValueError("idx int32, w and bias float32")
        self.idx, self.w, self.bias = idx.contiguous(), w.contiguous(), bias.contiguous()
        L, N, k = idx.shape
        self.n_layers, self.n_neurons, self.k = L, N, k
        self.clamp, self.ckpt_every, self.flags, self.max_rows = clamp, ckpt_every, flags, max_rows
        self.desc = make_desc(N, L, max_rows, clamp, k, ckpt_every, flags)
        self.ws_bytes = sdnn_workspace_size(self.desc)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=idx.device)
        self.h = None
        self.h = sdnn_create(self.desc, self.idx, self.w, self.bias, self.workspace, self.ws_bytes, stream)
        _live_nets.add(self)
        self.set_exec(exec_mode)

    def set_exec(self, mode) -> None:
        sdnn_set_exec(self.h, EXEC_NAMES[mode] if isinstance(mode, str) else int(mode))

    @property
    def plan(self) -> dict:
        return sdnn_get_plan(self.h)

    def set_timing(self, enable: bool) -> None:
        sdnn_set_timing(self.h, enable)

    def kernel_time(self):
        return sdnn_kernel_time(self.h)

    def set_plan(self, rows_per_tile: int, threads: int, variant: int) -> dict:
        sdnn_set_plan(self.h, rows_per_tile, threads, variant)
        return self.plan

    def tune(self, rows: int, y_sample: Optional[torch.Tensor] = None, stream=None) -> dict:
        """Autotune the tile plan on `rows` rows: the first rows of y_sample (the
        workload's activations) when given, else all-ones rows."""
        if y_sample is not None:
            rows = min(rows, y_sample.shape[0])
            y_sample = y_sample[:rows].contiguous()
        sdnn_tune(self.h, rows, y_sample, stream)
        return self.plan

    def ckpt_numel(self, rows: int) -> int:
        return sdnn_ckpt_size(self.desc, rows) // 4

    def forward(self, y0: torch.Tensor, batch_off: Optional[Sequence[int]] = None, ckpt: bool = False,
                out: Optional[dict] = None, profile: bool = False, stream=None) -> dict:
        """Run sdnn_forward; returns dict(y, nz_rows, n_nz, ckpt, layer_rows) of device tensors."""
        rows = y0.shape[0]
        dev = y0.device
        o = {} if out is None else out
        if "y" not in o:
            o["y"] = torch.empty(rows, self.n_neurons, dtype=torch.float32, device=dev)
            o["nz_rows"] = torch.empty(max(rows, 1), dtype=torch.int32, device=dev)
            o["n_nz"] = torch.empty(1, dtype=torch.int32, device=dev)
            o["ckpt"] = torch.empty(max(self.ckpt_numel(rows), 1), dtype=torch.float32, device=dev) if ckpt else None
            o["layer_rows"] = torch.empty(self.n_layers + 1, dtype=torch.int32, device=dev) if profile else None
        nb = 1 if batch_off is None else len(batch_off) - 1
        sdnn_forward(self.h, y0, rows, batch_off, nb, o["y"], o["nz_rows"], o["n_nz"], o["ckpt"], o["layer_rows"],
                     stream)
        return o

    def layer(self, layer: int, y_in: torch.Tensor, y_out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if y_out is None:
            y_out = torch.empty_like(y_in)
        sdnn_layer(self.h, layer, y_in, y_in.shape[0], y_out, stream)
        return y_out

    def backward(self, y0, ckpt, nz_rows, n_nz, dy_out, want_dy0: bool = True, stream=None):
        dev = y0.device
        dw = torch.empty_like(self.w)
        db = torch.empty_like(self.bias)
        dy0 = torch.empty_like(y0) if want_dy0 else None
        sdnn_backward(self.h, y0, y0.shape[0], ckpt, nz_rows, n_nz, dy_out, dw, db, dy0, stream)
        return dw, db, dy0

    def layer_backward(self, layer, y_in, y_out, dy_out, want_dy_in=True, stream=None):
        dw = torch.empty_like(self.w[layer])
        db = torch.empty_like(self.bias[layer])
        dy_in = torch.empty_like(y_in) if want_dy_in else None
        sdnn_layer_backward(self.h, layer, y_in, y_out, dy_out, y_in.shape[0], dw, db, dy_in, stream)
        return dw, db, dy_in

    def check_device(self, stream=None) -> None:
        sdnn_check_device(self.h, stream)

    def inject_device_error(self, code: int, stream=None) -> None:
        sdnn_inject_device_error(self.h, code, stream)

    def close(self) -> None:
        if self.h is not None:
            sdnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mse(y: torch.Tensor, t: torch.Tensor, stream=None):
    """(loss [1] device tensor, dy) of the mean squared error, computed by the library."""
    n = y.numel()
    dy = torch.empty_like(y)
    loss = torch.empty(257, dtype=torch.float32, device=y.device)
    sdnn_mse(y, t, n, dy, loss, stream)
    return loss[:1], dy
