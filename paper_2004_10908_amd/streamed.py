"""Forward with the parameters in host memory, streamed through device slots.

The paper's GPUs (8 GB) could not hold the largest networks, so it decomposes the
model and copies its partitions to the GPU while earlier ones compute (paper,
section "Large Sparse Neural Network Inference").  MI355X holds every workload's
weights, so the resident path never streams; this is the out-of-core form for
nets larger than HBM or for sharing the GPU with other work.

Layer l's ids, weights and bias (pinned host memory) are copied into device slot
l mod S on a copy stream (DMA engines, no compute units) while the compute
stream runs layer l-1 from the other slot.  The copy into a slot waits for the
layer that last used it; the layer waits for its copy.  Each slot has its own
net (created with SDNN_NO_SCHEDULE, so the kernels read the slot's parameters on
every call) and every layer runs over all rows (no work lists); a row whose
activations become all zero stays zero, because every bias must be <= 0 here
exactly as for compaction, so results equal the resident forward of the same
kernel family.
"""
from typing import List

import torch

from .sdnn import SDNN_NO_COMPACTION, SDNN_NO_SCHEDULE, Net


class StreamedForward:
    """``idx_h`` int32 [L][N][K], ``w_h`` fp32 [L][N][K], ``b_h`` fp32 [L][N]: pinned host
    tensors (``pin_memory()``); ``slots`` device copies of one layer each (>= 2)."""

    def __init__(self, idx_h: torch.Tensor, w_h: torch.Tensor, b_h: torch.Tensor, max_rows: int,
                 clamp: float = 32.0, slots: int = 2, device="cuda:0"):
        if not (idx_h.is_pinned() and w_h.is_pinned() and b_h.is_pinned()):
            raise ValueError("host parameters must be pinned (pin_memory())")
        if idx_h.dim() != 3 or w_h.shape != idx_h.shape or b_h.shape != idx_h.shape[:2]:
            raise ValueError("idx/w must be [L][N][k] and bias [L][N]")
        if slots < 2:
            raise ValueError("at least two slots (one computing, one filling)")
        if float(b_h.max()) > 0.0:
            raise ValueError("streaming needs every bias <= 0 (dead rows stay dead)")
        self.idx_h, self.w_h, self.b_h = idx_h, w_h, b_h
        L, N, K = idx_h.shape
        self.n_layers, self.n_neurons = L, N
        self.S = min(slots, L) if L > 1 else 1
        dev = torch.device(device)
        self.slot = []
        for s in range(self.S):
            l = min(s, L - 1)   # a valid layer in every slot before its net is created
            self.slot.append((idx_h[l:l + 1].to(dev), w_h[l:l + 1].to(dev), b_h[l:l + 1].to(dev)))
        flags = SDNN_NO_SCHEDULE | SDNN_NO_COMPACTION
        self.nets: List[Net] = [Net(i, w, b, max_rows=max_rows, clamp=clamp, flags=flags, exec_mode="eager")
                                for (i, w, b) in self.slot]
        self.copy_stream = torch.cuda.Stream(device=dev)     # default priority
        self.ev_copied = [torch.cuda.Event() for _ in range(L)]
        self.ev_used = [torch.cuda.Event() for _ in range(L)]
        self.act = None

    @property
    def slot_bytes(self) -> int:
        i, w, b = self.slot[0]
        return self.S * (i.numel() * 4 + w.numel() * 4 + b.numel() * 4)

    def run(self, y0: torch.Tensor, y_out: torch.Tensor) -> None:
        """Y_L of every row of y0 ([rows][N]) into y_out; asynchronous on the current stream."""
        rows = y0.shape[0]
        if y_out.shape != y0.shape:
            raise ValueError("y_out must have y0's shape")
        if self.act is None or self.act.shape[0] < rows:
            self.act = torch.empty_like(y0)
        L, S = self.n_layers, self.S
        comp = torch.cuda.current_stream()
        self.copy_stream.wait_stream(comp)        # y0 and the slots are ready to use
        for l in range(L):
            s = l % S
            with torch.cuda.stream(self.copy_stream):
                if l >= S:
                    self.copy_stream.wait_event(self.ev_used[l - S])    # the slot's last layer is done
                i, w, b = self.slot[s]
                i.copy_(self.idx_h[l:l + 1], non_blocking=True)
                w.copy_(self.w_h[l:l + 1], non_blocking=True)
                b.copy_(self.b_h[l:l + 1], non_blocking=True)
                self.ev_copied[l].record(self.copy_stream)
            comp.wait_event(self.ev_copied[l])
            # ping-pong so that layer L-1 writes y_out
            dst = y_out if (L - 1 - l) % 2 == 0 else self.act[:rows]
            src = y0 if l == 0 else (y_out if (L - l) % 2 == 0 else self.act[:rows])
            self.nets[s].layer(0, src, dst)
            self.ev_used[l].record(comp)

    def close(self) -> None:
        for n in self.nets:
            n.close()
