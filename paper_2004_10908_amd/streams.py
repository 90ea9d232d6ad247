"""Batches of one forward spread over several HIP streams, issued directly or captured.

The paper's GPU task graph puts independent operations on a pool of streams and
compares a graph captured from those streams with an explicitly built one, for
one to eight streams (paper, section "Large Sparse Neural Network Inference",
the experiment on the number of streams; the capture algorithm of the GPU
task-graph section).  Here the independent work is the batches: batch b's whole
layer chain (one kernel node per layer, in eager mode) goes to stream b mod K.
Nodes of one chain depend on each other in issue order; chains of different
batches share nothing, so stream order is the only dependency the launches need.

Each stream has its own net (its own workspace: ping-pong rows, work lists,
counters) over the same borrowed parameters, so chains on different streams never
touch the same scratch memory.  The captured form records exactly the same
launches under stream capture (the extra streams fork from the capturing stream
through events and join back) and replays them as one graph.  Every form computes
the same per-row arithmetic as ``Net.forward``, so outputs are bitwise equal.
"""
from typing import List, Optional, Sequence

import torch

from .sdnn import Net, sdnn_forward


class StreamForward:
    """Forward of fixed batches round-robin over ``n_streams`` streams.

    ``batch_off``: non-decreasing row offsets from 0 to rows (batch b = rows
    off[b] .. off[b+1]-1).  ``capture``: record the launches once as one graph
    and replay it (re-recorded when the input or output buffer changes).
    """

    def __init__(self, idx: torch.Tensor, w: torch.Tensor, bias: torch.Tensor, batch_off: Sequence[int],
                 n_streams: int, clamp: float = 32.0, flags: int = 0, capture: bool = False):
        self.off: List[int] = [int(v) for v in batch_off]
        nb = len(self.off) - 1
        if nb < 1 or self.off[0] != 0 or any(self.off[i + 1] < self.off[i] for i in range(nb)):
            raise ValueError("batch offsets must run non-decreasing from 0")
        if n_streams < 1:
            raise ValueError("n_streams must be >= 1")
        self.n_batches = nb
        self.k = min(n_streams, nb)
        sizes = [self.off[b + 1] - self.off[b] for b in range(nb)]
        self.nets = [Net(idx, w, bias, max_rows=max(1, max(sizes[b] for b in range(s, nb, self.k))), clamp=clamp,
                         flags=flags, exec_mode="eager") for s in range(self.k)]
        # default-priority streams (no priority other than the default anywhere)
        self.streams = [torch.cuda.Stream(device=idx.device) for _ in range(self.k)]
        dev = idx.device
        self.nz = [torch.empty(max(s, 1), dtype=torch.int32, device=dev) for s in sizes]
        self.n_nz = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.capture = capture
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.key = None

    @property
    def workspace_bytes(self) -> int:
        return sum(n.ws_bytes for n in self.nets)

    def _issue(self, y0: torch.Tensor, y_out: torch.Tensor) -> None:
        cur = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(cur)
        for b in range(self.n_batches):
            lo, hi = self.off[b], self.off[b + 1]
            if hi == lo:
                continue
            k = b % self.k
            sdnn_forward(self.nets[k].h, y0[lo:hi], hi - lo, None, 1, y_out[lo:hi], self.nz[b],
                         self.n_nz[b:b + 1], stream=self.streams[k])
        for s in self.streams:
            cur.wait_stream(s)

    def run(self, y0: torch.Tensor, y_out: torch.Tensor) -> None:
        """Y_L of every row into y_out ([rows][N], rows = off[-1]); asynchronous."""
        if y0.shape[0] != self.off[-1] or y_out.shape != y0.shape:
            raise ValueError("y0 and y_out must be [rows][N] with rows = the last batch offset")
        if not self.capture:
            self._issue(y0, y_out)
            return
        key = (y0.data_ptr(), y_out.data_ptr())
        if self.graph is None or key != self.key:
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream(device=y0.device)
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(g, stream=side):
                self._issue(y0, y_out)
            torch.cuda.current_stream().wait_stream(side)
            self.graph, self.key = g, key
        self.graph.replay()

    def nz_rows(self) -> torch.Tensor:
        """Ascending global ids of the nonzero output rows (synchronizes)."""
        counts = self.n_nz.cpu().tolist()
        parts = [self.nz[b][:counts[b]].long() + self.off[b] for b in range(self.n_batches) if counts[b] > 0]
        if not parts:
            return torch.empty(0, dtype=torch.int64, device=self.n_nz.device)
        return torch.cat(parts)

    def close(self) -> None:
        self.graph = None
        for n in self.nets:
            n.close()
