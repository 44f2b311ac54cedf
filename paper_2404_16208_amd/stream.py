"""Streaming execution: a long input stream passes through one or more
instances chunk by chunk (GPU-RANC Sec. V names streaming execution as the
next step; its applications run thousands of ticks through one instance,
Table I).

Per chunk of k ticks, on torch streams of default priority:
  - upload stream: the chunk's inputs go from pinned host memory to one of
    two device input buffers (after the chunk that last used the buffer ran);
  - the handle's stream: the k ticks run (a captured tick loop per input
    buffer), then ranc_copy_raster packs the chunk's output-bus spikes of every
    sample into one of two device raster buffers (after the previous drain of
    that buffer finished);
  - drain stream: the packed raster goes to one of two pinned host buffers;
  - host: while the GPU runs chunk i, the caller's consumer gets chunk i - 1's
    raster (a numpy view of the pinned buffer, valid during the call).
Every tick of the simulation and the packing run in the library's kernels;
this module only orders copies and launches.
"""
from __future__ import annotations

import numpy as np

from .ranc import RancNet


class Streamer:
    """Double-buffered streaming of a RancNet in chunks of at most ``chunk``
    ticks (<= the handle's max_ticks_per_call)."""

    def __init__(self, g: RancNet, chunk: int, layout: str = "sample", graph: bool = True):
        import torch

        if not 1 <= chunk <= g.RT:
            raise ValueError(f"chunk {chunk} outside [1, max_ticks_per_call={g.RT}]")
        self.g, self.chunk, self.layout, self.graph = g, chunk, layout, graph
        self.dev = g.stream.device
        self.up = torch.cuda.Stream(device=self.dev)
        self.down = torch.cuda.Stream(device=self.dev)
        self.nbytes = g.raster_bytes(chunk, layout)
        n = max(self.nbytes, 8)
        self.out_dev = [torch.empty(n, dtype=torch.uint8, device=self.dev) for _ in range(2)]
        self.out_host = [torch.empty(n, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self._in = {}

    def _in_buf(self, shape, slot):
        import torch
        key = (tuple(shape), slot)
        if key not in self._in:   # fixed addresses, so captured tick loops are reused
            self._in[key] = torch.empty(shape, dtype=torch.int32, device=self.dev)
        return self._in[key]

    def _words(self, host, k):
        nb = self.g.raster_bytes(k, self.layout)
        a = host[:nb].numpy()
        if self.layout == "sample":
            return a.view(np.uint32).reshape(k, self.g.S, -1)
        return a.view(np.uint64).reshape(k, -1, (self.g.S + 63) // 64)

    def run(self, inputs, num_ticks: int, consume=None):
        """Advance by num_ticks ticks. ``inputs``: None or a pinned host int32
        tensor [S, >= num_ticks, C_in, A/32] (tick 0 = the handle's current
        tick). ``consume(tick_begin, words)`` receives each chunk's output
        raster (layout as ranc_copy_raster) while the next chunk runs."""
        import torch

        g = self.g
        main = g.stream
        t_start = g.tick
        chunks = [(t0, min(self.chunk, num_ticks - t0)) for t0 in range(0, num_ticks, self.chunk)]
        ran = [None, None]      # main-stream event: the chunk that last read input buffer b has run
        drained = [None, None]  # drain-stream event: raster buffer b is free again
        pending = None          # (tick_begin, k, buffer) of the chunk the host consumes next

        def upload(i):
            t0, k = chunks[i]
            b = i % 2
            buf = self._in_buf((g.S, k) + tuple(inputs.shape[2:]), b if k == self.chunk else 2)
            with torch.cuda.stream(self.up):
                if ran[b] is not None:
                    self.up.wait_event(ran[b])
                buf.copy_(inputs[:, t0:t0 + k], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.up)
            return buf, ev

        nxt = upload(0) if inputs is not None else None
        for i, (t0, k) in enumerate(chunks):
            b = i % 2
            cur = nxt
            if inputs is not None and i + 1 < len(chunks):
                nxt = upload(i + 1)
            if cur is not None:
                main.wait_event(cur[1])
            g.run(cur[0] if cur is not None else None, k, graph=self.graph)
            ev = torch.cuda.Event()
            ev.record(main)
            ran[b] = ev
            if drained[b] is not None:
                main.wait_event(drained[b])
            g.copy_raster(t_start + t0, t_start + t0 + k, self.out_dev[b], self.layout)
            packed = torch.cuda.Event()
            packed.record(main)
            nb = g.raster_bytes(k, self.layout)
            with torch.cuda.stream(self.down):
                self.down.wait_event(packed)
                if nb:
                    self.out_host[b][:nb].copy_(self.out_dev[b][:nb], non_blocking=True)
                dev = torch.cuda.Event()
                dev.record(self.down)
            drained[b] = dev
            if pending is not None:
                pt, pk, pb = pending
                drained[pb].synchronize()
                if consume is not None:
                    consume(t_start + pt, self._words(self.out_host[pb], pk))
            pending = (t0, k, b)
        if pending is not None:
            pt, pk, pb = pending
            drained[pb].synchronize()
            if consume is not None:
                consume(t_start + pt, self._words(self.out_host[pb], pk))
        return g
