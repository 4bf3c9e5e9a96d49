"""Batched execution of several beams (each with its own plan) through snd_batch_execute:
one grid per (stage, kernel class).  Argument marshalling only."""

from __future__ import annotations

import ctypes as C

from . import _capi as capi
from .plan import Plan, _stream_handle, row_pitch


def _arr(ctype, values):
    return (ctype * len(values))(*values)


def records_bytes(plans) -> tuple:
    """(device record bytes, number of grids) for a batch of these plans."""
    hs = _arr(C.c_void_p, [p.handle.value for p in plans])
    b, n = C.c_int64(), C.c_int32()
    capi.check(capi.lib().snd_batch_records_bytes(len(plans), hs, C.byref(b), C.byref(n)))
    return b.value, n.value


class Batch:
    """A fixed set of beams.  Owns the record buffer and one workspace per beam."""

    def __init__(self, plans, device="cuda"):
        import torch
        self.plans = list(plans)
        self.device = torch.device(device)
        for p in self.plans:
            if p._tables is None:
                p.upload(self.device)
        nb, self.n_launches = records_bytes(self.plans)
        self.records = torch.empty(max(256, nb), dtype=torch.uint8, device=self.device)
        self.workspaces = [torch.empty(max(256, p.info["workspace_bytes"]), dtype=torch.uint8, device=self.device)
                           for p in self.plans]

    def execute(self, inputs, outputs, n_run=None, stream=None) -> int:
        """Run every beam: inputs[i] [nchan][>= nsamp], outputs[i] [ndm][>= n_out] (or >= n_run[i]).
        Returns the number of grids launched."""
        n = len(self.plans)
        if len(inputs) != n or len(outputs) != n:
            raise ValueError("one input and one output per beam")
        for p, x, y in zip(self.plans, inputs, outputs):
            if x.dim() != 2 or x.shape[0] != p.nchan or x.stride(1) != 1:
                raise ValueError("input must be [nchan][T] with unit time stride")
            if y.dim() != 2 or y.shape[0] != p.ndm or y.stride(1) != 1 or y.dtype != p.out_dtype:
                raise ValueError("output must be [ndm][T] of the plan's output dtype")
        hs = _arr(C.c_void_p, [p.handle.value for p in self.plans])
        ins = _arr(C.c_void_p, [x.data_ptr() for x in inputs])
        inp = _arr(C.c_int64, [row_pitch(x, p.in_dtype) for p, x in zip(self.plans, inputs)])
        outs = _arr(C.c_void_p, [y.data_ptr() for y in outputs])
        outp = _arr(C.c_int64, [y.stride(0) for y in outputs])
        wss = _arr(C.c_void_p, [w.data_ptr() for w in self.workspaces])
        wsb = _arr(C.c_int64, [w.numel() for w in self.workspaces])
        nr = None if n_run is None else _arr(C.c_int64, [int(v) for v in n_run])
        nl = C.c_int32()
        capi.check(capi.lib().snd_batch_execute(n, hs, ins, inp, outs, outp, wss, wsb, nr,
                                                C.c_void_p(self.records.data_ptr()), self.records.numel(),
                                                _stream_handle(stream, self.device), C.byref(nl)))
        return nl.value
