"""FDMT baseline with the no-smear initialisation (snd_fdmt_*).  Argument marshalling only; the
merges run in libsnd."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from .plan import _stream_handle


class Fdmt:
    """One FDMT shape: channels, sampling, maximum DM and block length.  Tables and workspace
    live on `device`."""

    def __init__(self, freqs, chan_bw_mhz: float, tsamp_s: float, dm_max: float, nsamp: int, device="cuda"):
        import torch
        f = np.ascontiguousarray(freqs, dtype=np.float64)
        h = C.c_void_p()
        capi.check(capi.lib().snd_fdmt_create(f.size, f.ctypes.data_as(C.c_void_p), float(chan_bw_mhz),
                                              float(tsamp_s), float(dm_max), int(nsamp), C.byref(h)))
        self._h = h
        nd, no, tb, wb = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        step = C.c_double()
        capi.check(capi.lib().snd_fdmt_query(h, C.byref(nd), C.byref(no), C.byref(tb), C.byref(wb), C.byref(step)))
        self.n_delays, self.n_out, self.dm_per_delay = nd.value, no.value, step.value
        self.nchan, self.nsamp = f.size, int(nsamp)
        self.workspace_bytes = wb.value
        self.table_rows = tb.value // 16  # output rows over all merges (4 int32 words each)
        self._tables = torch.empty(max(tb.value, 4), dtype=torch.uint8, device=device)
        capi.check(capi.lib().snd_fdmt_upload(h, C.c_void_p(self._tables.data_ptr()), self._tables.numel(),
                                              _stream_handle(None, self._tables.device)))
        self._ws = torch.empty(max(wb.value, 4), dtype=torch.uint8, device=device)

    def dms(self) -> np.ndarray:
        return np.arange(self.n_delays) * self.dm_per_delay

    def execute(self, x, out=None, stream=None):
        """float32 [nchan][nsamp] -> float32 [n_delays][nsamp] (rows valid for t < n_out)."""
        import torch
        if x.dtype != torch.float32 or x.stride(1) != 1 or x.shape[0] != self.nchan or x.shape[1] < self.nsamp:
            raise ValueError("x must be float32 [nchan][>= nsamp] with unit inner stride")
        if out is None:
            out = torch.empty((self.n_delays, self.nsamp), dtype=torch.float32, device=x.device)
        capi.check(capi.lib().snd_fdmt_execute(self._h, C.c_void_p(x.data_ptr()), x.stride(0),
                                               C.c_void_p(out.data_ptr()), out.stride(0),
                                               C.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                               _stream_handle(stream, x.device)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                capi.lib().snd_fdmt_destroy(h)
            except Exception:
                pass
            self._h = None
