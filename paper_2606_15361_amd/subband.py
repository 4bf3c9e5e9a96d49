"""Approximate (coarse-DM) sub-band dedispersion, a comparison baseline (snd_subband_combine).

Step one runs an SND float plan per sub-band of adjacent channels over a coarse DM grid (every
coarse_step-th fine DM in increasing order), each channel at its delay relative to the band's
top frequency; step two sums, for every fine DM, the sub-bands' rows of the nearest coarse DM at
or below it, each shifted by its top channel's extra sweep.  Host orchestration and argument
marshalling only: both steps run in libsnd's kernels.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from .batch import Batch
from .plan import Plan, _stream_handle


class SubbandApprox:
    """freqs [nchan] (any order; sub-bands are runs of nsub-th of the channels in that order),
    dms [ndm] fine trial DMs, nsamp input samples per block."""

    def __init__(self, freqs, dms, tsamp_s: float, nsamp: int, *, nsub: int = 32, coarse_step: int = 8,
                 branching: int = 4, cluster: int = 4, device="cuda"):
        import torch
        f = np.ascontiguousarray(freqs, dtype=np.float64)
        d = np.ascontiguousarray(dms, dtype=np.float64)
        if f.size % nsub:
            raise ValueError("nsub must divide the channel count")
        m = f.size // nsub
        self.device = torch.device(device)
        self.nsub, self.m, self.ndm, self.nsamp = nsub, m, d.size, int(nsamp)
        ftop = float(f.max())
        self.coarse = np.unique(d)[::max(1, int(coarse_step))]
        # every fine DM takes the largest coarse DM at or below it
        self.coarse_row = (np.searchsorted(self.coarse, d, side="right") - 1).astype(np.int32)
        # delays of the whole band at the fine DMs (the library's own table; fref = top)
        fine = Plan(f, d, tsamp_s, self.nsamp, mode="float", branching=branching, cluster=cluster)
        dF = fine.delays()
        self.plans, tops = [], []
        for s in range(nsub):
            fs = f[s * m:(s + 1) * m]
            self.plans.append(Plan(fs, self.coarse, tsamp_s, self.nsamp, mode="float", branching=branching,
                                   cluster=cluster, fref=ftop))
            tops.append(s * m + int(np.argmax(fs)))
        dC = [p.delays() for p in self.plans]  # [ncoarse][m] per sub-band, relative to the top
        offs = np.empty((d.size, nsub), dtype=np.int64)
        for s in range(nsub):
            top_local = tops[s] - s * m
            offs[:, s] = dF[:, tops[s]] - dC[s][self.coarse_row, top_local]
        if offs.min() < 0:
            raise ValueError("a fine DM below its coarse DM")
        self.offsets = np.ascontiguousarray(offs, dtype=np.int32)
        self.n_valid = np.array([p.n_out for p in self.plans], dtype=np.int64)
        self.n_out = int(np.min(self.n_valid[None, :] - offs))
        if self.n_out < 1:
            raise ValueError("block too short for the sub-band sweeps")
        self.batch = Batch(self.plans, device)
        self.planes = [p.empty_output(self.device) for p in self.plans]
        nb = C.c_int64()
        capi.check(capi.lib().snd_subband_workspace_bytes(self.ndm, nsub, C.byref(nb)))
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.inputs_per_sample = nsub * (self.coarse.size * m) / self.ndm + nsub  # per fine DM row

    def empty_output(self):
        import torch
        pitch = (self.n_out + 63) // 64 * 64
        return torch.empty((self.ndm, pitch), dtype=torch.float32, device=self.device)[:, : self.n_out]

    def execute(self, x, out=None, stream=None):
        """x float32 [nchan][>= nsamp] on the device -> [ndm][n_out] float32."""
        if out is None:
            out = self.empty_output()
        self.batch.execute([x[s * self.m:(s + 1) * self.m] for s in range(self.nsub)], self.planes, stream=stream)
        ptrs = (C.c_void_p * self.nsub)(*[y.data_ptr() for y in self.planes])
        pit = (C.c_int64 * self.nsub)(*[y.stride(0) for y in self.planes])
        nv = (C.c_int64 * self.nsub)(*[int(v) for v in self.n_valid])
        capi.check(capi.lib().snd_subband_combine(
            self.ndm, self.nsub, ptrs, pit, nv, int(self.coarse.size),
            self.coarse_row.ctypes.data_as(C.c_void_p), self.offsets.ctypes.data_as(C.c_void_p),
            C.c_void_p(out.data_ptr()), out.stride(0), self.n_out, C.c_void_p(self._ws.data_ptr()),
            self._ws.numel(), _stream_handle(stream, self.device)))
        return out
