"""Multi-rate pipeline (Methods, "Multi-rate extension"): the DM grid split into bands by
scrunch factor, one plan per band on a time-scrunched (and, for binary and graded modes,
re-encoded) copy of the filterbank, candidates merged across bands.  Argument marshalling and
scheduling of library calls only; scrunch, encode, tree and detection run in libsnd."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from .detect import Detector
from .plan import Plan, _stream_handle, encode, encode_bits


def scrunch_factors(freqs, dms, tsamp_s: float, s_max: int = 16) -> np.ndarray:
    """int32 [ndm] scrunch factor of each trial DM (snd_scrunch_factors)."""
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.empty(d.size, dtype=np.int32)
    capi.check(capi.lib().snd_scrunch_factors(f.size, f.ctypes.data_as(C.c_void_p), float(tsamp_s), d.size,
                                              d.ctypes.data_as(C.c_void_p), int(s_max),
                                              out.ctypes.data_as(C.c_void_p)))
    return out


def scrunch(z, s: int, out=None, stream=None):
    """float32 [nchan][n] -> [nchan][n // s] time scrunch on the GPU (snd_scrunch)."""
    import torch
    if z.dtype != torch.float32 or z.stride(1) != 1:
        raise TypeError("z must be float32 with unit inner stride")
    nchan, n = z.shape
    if out is None:
        out = torch.empty((nchan, n // s), dtype=torch.float32, device=z.device)
    capi.check(capi.lib().snd_scrunch(C.c_void_p(z.data_ptr()), z.stride(0), nchan, n, int(s),
                                      C.c_void_p(out.data_ptr()), out.stride(0), _stream_handle(stream, z.device)))
    return out


def merge_candidates(cands, dm_tol: float = 20.0, t_tol_ms: float = 200.0) -> list:
    """Cross-band merge (snd_merge_candidates) of dicts with dm, t_ms, snr, band, k, t, width, npix."""
    n = len(cands)
    arr = (capi.BandCandidate * max(n, 1))()
    for i, c in enumerate(cands):
        arr[i].dm, arr[i].t_ms, arr[i].snr = c["dm"], c["t_ms"], c["snr"]
        arr[i].band, arr[i].dm_index, arr[i].width = c.get("band", 0), c.get("k", 0), c.get("width", 0)
        arr[i].t, arr[i].npix = c.get("t", 0), c.get("npix", 0)
    out = (capi.BandCandidate * max(n, 1))()
    cnt = C.c_int64()
    capi.check(capi.lib().snd_merge_candidates(n, arr, float(dm_tol), float(t_tol_ms), out, C.byref(cnt)))
    return [dict(dm=out[i].dm, t_ms=out[i].t_ms, snr=out[i].snr, band=out[i].band, k=out[i].dm_index,
                 width=out[i].width, t=out[i].t, npix=out[i].npix) for i in range(cnt.value)]


class MultiRate:
    """One plan and detector per scrunch band of the DM grid.  `thresholds` encode binary /
    graded inputs (in sigma of the z-scored filterbank, applied again after each scrunch)."""

    def __init__(self, freqs, dms, tsamp_s: float, nsamp: int, *, mode: str = "float", s_max: int = 16,
                 thresholds=None, widths=(1, 2, 4, 8, 16, 32, 64), threshold: float = 7.0, sigma_min: float = 0.0,
                 n_min: int = 10, dm_tol: float = 20.0, t_tol_ms: float = 200.0, device="cuda", bit_input=False,
                 detect_kw=None, **plan_kw):
        """detect_kw: further Detector arguments for every band (e.g. n_base_widths and
        width_alpha for the DM-scaled width set, sigma)."""
        self.freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        self.dms = np.ascontiguousarray(dms, dtype=np.float64)
        self.tsamp_s, self.nsamp, self.mode = tsamp_s, int(nsamp), mode
        self.thresholds = None if thresholds is None else list(thresholds)
        if mode != "float" and not self.thresholds:
            raise ValueError("binary and graded modes need encoder thresholds")
        self.bit_input = bool(bit_input) and mode == "binary"
        self.dm_tol, self.t_tol_ms = dm_tol, t_tol_ms
        self.factors = scrunch_factors(self.freqs, self.dms, tsamp_s, s_max)
        self.bands = []
        for s in sorted(set(int(v) for v in self.factors)):
            idx = np.flatnonzero(self.factors == s)
            kw = dict(plan_kw)
            if self.bit_input:
                kw["in_dtype"] = "bits"
            plan = Plan(self.freqs, self.dms[idx], tsamp_s * s, self.nsamp // s, mode=mode, **kw)
            plan.upload(device)
            det = Detector(plan, widths=widths, threshold=threshold, sigma_min=sigma_min, n_min=n_min,
                           device=device, **(detect_kw or {}))
            self.bands.append(dict(s=s, idx=idx, plan=plan, det=det))

    def band_input(self, z, s: int):
        """The band's tree input from the z-scored float32 filterbank z."""
        zs = z if s == 1 else scrunch(z, s)
        if self.mode == "float":
            return zs
        if self.bit_input:
            return encode_bits(zs, self.thresholds[0])
        return encode(zs, self.thresholds)

    def run(self, z):
        """Candidates of the block z [nchan][nsamp] (float32, z-scored), merged across bands, and
        the per-band candidate lists."""
        per_band = []
        allc = []
        tms = self.tsamp_s * 1e3
        for bi, b in enumerate(self.bands):
            x = self.band_input(z, b["s"])
            out = b["plan"].execute(x)
            cands = b["det"].run(out)
            mapped = [dict(dm=float(self.dms[b["idx"][c["k"]]]), t_ms=c["t"] * b["s"] * tms, snr=c["snr"], band=bi,
                           k=int(b["idx"][c["k"]]), width=c["width"], t=c["t"], npix=c["npix"]) for c in cands]
            per_band.append(mapped)
            allc.extend(mapped)
        return merge_candidates(allc, self.dm_tol, self.t_tol_ms), per_band
