"""Matched filter and candidate stage (snd_snr_plane / snd_detect) from Python."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from .plan import _stream_handle


class Detector:
    """Boxcar S/N and candidate extraction for the DM-time planes of one plan."""

    def __init__(self, plan, widths=(1, 2, 4, 8, 16, 32, 64), threshold: float = 7.0, sigma_min: float = 0.0,
                 closing_radius: int = 4, n_min: int = 10, max_pixels: int = 1 << 20, device="cuda",
                 n_base_widths: int = 0, width_alpha: float = 0.0, sigma: str = "std", label: str = "host"):
        """n_base_widths > 0 selects the DM-scaled width set: each row uses the first
        n_base_widths widths and the further ones up to width_alpha times its dispersive sweep
        (the paper: widths 1..1024 in powers of two, n_base_widths 4, width_alpha 0.1).
        sigma: "std" (row standard deviation) or "mad" (median absolute deviation, scaled).
        label: "host" or "device": where run() closes and labels the thresholded cells."""
        import torch
        self.plan = plan
        self._w = np.ascontiguousarray(widths, dtype=np.int32)
        d = capi.DetectDesc()
        d.widths = self._w.ctypes.data_as(C.POINTER(C.c_int32))
        d.nwidths = self._w.size
        d.threshold = threshold
        d.sigma_min = sigma_min
        d.closing_radius = closing_radius
        d.n_min = n_min
        d.n_base_widths = n_base_widths
        d.width_alpha = width_alpha
        if sigma not in ("std", "mad"):
            raise ValueError('sigma must be "std" or "mad"')
        d.sigma_estimator = 1 if sigma == "mad" else 0
        if label not in ("host", "device"):
            raise ValueError('label must be "host" or "device"')
        d.label_on_device = 1 if label == "device" else 0
        d.max_pixels = max_pixels
        self.desc = d
        nb = C.c_int64()
        capi.check(capi.lib().snd_detect_workspace(plan.handle, C.byref(d), C.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.widths = [int(w) for w in self._w]
        self.npixels = 0
        self._cap = 1 << 16
        self._buf = (capi.Candidate * self._cap)()

    def row_stats(self):
        """(mu, sigma) per DM row from the last run (float64 tensors on the device)."""
        n = self.plan.ndm
        v = self.ws[256:256 + 16 * n].view(__import__("torch").float64).view(n, 2)
        return v[:, 0], v[:, 1]

    def snr_plane(self, plane, stream=None):
        """(snr float32 [ndm][n_out], width index int8 [ndm][n_out])."""
        import torch
        n = self.plan.n_out
        snr = torch.empty((self.plan.ndm, n), dtype=torch.float32, device=plane.device)
        widx = torch.empty((self.plan.ndm, n), dtype=torch.int8, device=plane.device)
        capi.check(capi.lib().snd_snr_plane(self.plan.handle, C.c_void_p(plane.data_ptr()), plane.stride(0),
                                            C.byref(self.desc), C.c_void_p(snr.data_ptr()), snr.stride(0),
                                            C.c_void_p(widx.data_ptr()), widx.stride(0),
                                            C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                            _stream_handle(stream, plane.device)))
        return snr, widx

    def launch(self, plane, stage_cells: int = 1 << 18, stream=None):
        """Enqueue this plane's detection and the read-back of up to stage_cells thresholded
        cells into a page-locked host buffer (snd_detect_launch); returns a ticket for
        collect().  Launches on one stream may follow each other (the workspace is reused in
        stream order); the plane must stay unchanged until collect() returns, since collect()
        detects it again with run() when the staged cells do not hold them all."""
        import torch
        dev = plane.device
        nb = capi.DETECT_STAGE_HEADER + capi.DETECT_CELL_BYTES * int(stage_cells)
        stage = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
        capi.check(capi.lib().snd_detect_launch(self.plan.handle, C.c_void_p(plane.data_ptr()), plane.stride(0),
                                                C.byref(self.desc), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                C.c_void_p(stage.data_ptr()), nb, _stream_handle(stream, dev)))
        st = torch.cuda.current_stream(dev) if stream is None else stream
        ev = torch.cuda.Event()
        ev.record(st)
        return (stage, ev, plane, st)

    def collect(self, ticket):
        """Candidates of a launched plane: waits for its read-back, then extracts them on the host
        (snd_detect_collect), while the device may already run later work.  Falls back to run()
        on the plane when the staged cells do not hold them all."""
        stage, ev, plane, st = ticket
        ev.synchronize()
        cnt, npx = C.c_int64(), C.c_int64()
        rc = capi.lib().snd_detect_collect(self.plan.handle, C.byref(self.desc), C.c_void_p(stage.data_ptr()),
                                           stage.numel(), self._buf, self._cap, C.byref(cnt), C.byref(npx))
        if rc == capi.ERR_CAPACITY and npx.value <= self.desc.max_pixels:
            return self.run(plane, stream=st)  # on the launch's stream: the workspace stays in order
        capi.check(rc)
        self.npixels = npx.value
        return self._candidates(cnt.value)

    def run(self, plane, stream=None):
        """Candidates of a plane, as dicts ordered by (k, t) of the peak.  Synchronises the stream."""
        cnt, npx = C.c_int64(), C.c_int64()
        capi.check(capi.lib().snd_detect(self.plan.handle, C.c_void_p(plane.data_ptr()), plane.stride(0),
                                         C.byref(self.desc), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                         self._buf, self._cap, C.byref(cnt), C.byref(npx),
                                         _stream_handle(stream, plane.device)))
        self.npixels = npx.value
        return self._candidates(cnt.value)

    def _candidates(self, n):
        out = []
        for i in range(min(n, self._cap)):
            c = self._buf[i]
            out.append(dict(k=c.dm_index, t=c.t, width=c.width, widx=self.widths.index(c.width), snr=c.snr,
                            dm=c.dm, npix=c.npix))
        return out


class BatchDetector:
    """Detection of the planes of several beams in shared grids (snd_detect_batch_*): one
    statistics and one S/N launch per plane dtype for all of them and one read-back, the same
    candidates as a Detector per beam.  Standard-deviation sigma and host labelling."""

    def __init__(self, widths=(1, 2, 4, 8, 16, 32, 64), threshold: float = 7.0, sigma_min: float = 0.0,
                 closing_radius: int = 4, n_min: int = 10, max_pixels: int = 1 << 20, device="cuda",
                 n_base_widths: int = 0, width_alpha: float = 0.0):
        import torch
        self._w = np.ascontiguousarray(widths, dtype=np.int32)
        d = capi.DetectDesc()
        d.widths = self._w.ctypes.data_as(C.POINTER(C.c_int32))
        d.nwidths = self._w.size
        d.threshold = threshold
        d.sigma_min = sigma_min
        d.closing_radius = closing_radius
        d.n_min = n_min
        d.n_base_widths = n_base_widths
        d.width_alpha = width_alpha
        d.max_pixels = max_pixels
        self.desc = d
        self.device = torch.device(device)
        self.widths = [int(w) for w in self._w]
        self.ws = None
        self.cap = 1 << 12  # candidates kept per beam
        self.npixels = []

    def launch(self, plans, planes, stage_cells: int = 1 << 18, stream=None):
        """Enqueue the detection of planes[i] (of plans[i]) and the read-back of up to stage_cells
        cells of all of them; returns a ticket for collect().  The workspace is reused in stream
        order; the planes must stay unchanged until collect() returns."""
        import torch
        n = len(plans)
        ph = (C.c_void_p * n)(*[p.handle for p in plans])
        nb = C.c_int64()
        capi.check(capi.lib().snd_detect_batch_workspace(n, ph, C.byref(self.desc), C.byref(nb)))
        if self.ws is None or self.ws.numel() < nb.value:
            self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        dp = (C.c_void_p * n)(*[y.data_ptr() for y in planes])
        pit = (C.c_int64 * n)(*[y.stride(0) for y in planes])
        sb = capi.DETECT_STAGE_HEADER + capi.DETECT_CELL_BYTES * int(stage_cells)
        stage = torch.empty(sb, dtype=torch.uint8, pin_memory=True)
        capi.check(capi.lib().snd_detect_batch_launch(n, ph, dp, pit, C.byref(self.desc),
                                                      C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                      C.c_void_p(stage.data_ptr()), sb,
                                                      _stream_handle(stream, self.device)))
        st = torch.cuda.current_stream(self.device) if stream is None else stream
        ev = torch.cuda.Event()
        ev.record(st)
        return (list(plans), list(planes), ph, stage, ev, st)

    def collect(self, ticket):
        """Candidates of each launched beam (a list of lists of dicts, as Detector.run); falls back
        to one Detector run per beam when the staged cells do not hold them all."""
        plans, planes, ph, stage, ev, st = ticket
        ev.synchronize()
        n = len(plans)
        buf = (capi.Candidate * (n * self.cap))()
        cnt, npx = (C.c_int64 * n)(), (C.c_int64 * n)()
        rc = capi.lib().snd_detect_batch_collect(n, ph, C.byref(self.desc), C.c_void_p(stage.data_ptr()),
                                                 stage.numel(), buf, self.cap, cnt, npx)
        if rc == capi.ERR_CAPACITY:
            out = []
            for p, y in zip(plans, planes):
                d = Detector(p, widths=self.widths, threshold=self.desc.threshold, sigma_min=self.desc.sigma_min,
                             closing_radius=self.desc.closing_radius, n_min=self.desc.n_min,
                             max_pixels=self.desc.max_pixels, device=self.device,
                             n_base_widths=self.desc.n_base_widths, width_alpha=self.desc.width_alpha)
                out.append(d.run(y, stream=st))
            return out
        capi.check(rc)
        self.npixels = [int(v) for v in npx]
        out = []
        for i in range(n):
            rows = []
            for j in range(min(int(cnt[i]), self.cap)):
                c = buf[i * self.cap + j]
                rows.append(dict(k=c.dm_index, t=c.t, width=c.width, widx=self.widths.index(c.width), snr=c.snr,
                                 dm=c.dm, npix=c.npix))
            out.append(rows)
        return out
