"""Streaming form of the SND path: beams admitted against a device-memory budget, each with
its input history ring in device memory, and chunk pushes that return the newly complete
output samples.  Argument marshalling over libsnd's snd_stream_* entry points."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from .plan import Plan, _stream_handle


def history_bytes(plan: Plan) -> int:
    """Device bytes of one beam's input ring for this plan."""
    b = C.c_int64()
    capi.check(capi.lib().snd_stream_history_bytes(plan.handle, C.byref(b)))
    return int(b.value)


def admission_bytes(plan: Plan) -> int:
    """Device bytes a beam of this plan is charged against a stream's budget: its ring plus its
    share of a batched push's workspace."""
    b = C.c_int64()
    capi.check(capi.lib().snd_stream_admission_bytes(plan.handle, C.byref(b)))
    return int(b.value)


class Stream:
    """A set of beams sharing one device-memory budget for their histories and the workspace of
    a batched push of all of them."""

    def __init__(self, budget_bytes: int, device="cuda"):
        import torch
        h = C.c_void_p()
        capi.check(capi.lib().snd_stream_create(int(budget_bytes), C.byref(h)))
        self._h = h
        self.device = torch.device(device)
        self._beams = {}  # beam id -> (plan, history tensor)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                capi.lib().snd_stream_destroy(h)
            except Exception:
                pass
            self._h = None

    def admit(self, beam_id: int, plan: Plan):
        """Admit a beam; raises SndError with status ERR_CAPACITY when over budget."""
        import torch
        nb = history_bytes(plan)
        hist = torch.empty(max(256, nb), dtype=torch.uint8, device=self.device)
        if plan._tables is None:
            plan.upload(self.device)
        capi.check(capi.lib().snd_stream_admit(self._h, int(beam_id), plan.handle, C.c_void_p(hist.data_ptr()),
                                               hist.numel()))
        self._beams[int(beam_id)] = (plan, hist)

    def evict(self, beam_id: int):
        capi.check(capi.lib().snd_stream_evict(self._h, int(beam_id)))
        self._beams.pop(int(beam_id), None)

    def beams(self):
        return sorted(self._beams)

    def plan_of(self, beam_id: int) -> Plan:
        return self._beams[int(beam_id)][0]

    def batch_bytes(self, beam_ids):
        """(workspace bytes, record bytes) of a batched push of these beams."""
        ids = (C.c_int32 * max(1, len(beam_ids)))(*[int(b) for b in beam_ids])
        w, r = C.c_int64(), C.c_int64()
        capi.check(capi.lib().snd_stream_batch_bytes(self._h, len(beam_ids), ids, C.byref(w), C.byref(r)))
        return w.value, r.value

    def push(self, items, workspace=None, stream=None, batched=False):
        """items: sequence of (beam_id, chunk_idx, chunk [nchan][L] tensor, out [ndm][>= n_out] tensor);
        bit-input beams take (beam_id, chunk_idx, chunk int32 [nchan][words] of bit rows, out, L bits).
        Returns [(out_t0, out_n, status)] per item; a chunk-index gap resets that beam (status
        ERR_GAP) and is not raised; every other failure raises SndError.  batched=True runs the
        beams' stages in shared grids (snd_stream_push_batched); its workspace and record
        buffers are kept by this object and grown on demand."""
        n = len(items)
        arr = (capi.StreamItem * max(1, n))()
        ws_need = 0
        for i, item in enumerate(items):
            bid, idx, chunk, out = item[:4]
            plan = self._beams[int(bid)][0]
            if chunk.dim() != 2 or chunk.shape[0] != plan.nchan or chunk.stride(1) != 1:
                raise ValueError("chunk must be [nchan][L] with unit time stride")
            bits = plan.in_dtype == "bits"
            if bits and len(item) != 5:
                raise ValueError("a bit-input beam's item carries its chunk length in bits")
            if out.dim() != 2 or out.shape[0] != plan.ndm or out.stride(1) != 1 or out.dtype != plan.out_dtype:
                raise ValueError("output must be [ndm][>= n_out] of the plan's output dtype")
            it = arr[i]
            it.beam_id, it.chunk_idx = int(bid), int(idx)
            it.chunk_len = int(item[4]) if bits else int(chunk.shape[1])
            it.d_chunk, it.chunk_pitch = chunk.data_ptr(), chunk.stride(0) * (32 if bits else 1)
            it.d_out, it.out_pitch = out.data_ptr(), out.stride(0)
            ws_need = max(ws_need, plan.info["workspace_bytes"])
        if batched:
            import torch
            wneed, rneed = self.batch_bytes([it[0] for it in items])
            if getattr(self, "_bws", None) is None or self._bws.numel() < wneed:
                self._bws = torch.empty(max(256, wneed), dtype=torch.uint8, device=self.device)
            if getattr(self, "_brec", None) is None or self._brec.numel() < rneed:
                self._brec = torch.empty(max(256, rneed), dtype=torch.uint8, device=self.device)
            rc = capi.lib().snd_stream_push_batched(self._h, n, arr, C.c_void_p(self._bws.data_ptr()),
                                                    self._bws.numel(), C.c_void_p(self._brec.data_ptr()),
                                                    self._brec.numel(), _stream_handle(stream, self.device))
            if rc not in (capi.OK, capi.ERR_GAP):
                capi.check(rc)
            return [(arr[i].out_t0, arr[i].out_n, arr[i].status) for i in range(n)]
        if workspace is None and ws_need > 0:
            raise ValueError("a workspace of at least the plans' workspace_bytes is required")
        wsp = C.c_void_p(workspace.data_ptr()) if workspace is not None else None
        wsb = workspace.numel() if workspace is not None else 0
        rc = capi.lib().snd_stream_push(self._h, n, arr, wsp, wsb, _stream_handle(stream, self.device))
        if rc not in (capi.OK, capi.ERR_GAP):
            capi.check(rc)
        return [(arr[i].out_t0, arr[i].out_n, arr[i].status) for i in range(n)]

    def state(self, beam_id: int):
        r, nx, e = C.c_int64(), C.c_int64(), C.c_int64()
        capi.check(capi.lib().snd_stream_beam_state(self._h, int(beam_id), C.byref(r), C.byref(nx), C.byref(e)))
        return dict(received=r.value, next_chunk=nx.value, emitted=e.value)

    def usage(self):
        b, u, n = C.c_int64(), C.c_int64(), C.c_int32()
        capi.check(capi.lib().snd_stream_usage(self._h, C.byref(b), C.byref(u), C.byref(n)))
        return dict(budget=b.value, used=u.value, n_beams=n.value)

    def export(self, beam_id: int, stream=None) -> np.ndarray:
        nb = C.c_int64()
        capi.check(capi.lib().snd_stream_export_bytes(self._h, int(beam_id), C.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        capi.check(capi.lib().snd_stream_export(self._h, int(beam_id), buf.ctypes.data_as(C.c_void_p), buf.size,
                                                _stream_handle(stream, self.device)))
        return buf

    def restore(self, beam_id: int, buf: np.ndarray, stream=None):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        capi.check(capi.lib().snd_stream_import(self._h, int(beam_id), buf.ctypes.data_as(C.c_void_p), buf.size,
                                                _stream_handle(stream, self.device)))
