"""Serving loop over many beams: each arriving filterbank chunk is encoded (graded beams) or cast
to its storage type (reduced-precision float beams) on the device, all ready beams are pushed
through the streaming form in shared grids, and every complete output chunk goes through the
matched filter and candidate stage.  Beams are admitted against a device-memory budget for
their histories.  Host orchestration only: every step of the path runs in libsnd's kernels."""

from __future__ import annotations

import time

from . import _capi as capi
from .detect import BatchDetector, Detector
from .plan import cast, encode
from .stream import Stream, admission_bytes, history_bytes


class Server:
    """kinds: {name: (plan, encoder thresholds or None)} -- a beam of a kind streams through
    that kind's plan; thresholds encode z-scored chunks to levels, None casts them to the
    plan's input storage type."""

    def __init__(self, kinds: dict, budget_bytes: int, *, widths=(1, 2, 4, 8, 16, 32, 64), threshold=7.0,
                 n_min=10, batched=True, device="cuda", stage_cells=1 << 15):
        import torch
        self.device = torch.device(device)
        self.kinds = kinds
        self.batched = batched
        self.stage_cells = stage_cells  # thresholded cells read back per chunk (more: run again)
        self.stream = Stream(budget_bytes, device)
        self.det = {k: Detector(p, widths=widths, threshold=threshold, n_min=n_min, device=device)
                    for k, (p, _) in kinds.items()}
        # the batched form detects all complete chunks of a push in shared grids
        self.bdet = BatchDetector(widths=widths, threshold=threshold, n_min=n_min, device=device) if batched else None
        self.kind_of, self.out = {}, {}
        self.ws = None
        if not batched:
            self.ws = torch.empty(max(256, max(p.info["workspace_bytes"] for p, _ in kinds.values())),
                                  dtype=torch.uint8, device=device)

    def history_bytes(self, kind: str) -> int:
        return history_bytes(self.kinds[kind][0])

    def admission_bytes(self, kind: str) -> int:
        return admission_bytes(self.kinds[kind][0])

    def admit(self, beam: int, kind: str) -> bool:
        """False when the budget cannot hold the beam's history and workspace share."""
        plan = self.kinds[kind][0]
        try:
            self.stream.admit(beam, plan)
        except capi.SndError as e:
            if e.status == capi.ERR_CAPACITY:
                return False
            raise
        self.kind_of[beam] = kind
        self.out[beam] = plan.empty_output(self.device)
        return True

    def evict(self, beam: int):
        self.stream.evict(beam)
        self.kind_of.pop(beam, None)
        self.out.pop(beam, None)

    def beams(self):
        return sorted(self.kind_of)

    def next_index(self, beam: int) -> int:
        """The chunk index the beam expects next (0 before its first chunk)."""
        return max(0, self.stream.state(beam)["next_chunk"])

    def process(self, ready):
        """ready: [(beam, chunk index, z-scored float32 chunk [nchan][T] on the device)].
        Returns [(beam, chunk index, output t0, output samples, candidates or None)]; candidates
        are None while the history fills (fewer output samples than the chunk)."""
        items = []
        for beam, idx, z in ready:
            plan, thr = self.kinds[self.kind_of[beam]]
            x = encode(z, thr) if thr is not None else (z if plan.in_dtype == "f32" else cast(z, plan.in_dtype))
            items.append((beam, idx, x, self.out[beam]))
        res = self.stream.push(items, workspace=self.ws, batched=self.batched)
        if self.batched:
            # the complete chunks of every beam in one batched detection: shared grids, one
            # read-back, candidates extracted per beam on the host
            full = [i for i, ((beam, _, _, _), (t0, n, st)) in enumerate(zip(items, res))
                    if n == self.kinds[self.kind_of[beam]][0].n_out]
            found = {}
            if full:
                tk = self.bdet.launch([self.kinds[self.kind_of[items[i][0]]][0] for i in full],
                                      [items[i][3] for i in full], stage_cells=self.stage_cells * len(full))
                found = dict(zip(full, self.bdet.collect(tk)))
            return [(beam, idx, t0, n, found.get(i)) for i, ((beam, idx, _, _), (t0, n, _)) in
                    enumerate(zip(items, res))]
        # every complete chunk's detection is enqueued first (kernels and the read-back of its
        # thresholded cells, on the push's stream), then the host extracts the candidates of
        # each in turn while the device works through the rest
        tickets = []
        for (beam, idx, _, out), (t0, n, status) in zip(items, res):
            kind = self.kind_of[beam]
            full = n == self.kinds[kind][0].n_out
            tickets.append((beam, idx, t0, n, kind, self.det[kind].launch(out, stage_cells=self.stage_cells)
                            if full else None))
        return [(beam, idx, t0, n, None if tk is None else self.det[kind].collect(tk))
                for beam, idx, t0, n, kind, tk in tickets]


def run_schedule(server: Server, arrivals, make_chunk, *, duration_s: float, joins=(), leaves=(), warm_chunks=5,
                 clock=time.perf_counter, log=None):
    """Drive `server` in real time.  arrivals: {beam: sorted arrival times (s)}; make_chunk(beam,
    idx) returns the z-scored device chunk; joins / leaves: [(time s, beam, kind)] / [(time s,
    beam)].  Chunks that arrived by `now` are processed together.  Returns per-chunk records
    (beam, idx, arrival, done, latency, n candidates) and the admission decisions."""
    import torch
    t_start = clock()
    nxt = {b: 0 for b in arrivals}
    recs, admissions = [], []
    joins, leaves = sorted(joins), sorted(leaves)
    while True:
        now = clock() - t_start
        if now >= duration_s:
            break
        while leaves and leaves[0][0] <= now:
            _, b = leaves.pop(0)
            if b in server.kind_of:
                server.evict(b)
        while joins and joins[0][0] <= now:
            tj, b, kind = joins.pop(0)
            ok = server.admit(b, kind)
            admissions.append((tj, b, kind, ok))
            if ok:
                nxt[b] = 0
                arrivals[b] = arrivals[b][arrivals[b] >= tj]
        ready, meta = [], []
        for b in server.beams():
            ts = arrivals.get(b)
            if ts is None or nxt[b] >= len(ts) or ts[nxt[b]] > now:
                continue
            ready.append((b, nxt[b], make_chunk(b, nxt[b])))
            meta.append(ts[nxt[b]])
            nxt[b] += 1
        if not ready:
            time.sleep(0.0005)
            continue
        out = server.process(ready)
        torch.cuda.synchronize()
        t_done = clock() - t_start
        for (b, idx, t0, n, cands), t_arr in zip(out, meta):
            recs.append(dict(beam=b, idx=idx, arrival=t_arr, done=t_done, latency=t_done - t_arr,
                             counted=idx >= warm_chunks and cands is not None,
                             candidates=0 if cands is None else len(cands)))
        if log is not None and len(recs) % 200 < len(out):
            log(f"[serve] t={t_done:.1f}s chunks={len(recs)} beams={len(server.beams())}")
    return recs, admissions
