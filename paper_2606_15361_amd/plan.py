"""Python view of an SND plan: marshals arguments to the C ABI; torch supplies device memory
and the HIP stream.  Every step of the dedispersion path runs in libsnd's HIP kernels."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi

MODES = {"binary": capi.MODE_BINARY, "graded": capi.MODE_GRADED, "float": capi.MODE_FLOAT}
DTYPES = {"u8": capi.DT_U8, "u16": capi.DT_U16, "f32": capi.DT_F32, "bf16": capi.DT_BF16, "f16": capi.DT_F16,
          "bits": capi.DT_BITS}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}


def torch_dtype(dt: int):
    """Tensor dtype holding rows of this storage type (bit rows: int32 words)."""
    import torch
    return {capi.DT_U8: torch.uint8, capi.DT_U16: torch.uint16, capi.DT_F32: torch.float32,
            capi.DT_BF16: torch.bfloat16, capi.DT_F16: torch.float16, capi.DT_BITS: torch.int32}[dt]


def row_pitch(x, dtype: str) -> int:
    """Row pitch of tensor x in elements of the storage type (bit rows: in bits)."""
    return x.stride(0) * 32 if dtype == "bits" else x.stride(0)


def row_samples(x, dtype: str) -> int:
    """Samples a row of tensor x can hold."""
    return x.shape[1] * 32 if dtype == "bits" else x.shape[1]


def _stream_handle(stream, device):
    import torch
    s = torch.cuda.current_stream(device) if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_desc(freqs, dms, tsamp_s, nsamp, *, mode="float", branching=4, cluster=4, k_leaf=2, k_int=2, cap=255,
              in_dtype=None, node_dtype=None, root_norm=False, fref=0.0, stage_levels=0, generic_kernels=False,
              chunk=0, tune=0):
    """snd_plan_desc for these parameters; also returns the frequency and DM arrays it points to
    (keep them alive while the descriptor is used) and the resolved storage types."""
    freq = np.ascontiguousarray(freqs, dtype=np.float64)
    dm = np.ascontiguousarray(dms, dtype=np.float64)
    if in_dtype is None:
        in_dtype = "f32" if mode == "float" else "u8"
    if node_dtype is None:
        node_dtype = "f32" if mode == "float" else ("bits" if mode == "binary" else "u8" if cap <= 255 else "u16")
    d = capi.PlanDesc()
    d.nchan = freq.size
    d.freq_mhz = freq.ctypes.data_as(C.POINTER(C.c_double))
    d.tsamp_s = tsamp_s
    d.fref_mhz = fref
    d.ndm = dm.size
    d.dm = dm.ctypes.data_as(C.POINTER(C.c_double))
    d.branching, d.cluster, d.mode = branching, cluster, MODES[mode]
    d.k_leaf, d.k_int, d.cap = k_leaf, k_int, cap
    d.in_dtype, d.node_dtype = DTYPES[in_dtype], DTYPES[node_dtype]
    d.root_norm = int(root_norm)
    d.nsamp = int(nsamp or 0)
    d.chunk = int(chunk)
    d.stage_levels = int(stage_levels)
    d.generic_kernels = int(generic_kernels)
    d.tune = int(tune)
    return d, freq, dm, in_dtype, node_dtype


def tune_word(leaf_window: int = 0, xcd_groups: int = 0, lds_quarters_off: int = 0) -> int:
    """snd_plan_desc.tune from its fields: leaf-stage window (0 auto, else 512, 1024, 2048 or
    4096 samples), final-stage DM groups dealt per XCD and time tile (0 auto, else a power of two
    up to 64), and quarters of the final stage's LDS batch buffer left unused (0..3)."""
    w = {0: 0, 512: 1, 1024: 2, 2048: 3, 4096: 4}[int(leaf_window)]
    x = 0 if not xcd_groups else int(xcd_groups).bit_length()
    if xcd_groups and (1 << (x - 1)) != xcd_groups or x > 7:
        raise ValueError("xcd_groups must be 0 or a power of two up to 64")
    if not 0 <= lds_quarters_off <= 3:
        raise ValueError("lds_quarters_off must be 0..3")
    return w | (x << 4) | (int(lds_quarters_off) << 8)


def tune_fields(tune: int) -> dict:
    """The fields of a tune word (see tune_word)."""
    w, x, q = tune & 15, (tune >> 4) & 15, (tune >> 8) & 15
    return dict(leaf_window=0 if not w else 512 << (w - 1), xcd_groups=0 if not x else 1 << (x - 1),
                lds_quarters_off=q)


def autotune(freqs, dms, tsamp_s, x, candidates, *, reps=2, out=None, stream=None, nsamp=None, **plan_kw):
    """Time every candidate on the block x [nchan][nsamp] with snd_autotune (nsamp defaults to
    the samples a row of x holds).  A candidate is (stage_levels, chunk) or (stage_levels, chunk,
    tune).  Returns (index of the fastest, [dict(stage_levels, chunk, tune, ms, workspace_bytes,
    table_bytes)]); a skipped candidate has ms -1.  Buffers are sized for the largest candidate
    that is probed host-side first."""
    import torch
    cands = [tuple(c) + (0,) * (3 - len(c)) for c in candidates]
    in_dt = plan_kw.get("in_dtype") or ""
    nsamp = int(nsamp or row_samples(x, in_dt))
    probes = []
    for s, c, t in cands:
        try:
            probes.append(Plan(freqs, dms, tsamp_s, None if c else nsamp, stage_levels=s, chunk=c, tune=t, **plan_kw))
        except capi.SndError as e:
            if e.status != capi.ERR_UNSUPPORTED:
                raise
    wsb = max(p.info["workspace_bytes"] for p in probes)
    tb = max(p.info["table_bytes"] for p in probes)
    n_out = nsamp - probes[0].max_delay
    dev = x.device
    ws = torch.empty(max(256, wsb), dtype=torch.uint8, device=dev)
    tables = torch.empty(max(256, tb), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((probes[0].ndm, n_out), dtype=probes[0].out_dtype, device=dev)
    del probes
    d, _f, _d, _, _ = make_desc(freqs, dms, tsamp_s, nsamp, stage_levels=0, chunk=0, **plan_kw)
    arr = (capi.TuneCandidate * len(cands))()
    for i, (s, c, t) in enumerate(cands):
        arr[i].stage_levels, arr[i].chunk, arr[i].tune = int(s), int(c), int(t)
    best = C.c_int32()
    capi.check(capi.lib().snd_autotune(C.byref(d), arr, len(cands), C.c_void_p(x.data_ptr()), row_pitch(x, in_dt),
                                       C.c_void_p(out.data_ptr()), out.stride(0), C.c_void_p(ws.data_ptr()),
                                       ws.numel(), C.c_void_p(tables.data_ptr()), tables.numel(), int(reps),
                                       C.byref(best), _stream_handle(stream, dev)))
    return best.value, [dict(stage_levels=a.stage_levels, chunk=a.chunk, tune=a.tune, ms=a.ms,
                             workspace_bytes=a.workspace_bytes, table_bytes=a.table_bytes) for a in arr]


def tune_cache_path() -> str:
    """File of the autotune cache: $SND_TUNE_CACHE, else ~/.cache/snd/tune.json."""
    import os
    return os.environ.get("SND_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "snd", "tune.json")


def tune_key(freqs, dms, tsamp_s, nsamp, device, **plan_kw) -> str:
    """Cache key of a tuning problem: GPU architecture, mode, storage types, branching, cluster,
    the tree's shape (nodes and shared neurons per level), DM rows and output samples."""
    import torch
    kw = {k: v for k, v in plan_kw.items() if k not in ("stage_levels", "chunk", "tune")}
    p = Plan(freqs, dms, tsamp_s, nsamp, **kw)
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    return "|".join(str(v) for v in (arch, p.mode, p.in_dtype, p.node_dtype, p.params["branching"],
                                        p.params["cluster"], p.params["cap"] if p.mode == "graded" else "-",
                                        ",".join(map(str, p.info["nodes_per_level"])),
                                        ",".join(map(str, p.info["neurons_per_level"])), p.ndm, p.n_out))


def autotune_cached(freqs, dms, tsamp_s, x, candidates, *, nsamp=None, cache_path=None, reps=2, **plan_kw):
    """autotune() with an on-disk cache keyed by tune_key(): a stored choice for the same key and
    candidate list is returned without timing.  Returns (best candidate as a tuple, records, hit)."""
    import json
    import os
    path = cache_path or tune_cache_path()
    in_dt = plan_kw.get("in_dtype") or ""
    nsamp = int(nsamp or row_samples(x, in_dt))
    key = tune_key(freqs, dms, tsamp_s, nsamp, x.device, **plan_kw)
    cands = [list(tuple(c) + (0,) * (3 - len(c))) for c in candidates]
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    ent = db.get(key)
    if ent is not None and ent.get("candidates") == cands:
        return tuple(ent["best"]), ent["records"], True
    best, recs = autotune(freqs, dms, tsamp_s, x, [tuple(c) for c in cands], reps=reps, nsamp=nsamp, **plan_kw)
    db[key] = dict(candidates=cands, best=cands[best], records=recs)
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only cache location: the result is still returned
    return tuple(cands[best]), recs, False


class Plan:
    """An SND dedispersion plan (host tables, built by snd_plan_create)."""

    def __init__(self, freqs, dms, tsamp_s: float, nsamp: int | None, *, mode: str = "float", branching: int = 4,
                 cluster: int = 4, k_leaf: int = 2, k_int: int = 2, cap: int = 255, in_dtype: str | None = None,
                 node_dtype: str | None = None, root_norm: bool = False, fref: float = 0.0, stage_levels: int = 0,
                 generic_kernels: bool = False, chunk: int = 0, tune: int = 0):
        """nsamp: input samples per execute; or chunk > 0 (nsamp None): a streaming plan whose
        n_out is `chunk` and whose nsamp is max_delay + chunk.  tune: launch shapes
        (snd_plan_desc.tune; 0 = defaults, see tune_word)."""
        L = capi.lib()
        # binary mode stores tree rows as bits unless asked otherwise; trees and schedules that
        # bit rows do not support (irregular level-1 nodes, other stage schedules) use bytes
        auto_bits = mode == "binary" and node_dtype is None
        d, self._freq, self._dm, in_dtype, node_dtype = make_desc(
            freqs, dms, tsamp_s, nsamp, mode=mode, branching=branching, cluster=cluster, k_leaf=k_leaf, k_int=k_int,
            cap=cap, in_dtype=in_dtype, node_dtype=node_dtype, root_norm=root_norm, fref=fref,
            stage_levels=stage_levels, generic_kernels=generic_kernels, chunk=chunk, tune=tune)
        self.tune = int(tune)
        h = C.c_void_p()
        rc = L.snd_plan_create(C.byref(d), C.byref(h))
        if rc == capi.ERR_UNSUPPORTED and auto_bits:
            node_dtype = "u8"
            d.node_dtype = DTYPES[node_dtype]
            rc = L.snd_plan_create(C.byref(d), C.byref(h))
        capi.check(rc)
        self._h = h
        self.mode, self.nchan, self.ndm = mode, self._freq.size, self._dm.size
        self.in_dtype, self.node_dtype = in_dtype, node_dtype
        self.params = dict(mode=mode, branching=branching, cluster=cluster, k_leaf=k_leaf, k_int=k_int, cap=cap,
                           root_norm=root_norm)
        info = capi.PlanInfo()
        capi.check(L.snd_plan_query(h, C.byref(info)))
        nl, ns = info.n_levels, info.n_stages
        self.info = dict(
            n_out=info.n_out, max_delay=info.max_delay, n_levels=nl, n_stages=ns, out_dtype=info.out_dtype,
            n_neurons=info.n_neurons, n_synapses=info.n_synapses,
            neurons_per_level=list(info.neurons_per_level[:nl]), synapses_per_level=list(info.synapses_per_level[:nl]),
            nodes_per_level=list(info.nodes_per_level[:nl]), table_bytes=info.table_bytes,
            workspace_bytes=info.workspace_bytes, alg_bytes=info.alg_bytes,
            stage_alg_bytes=list(info.stage_alg_bytes[:ns]), stage_rows=list(info.stage_rows[:ns]),
            stage_entries=list(info.stage_entries[:ns]), build_seconds=info.build_seconds,
            stage_kernel=[("generic", "group_lds", "anchored", "group_fast", "group_bits", "anchored_bits",
                           "group_lin", "group_pack")[k]
                          for k in info.stage_kernel[:ns]],
            stage_staged=list(info.stage_staged[:ns]), stage_batches=list(info.stage_batches[:ns]),
            stage_windows=list(info.stage_windows[:ns]),
            stage_src_dtype=[in_dtype if s == 0 else node_dtype for s in range(ns)])
        self.n_out = info.n_out
        self.nsamp = info.n_out + info.max_delay
        self.max_delay = info.max_delay
        self._tables = None
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                capi.lib().snd_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def delays(self) -> np.ndarray:
        out = np.empty((self.ndm, self.nchan), dtype=np.int32)
        capi.check(capi.lib().snd_plan_delays(self._h, out.ctypes.data_as(C.c_void_p), out.size))
        return out

    @property
    def out_dtype(self):
        return torch_dtype(self.info["out_dtype"])

    def upload(self, device="cuda", stream=None):
        import torch
        dev = torch.device(device)
        self._tables = torch.empty(max(256, self.info["table_bytes"]), dtype=torch.uint8, device=dev)
        capi.check(capi.lib().snd_plan_upload(self._h, C.c_void_p(self._tables.data_ptr()), self._tables.numel(),
                                              _stream_handle(stream, dev)))
        return self

    def workspace(self, device="cuda"):
        import torch
        if self._ws is None or self._ws.device != torch.device(device):
            self._ws = torch.empty(max(256, self.info["workspace_bytes"]), dtype=torch.uint8, device=device)
        return self._ws

    def empty_output(self, device="cuda"):
        """[ndm][n_out] view of rows whose pitch is a multiple of 64 samples, so that every row
        starts on a 256-byte boundary (whole-line stores)."""
        import torch
        pitch = (self.n_out + 63) // 64 * 64
        return torch.empty((self.ndm, pitch), dtype=self.out_dtype, device=device)[:, : self.n_out]

    def execute(self, x, out=None, workspace=None, stream=None, stage=None):
        """Dedisperse x [nchan][>= nsamp] (device tensor of the input dtype) into out [ndm][>= n_out].
        With ``stage`` set, run only that stage of the schedule (see snd_execute_stage)."""
        import torch
        if self._tables is None:
            self.upload(x.device, stream)
        if x.dim() != 2 or x.shape[0] != self.nchan or row_samples(x, self.in_dtype) < self.nsamp or x.stride(1) != 1:
            raise ValueError(f"input must be [{self.nchan}][>= {self.nsamp} samples] with unit time stride")
        want = torch_dtype(DTYPES[self.in_dtype])
        if x.dtype != want:
            raise TypeError(f"input dtype {x.dtype}, plan expects {want}")
        if out is None:
            out = self.empty_output(x.device)
        if out.dim() != 2 or out.shape[0] != self.ndm or out.shape[1] < self.n_out or out.stride(1) != 1 \
                or out.dtype != self.out_dtype:
            raise ValueError("bad output tensor")
        ws = self.workspace(x.device) if workspace is None else workspace
        args = (C.c_void_p(x.data_ptr()), row_pitch(x, self.in_dtype), C.c_void_p(out.data_ptr()), out.stride(0),
                C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream, x.device))
        if stage is None:
            capi.check(capi.lib().snd_execute(self._h, *args))
        else:
            capi.check(capi.lib().snd_execute_stage(self._h, int(stage), *args))
        return out


def encode(z, thresholds, time_major: bool = False, out=None, stream=None):
    """Delta encoder on the GPU: uint8 level = number of thresholds exceeded by z (float32)."""
    import torch
    th = np.ascontiguousarray(thresholds, dtype=np.float32)
    if z.dtype != torch.float32 or z.stride(1) != 1:
        raise TypeError("z must be float32 with unit inner stride")
    nchan, nsamp = (z.shape[1], z.shape[0]) if time_major else (z.shape[0], z.shape[1])
    if out is None:
        out = torch.empty((nchan, nsamp), dtype=torch.uint8, device=z.device)
    capi.check(capi.lib().snd_encode(C.c_void_p(z.data_ptr()), z.stride(0), int(time_major), nchan, nsamp,
                                     th.ctypes.data_as(C.c_void_p), th.size, C.c_void_p(out.data_ptr()),
                                     out.stride(0), _stream_handle(stream, z.device)))
    return out


def encode_bits(z, threshold: float, time_major: bool = False, out=None, stream=None):
    """Delta encoder to bit rows on the GPU: bit i of word w of channel c = 1[z_c(32 w + i) > threshold].
    Returns int32 [nchan][words], words a multiple of 4 (row pitch a multiple of 128 bits)."""
    import torch
    if z.dtype != torch.float32 or z.stride(1) != 1:
        raise TypeError("z must be float32 with unit inner stride")
    nchan, nsamp = (z.shape[1], z.shape[0]) if time_major else (z.shape[0], z.shape[1])
    if out is None:
        out = torch.zeros((nchan, (nsamp + 127) // 128 * 4), dtype=torch.int32, device=z.device)
    if out.dtype != torch.int32 or out.stride(1) != 1 or out.shape[0] != nchan or out.shape[1] * 32 < nsamp:
        raise ValueError("out must be int32 [nchan][>= nsamp / 32] with unit inner stride")
    capi.check(capi.lib().snd_encode_bits(C.c_void_p(z.data_ptr()), z.stride(0), int(time_major), nchan, nsamp,
                                          float(threshold), C.c_void_p(out.data_ptr()), out.stride(0) * 32,
                                          _stream_handle(stream, z.device)))
    return out


def channel_stats(p, clip: float = 5.0, stream=None):
    """Two-pass sigma-clip statistics of raw power p [nchan][nsamp] (float32, on the GPU):
    float64 [nchan][2] of (mu, sigma) per channel (snd_channel_stats)."""
    import torch
    if p.dtype != torch.float32 or p.stride(1) != 1:
        raise TypeError("p must be float32 with unit inner stride")
    st = torch.empty((p.shape[0], 2), dtype=torch.float64, device=p.device)
    capi.check(capi.lib().snd_channel_stats(C.c_void_p(p.data_ptr()), p.stride(0), p.shape[0], p.shape[1],
                                            float(clip), C.c_void_p(st.data_ptr()), _stream_handle(stream, p.device)))
    return st


def normalize(p, stats, out=None, stream=None):
    """z = (P - mu) / sigma per channel as float32 (snd_normalize)."""
    import torch
    if p.dtype != torch.float32 or p.stride(1) != 1:
        raise TypeError("p must be float32 with unit inner stride")
    if stats.dtype != torch.float64 or not stats.is_contiguous() or stats.shape != (p.shape[0], 2):
        raise ValueError("stats must be contiguous float64 [nchan][2]")
    if out is None:
        out = torch.empty(p.shape, dtype=torch.float32, device=p.device)
    capi.check(capi.lib().snd_normalize(C.c_void_p(p.data_ptr()), p.stride(0), p.shape[0], p.shape[1],
                                        C.c_void_p(stats.data_ptr()), C.c_void_p(out.data_ptr()), out.stride(0),
                                        _stream_handle(stream, p.device)))
    return out


def zero_dm(z, gamma: float = 5.0, count=None, stream=None):
    """Zero-DM subtraction in place on a z-scored float32 filterbank [nchan][nsamp] (snd_zero_dm);
    count: optional int32 device tensor of one element, incremented by the samples changed."""
    import torch
    if z.dtype != torch.float32 or z.stride(1) != 1:
        raise TypeError("z must be float32 with unit inner stride")
    if count is not None and (count.dtype != torch.int32 or count.device != z.device):
        raise TypeError("count must be an int32 tensor on z's device")
    capi.check(capi.lib().snd_zero_dm(C.c_void_p(z.data_ptr()), z.stride(0), z.shape[0], z.shape[1], float(gamma),
                                      None if count is None else C.c_void_p(count.data_ptr()),
                                      _stream_handle(stream, z.device)))
    return z


def flag_channels(z, window: int, k: float = 5.0, stream=None, return_sigma: bool = False):
    """Windowed MAD channel flagging in place on a z-scored float32 filterbank [nchan][nsamp]
    (snd_flag_channels); returns the uint8 flags [nwin][nchan] (and the float64 per-window
    channel sigmas [nwin][nchan] with return_sigma)."""
    import torch
    if z.dtype != torch.float32 or z.stride(1) != 1:
        raise TypeError("z must be float32 with unit inner stride")
    nwin = (z.shape[1] + window - 1) // window
    flags = torch.empty((nwin, z.shape[0]), dtype=torch.uint8, device=z.device)
    sigma = torch.empty((nwin, z.shape[0]), dtype=torch.float64, device=z.device)
    capi.check(capi.lib().snd_flag_channels(C.c_void_p(z.data_ptr()), z.stride(0), z.shape[0], z.shape[1],
                                            int(window), float(k), C.c_void_p(sigma.data_ptr()),
                                            C.c_void_p(flags.data_ptr()), flags.stride(0),
                                            _stream_handle(stream, z.device)))
    return (flags, sigma) if return_sigma else flags


def cast(x, dtype: str, stream=None):
    """float32 [rows][cols] -> bf16/f16 with round-to-nearest-even, on the GPU."""
    import torch
    dt = DTYPES[dtype]
    out = torch.empty(x.shape, dtype=torch_dtype(dt), device=x.device)
    capi.check(capi.lib().snd_cast(C.c_void_p(x.data_ptr()), x.stride(0), x.shape[0], x.shape[1],
                                   C.c_void_p(out.data_ptr()), out.stride(0), dt, _stream_handle(stream, x.device)))
    return out
