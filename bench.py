"""Benchmark of the SND hot path on one MI355X.

Default workload: one Northern-Cross-shaped beam (1024 channels, 400-416 MHz, 0.138 ms,
2^17 samples, 16 injected pulses), 4096 trial DMs uniform over 0-2000, branching factor 4,
float32 mode.  One step = one full pass of the path over that block: the SND tree (leaf
stage + fused upper-tree stage) followed by the boxcar S/N and candidate stage.  Inputs
are resident in device memory before timing starts.

Prints one JSON line (see the repository's benchmark contract).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "dedispersed DM\u00d7time samples/s (1024 ch, 4096 DM) + %HBM peak; p99 chunk latency"
# LDS read peak of gfx950: 256 CUs x 256 B/clk (CDNA4 doubled the per-CU LDS read rate of
# CDNA3's 128 B/clk for 128-bit reads) x 2.4 GHz = 157.3 TB/s; a ds_read_b128 probe on the
# part reaches 132 TB/s, 84 % of it
LDS_PEAK_GBS = 256 * 256 * 2.4
KERNEL_SYMBOL = {"generic": "k_stage", "group_lds": "k_group", "anchored": "k_anchored", "group_fast": "k_group_fast",
                 "group_bits": "k_group_bits", "anchored_bits": "k_anchored_bits",
                 "group_lin": "k_group_lin", "group_pack": "k_group_pack"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


# sources that decide what the tree kernels do: device code, the headers it includes, the plan
# builder (tables, windows, batches) and the launch path; the other host files (detection's
# host part, streaming, batching, tuning, multi-rate, validation) and the detection kernels,
# which the tree kernels do not include, do not change their traffic
DIGEST_CPP = ("plan.cpp", "capi.cpp")
DIGEST_SKIP = ("detect.hip", "detect_noalloc.hip", "label.hip", "snd_detect.h")


def source_digest():
    """Digest of the sources the counter readings depend on: they are only valid for that code."""
    import hashlib
    h = hashlib.sha256()
    for d in ("paper_2606_15361_amd/csrc", "include"):
        for name in sorted(os.listdir(os.path.join(ROOT, d))):
            if (name.endswith((".hip", ".h")) and name not in DIGEST_SKIP) or name in DIGEST_CPP:
                with open(os.path.join(ROOT, d, name), "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, or None when
    the summary is absent or was taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    e = rec.get("kernels", {}).get(key)
    if e is None:
        return None
    return (e["fetch_kib"] * rec["read_scale"] + e["write_kib"] * rec["write_scale"]) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="float", choices=["float", "graded", "binary"])
    ap.add_argument("--node-dtype", default=None)
    ap.add_argument("--input", default="auto", choices=["auto", "bytes", "bits"],
                    help="binary input storage: bit rows (auto) or one byte per sample")
    ap.add_argument("--stage-levels", type=lambda s: int(s, 0), default=0)
    ap.add_argument("--no-detect", action="store_true", help="time the tree only")
    ap.add_argument("--serial-detect", action="store_true",
                    help="extract each block's candidates before the next block starts (no host/device overlap)")
    ap.add_argument("--generic-kernels", action="store_true", help="run every stage on the generic stage kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2048,
                    help="output samples in the oracle's single-thread timed sample")
    ap.add_argument("--cpu-sample-all", type=int, default=16384,
                    help="output samples in the oracle's all-core timed sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default stage schedule")
    ap.add_argument("--legs", default="direct,fdmt,multirate,trees,frontend,batch,serve",
                    help="extra measurements after the headline: direct (the same block without shared neurons), "
                         "multirate (scrunch bands), trees (every mode and storage, B = 4 and 8), batch (48 beams), "
                         "serve (streaming loop and load sweep)")
    ap.add_argument("--serve-seconds", type=float, default=12.0, help="real-time length of each serving run")
    return ap.parse_args()


def _host_cpu():
    """(usable host cores, CPU model name)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n, model


def _cpu_slice(job):
    """One worker's share of the all-core oracle run (a fresh interpreter: nothing of the GPU
    process is inherited): the shared-pattern tree over one contiguous slice of DM rows, on the
    input cut to that slice's own sweep plus the sample, so that every DM row yields the same
    number of output samples.  Returns (output cells, seconds)."""
    import numpy as np
    import oracle
    path, freqs, d, mode, branching, n_sample = job
    x = np.load(path, mmap_mode="r")
    n = int(d.max()) + n_sample
    xs = np.ascontiguousarray(x[:, :n])
    t = time.perf_counter()
    y, _ = oracle.snd_dedup(xs, freqs, d, mode=mode, cluster=4, branching=branching, k_leaf=2, k_int=1, cap=255)
    return int(y.shape[0] * y.shape[1]), time.perf_counter() - t


def cpu_baseline(spec, mode, n_sample, n_sample_all):
    """The oracle's shared-pattern tree timed on the host, on bounded slices of the same beam:
    on one thread over every DM row, and on all usable host cores (up to 16, one process per
    contiguous DM slice) over a longer slice."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    d = oracle.delays(spec.freqs, spec.dms, spec.tsamp_s)
    n_long = max(n_sample, n_sample_all)
    z = spec.filterbank(int(d.max()) + n_long)
    x = z if mode == "float" else oracle.encode(z, [1.0, 2.0, 3.0, 4.0] if mode == "graded" else [2.0])
    kw = dict(mode=mode, cluster=4, branching=spec.branching, k_leaf=2, k_int=1, cap=255)
    t = time.perf_counter()
    y, _ = oracle.snd_dedup(x[:, :int(d.max()) + n_sample], spec.freqs, d, **kw)
    dt1 = time.perf_counter() - t
    v1 = float(spec.dms.size * n_sample / dt1)
    ncpu, model = _host_cpu()
    workers = max(1, min(16, ncpu))
    bounds = np.linspace(0, spec.dms.size, workers + 1).astype(int)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "x.npy")
        np.save(path, x)
        jobs = [(path, spec.freqs, d[bounds[i]:bounds[i + 1]], mode, spec.branching, n_sample_all)
                for i in range(workers)]
        # fresh interpreters ("spawn"), so that no worker inherits the GPU process's state
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_cpu_slice, [(path, spec.freqs, d[:1], mode, spec.branching, 1)] * workers)  # warm imports
            t = time.perf_counter()
            res = pool.map(_cpu_slice, jobs)
            dta = time.perf_counter() - t
    cells = sum(c for c, _ in res)
    va = float(cells / dta)
    return dict(value=va, unit="DM-time samples/s", cores=workers, kind="oracle",
                sample=f"shared-pattern SND tree (C, FP64) over all {spec.dms.size} DMs x {n_sample_all} output "
                       f"samples of the same 1024-channel beam, one process per contiguous DM slice on {workers} "
                       f"cores; {dta:.1f} s",
                seconds=round(dta, 2), host_cpus=ncpu, cpu_model=model,
                single_thread={"value": v1, "unit": "DM-time samples/s", "cores": 1,
                               "sample": f"all {spec.dms.size} DMs x {n_sample} output samples, 1 thread; "
                                         f"{dt1:.1f} s"}), np.asarray(y).shape


def direct_leg(snd, torch, spec, x, pkw, dev, ref_out, reps=3):
    """Comparison baseline on the same block: direct dedispersion, every DM row summing every
    channel at its own delay, with no neuron shared between DMs (a plan with no materialised
    level: SND_STAGE_NONE).  Float sums keep the tree's association, so the plane must equal
    the shared-neuron plane bit for bit."""
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, stage_levels=0x80000000, **pkw)
    p.upload(dev)
    out = p.empty_output(dev)
    ws = p.workspace(dev)
    stream = torch.cuda.current_stream(dev)
    p.execute(x, out=out, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p.execute(x, out=out, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = p.info
    a, b = out.float(), ref_out.float()
    rel = float(torch.sqrt(torch.mean((a - b) ** 2)) / torch.sqrt(torch.mean(b ** 2)).clamp_min(1e-30))
    return dict(method="direct (no shared neurons)", ms=round(ms, 3), value=p.ndm * p.n_out / (ms * 1e-3),
                unit="DM-time samples/s", kernel=info["stage_kernel"][0], inputs_per_sample=info["stage_entries"][0],
                identical_to_snd=bool(torch.equal(out, ref_out)), rel_rms_vs_snd=rel)


def trees_leg(snd, torch, spec, zt, dev, reps=3):
    """The tree alone (every stage, no detection) on the same block for each mode and storage,
    with the default branching B = 4 and the paper's own tree (Table S1: C = 4, B = 8, a
    4-input root): milliseconds per block, the final stage's kernel and its share."""
    rows = []
    variants = [("float", "f32", 4), ("float", "f32", 8), ("float", "bf16", 4), ("float", "bf16", 8),
                ("graded", "u8", 4), ("graded", "u8", 8), ("binary", "bits", 4), ("binary", "bits", 8)]
    for mode, node, B in variants:
        if mode == "float":
            x = zt if node == "f32" else snd.cast(zt, node)
            in_dtype = None if node == "f32" else node
        elif mode == "graded":
            x, in_dtype = snd.encode(zt, [1.0, 2.0, 3.0, 4.0]), None
        else:
            x, in_dtype = snd.encode_bits(zt, 2.0), "bits"
        p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode=mode, branching=B, cluster=spec.cluster,
                     k_leaf=2, k_int=1, cap=255, node_dtype=node, in_dtype=in_dtype)
        p.upload(dev)
        out = p.empty_output(dev)
        ws = p.workspace(dev)
        stream = torch.cuda.current_stream(dev)
        p.execute(x, out=out, workspace=ws)
        torch.cuda.synchronize()
        ns = p.info["n_stages"]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)]
        tot = [0.0] * ns
        for _ in range(reps):
            ev[0].record(stream)
            for st in range(ns):
                p.execute(x, out=out, workspace=ws, stage=st)
                ev[st + 1].record(stream)
            torch.cuda.synchronize()
            for st in range(ns):
                tot[st] += ev[st].elapsed_time(ev[st + 1]) / reps
        ms = sum(tot)
        rows.append(dict(mode=mode, storage=node, branching=B, ms=round(ms, 3),
                         stage_ms=[round(t, 3) for t in tot], kernels=p.info["stage_kernel"],
                         value=p.ndm * p.n_out / (ms * 1e-3), neurons=p.info["n_neurons"],
                         synapses=p.info["n_synapses"]))
        log(f"[bench] tree {mode}/{node} B={B}: {ms:.3f} ms {p.info['stage_kernel']}")
        del p, out, ws, x
        torch.cuda.empty_cache()
    return dict(workload="the same 1024 ch x 2^17 block, 4096 DMs 0-2000, C = 4", unit="DM-time samples/s",
                rows=rows)


def subband_leg(snd, torch, spec, x, pkw, dev, ref_out, reps=3):
    """Sub-band dedispersion on the same block, in its exact form: a two-level tree of 32
    sub-bands of 32 channels (each sub-band's partial sums shared by the DMs with the same
    delay pattern inside it) and one 32-input root per DM.  Float mode only: the tree is
    linear there, so the plane equals the SND plane up to FP32 association."""
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, **dict(pkw, cluster=32, branching=32))
    p.upload(dev)
    out = p.empty_output(dev)
    ws = p.workspace(dev)
    stream = torch.cuda.current_stream(dev)
    p.execute(x, out=out, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p.execute(x, out=out, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    info = p.info
    a, b = out.float(), ref_out.float()
    rel = float(torch.sqrt(torch.mean((a - b) ** 2)) / torch.sqrt(torch.mean(b ** 2)).clamp_min(1e-30))
    res = dict(method="sub-band (exact two-level tree: 32 sub-bands x 32 channels)", ms=round(ms, 3),
               value=p.ndm * p.n_out / (ms * 1e-3), unit="DM-time samples/s", kernels=info["stage_kernel"],
               sub_band_rows=info["stage_rows"][0], inputs_per_sample=sum(info["stage_entries"]),
               rel_rms_vs_snd=rel)
    del out, ws, p
    torch.cuda.empty_cache()
    return res


def subband_approx_leg(snd, torch, spec, x, dev, ref_out, nsub=32, coarse_step=8, reps=3):
    """Approximate (coarse-DM) sub-band dedispersion on the same float block: SND plans per
    sub-band over every coarse_step-th DM, then one combine kernel for the fine DMs.  Cheaper
    than the exact tree, at the cost of each sub-band's internal sweep taken at the coarse DM:
    its error against the SND plane is reported with its time."""
    import numpy as np
    sb = snd.SubbandApprox(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, nsub=nsub, coarse_step=coarse_step,
                           device=dev)
    out = sb.empty_output()
    stream = torch.cuda.current_stream(dev)
    sb.execute(x, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sb.execute(x, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = min(sb.n_out, ref_out.shape[1])
    a, b = out[:, :n].float(), ref_out[:, :n].float()
    rel = float(torch.sqrt(torch.mean((a - b) ** 2)) / torch.sqrt(torch.mean(b ** 2)).clamp_min(1e-30))

    # sensitivity: boxcar S/N of each injected pulse at its nearest trial DM in both planes
    def pulse_snr(plane, k, t0):
        row = plane[k, :n].double()
        sd = float(row.std())
        lo, hi = max(0, t0 - 64), min(n, t0 + 128)
        c = torch.cat([torch.zeros(1, dtype=row.dtype, device=row.device), torch.cumsum(row[lo:hi] - row.mean(), 0)])
        best = 0.0
        for w in (1, 2, 4, 8, 16, 32, 64):
            if hi - lo > w:
                best = max(best, float((c[w:] - c[:-w]).max()) / (sd * w ** 0.5))
        return best
    ratios = []
    for pl in spec.pulses:
        k = int(np.argmin(np.abs(spec.dms - pl.dm)))
        t0 = int(round(pl.t0))
        if t0 + 128 < n:
            s_snd = pulse_snr(b, k, t0)
            if s_snd > 0:
                ratios.append(pulse_snr(a, k, t0) / s_snd)
    res = dict(method=f"approximate sub-band ({nsub} sub-bands, every {coarse_step}th DM coarse)", ms=round(ms, 3),
               value=sb.ndm * sb.n_out / (ms * 1e-3), unit="DM-time samples/s", coarse_dms=int(sb.coarse.size),
               n_out=sb.n_out, rel_rms_vs_snd=rel,
               pulse_snr_ratio_vs_snd=dict(mean=round(float(np.mean(ratios)), 3) if ratios else None,
                                           min=round(float(np.min(ratios)), 3) if ratios else None,
                                           pulses=len(ratios)))
    del sb, out
    torch.cuda.empty_cache()
    return res


def completeness(snd, spec, cands, n_out):
    """Injected pulses of the block recovered by the candidates: greedy one-to-one matching in
    decreasing S/N with |dDM| <= 10 and |dt| <= 0.5 W_eff (snd_match_injections).  cands:
    dicts with dm, snr and the peak boxcar's first sample t and width in native samples
    (t_centre = t + (width - 1) / 2).  Only pulses arriving inside the n_out valid samples
    count."""
    tms = spec.tsamp_s * 1e3
    pulses = [p for p in spec.pulses if 0.0 <= p.t0 < n_out]
    if not pulses:
        return None
    weff = snd.effective_width(spec.freqs, spec.tsamp_s, [p.dm for p in pulses], [p.width_ms for p in pulses])
    match, n = snd.match_injections([c["dm"] for c in cands], [(c["t"] + 0.5 * (c["width"] - 1)) * tms for c in cands],
                                    [c["snr"] for c in cands], [p.dm for p in pulses], [p.t0 * tms for p in pulses],
                                    weff, 10.0, 0.5)
    return dict(injected=len(pulses), matched=n, completeness=round(n / len(pulses), 4), candidates=len(cands),
                rule="greedy one-to-one in decreasing S/N; |dDM| <= 10, |dt| <= 0.5 W_eff")


def multirate_leg(snd, torch, spec, zt, mode, dev, reps=3):
    """The same block through the multi-rate pipeline: DM bands by scrunch factor (S = 1..16),
    one plan per band on a scrunched, re-encoded copy, detection per band, cross-band merge."""
    thr = {"float": None, "graded": [1.0, 2.0, 3.0, 4.0], "binary": [2.0]}[mode]
    kw = dict(k_leaf=2, k_int=1) if mode == "binary" else {}
    t = time.perf_counter()
    mr = snd.MultiRate(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode=mode, thresholds=thr,
                       widths=spec.widths, threshold=7.0, branching=spec.branching, device=dev, **kw)
    build_s = time.perf_counter() - t
    merged, _ = mr.run(zt)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        merged, per_band = mr.run(zt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    bands = [dict(s=b["s"], dms=int(b["idx"].size), n_out=b["plan"].n_out, candidates=len(pb))
             for b, pb in zip(mr.bands, per_band)]
    # merged candidates in native samples: band sample t of scrunch s starts at native s t
    native = [dict(dm=c["dm"], snr=c["snr"], t=c["t"] * mr.bands[c["band"]]["s"],
                   width=c["width"] * mr.bands[c["band"]]["s"]) for c in merged]
    n_out = min(b["plan"].n_out * b["s"] for b in mr.bands)
    return dict(method="multi-rate (scrunch bands, per-band trees, merged candidates)", mode=mode,
                ms_per_block=round(ms, 3), plan_build_s=round(build_s, 2), bands=bands, candidates=len(merged),
                detection=completeness(snd, spec, native, n_out),
                note="includes scrunch, encode, trees, detection of every band and the merge; synchronous")


def fdmt_leg(snd, torch, spec, zt, tree_ms, reps=3):
    """FDMT with the no-smear initialisation on the same float32 block, DM 0-2000: one row per
    integer band sweep (28,353 rows against the tree's 4096 DMs)."""
    bw = float(abs(spec.freqs[0] - spec.freqs[1]))
    fd = snd.Fdmt(spec.freqs, bw, spec.tsamp_s, float(spec.dms.max()), spec.nsamp)
    out = fd.execute(zt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fd.execute(zt, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # algorithmic bytes: every merge reads two source samples and writes one per output sample,
    # over the rows of all merges
    alg = fd.table_rows * spec.nsamp * 12
    rows = fd.n_delays
    value = rows * fd.n_out / (ms * 1e-3)
    del out, fd
    torch.cuda.empty_cache()
    return dict(method="FDMT, no-smear initialisation (log2 1024 = 10 merges)", ms=round(ms, 3),
                rows=rows, dm_step=round(float(spec.dms.max()) / (rows - 1), 5),
                value=value, unit="DM-time samples/s", us_per_dm_row=round(ms * 1e3 / rows, 3),
                snd_tree_ms=round(tree_ms, 3), snd_us_per_dm_row=round(tree_ms * 1e3 / spec.dms.size, 3),
                alg_gb=round(alg / 1e9, 1), achieved_gbs=round(alg / (ms * 1e-3) / 1e9, 1),
                hbm_frac=round(alg / (ms * 1e-3) / 8e12, 3))


def completeness_leg(snd, synth, torch, spec, dev, blocks=8):
    """Completeness against injected S/N (Methods, "Validation methodology"), on synthetic
    blocks of the headline shape through the multi-rate pipeline at the paper's operating points
    (Table S1) with its tree (C = 4, B = 8, root of 4): binary 1.5 sigma spikes, K_L = K_I = 2,
    sigma_min 0.20; graded 0.75 sigma spikes
    summed to cap 255; float on the z-scored data; Theta = 7 and the DM-scaled width set
    {1, 2, 4, 8} + {16 .. 1024} with alpha = 0.1 in every mode.  Per block 16 pulses with DM
    log-uniform in [20, 2000] (the grid's range; the paper's reaches 3000), intrinsic width
    log-uniform in [0.5, 130] ms and matched-filter S/N uniform in [3, 13].  Gaussian noise only:
    no RFI, so false positives are not the paper's."""
    import math

    import numpy as np
    widths = [1 << i for i in range(11)]
    ops = {"float": dict(thresholds=None, kw={}),
           "graded": dict(thresholds=[0.75], kw=dict(cap=255)),
           "binary": dict(thresholds=[1.5], kw=dict(k_leaf=2, k_int=2), sigma_min=0.2)}
    # the paper's Northern Cross tree (Table S1): clusters of 4, branching 8, a 4-input root
    pipes = {m: snd.MultiRate(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode=m, thresholds=o["thresholds"],
                              widths=widths, threshold=7.0, sigma_min=o.get("sigma_min", 0.0),
                              branching=8, cluster=4, device=dev,
                              detect_kw=dict(n_base_widths=4, width_alpha=0.1), **o["kw"])
             for m, o in ops.items()}
    tms = spec.tsamp_s * 1e3
    edges = [3, 5, 7, 9, 11, 13.0001]
    sweep = synth.configs.sweep_samples(spec.freqs, 2000.0, spec.tsamp_s)
    nchan = spec.freqs.size
    out = dict(method="completeness vs injected S/N, multi-rate pipeline, paper operating points", blocks=blocks,
               snr_bins=[f"{edges[i]:.0f}-{edges[i + 1]:.0f}" for i in range(5)])
    # the S/N of an injection is the dedispersed matched-filter S/N of the pulse ("total")
    for conv, scale in (("total", 1.0),):
        hit = {m: np.zeros(len(edges) - 1) for m in ops}
        cnt = np.zeros(len(edges) - 1)
        cands = {m: 0 for m in ops}
        for b in range(blocks):
            rng = synth.make_rng(7000 + b)
            t0 = synth.random_pulse_slots(rng, 16, 300.0, spec.nsamp - sweep - 1500.0)
            dms = np.exp(rng.uniform(math.log(20.0), math.log(2000.0), 16))
            ws = np.exp(rng.uniform(math.log(0.5), math.log(130.0), 16))
            snrs = rng.uniform(3.0, 13.0, 16)
            pulses = [synth.Pulse(float(d), float(t), float(w), float(q * scale), 0.0)
                      for d, t, w, q in zip(dms, t0, ws, snrs)]
            z = synth.noise_filterbank(rng, nchan, spec.nsamp)
            synth.inject_pulses(z, spec.freqs, spec.tsamp_s, pulses)
            zt = torch.from_numpy(z).to(dev)
            del z
            weff = snd.effective_width(spec.freqs, spec.tsamp_s, dms, ws)
            bins = np.clip(np.searchsorted(edges, snrs, side="right") - 1, 0, len(edges) - 2)
            np.add.at(cnt, bins, 1)
            for m, mr in pipes.items():
                merged, _ = mr.run(zt)
                nat = [(c["dm"], (c["t"] * mr.bands[c["band"]]["s"] +
                                  0.5 * (c["width"] * mr.bands[c["band"]]["s"] - 1)) * tms, c["snr"]) for c in merged]
                match, _ = snd.match_injections([c[0] for c in nat], [c[1] for c in nat], [c[2] for c in nat], dms,
                                                t0 * tms, weff, 10.0, 0.5)
                np.add.at(hit[m], bins, (np.asarray(match) >= 0).astype(float))
                cands[m] += len(merged)
            del zt
        out[conv] = dict(injections_per_bin=[int(v) for v in cnt],
                         completeness={m: [round(float(h / c), 3) if c else None for h, c in zip(hit[m], cnt)]
                                       for m in ops},
                         overall={m: round(float(hit[m].sum() / cnt.sum()), 3) for m in ops},
                         candidates_per_block={m: round(cands[m] / blocks, 1) for m in ops})
    torch.cuda.empty_cache()
    return out


def frontend_leg(snd, torch, spec, dev, reps=3):
    """The on-device front end on one raw-power block of the same shape: two-pass sigma-clip
    statistics, normalisation, windowed MAD channel flagging (8192-sample windows, 5 MADs),
    zero-DM subtraction (gamma 5) and the delta encoder to bits (1.5 sigma).  Raw power is
    synthetic: exponential (chi-squared, 2 degrees of freedom) with per-channel gain and offset,
    one hot channel and broadband bursts."""
    import numpy as np
    rng = np.random.default_rng(99)
    nchan, n = spec.freqs.size, spec.nsamp
    p = rng.standard_exponential((nchan, n), dtype=np.float32)
    p *= rng.uniform(0.5, 3.0, (nchan, 1)).astype(np.float32)
    p += rng.uniform(0.0, 10.0, (nchan, 1)).astype(np.float32)
    p[100, : n // 4] *= 8.0
    p[:, ::20011] += 5.0
    pt = torch.from_numpy(p).to(dev)
    del p
    z = torch.empty_like(pt)
    bits = torch.empty((nchan, (n + 31) // 32), dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    names = ("channel_stats", "normalize", "flag_channels", "zero_dm", "encode_bits")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
    ms = np.zeros(len(names))
    for r in range(reps + 1):
        ev[0].record()
        st = snd.channel_stats(pt, 5.0)
        ev[1].record()
        snd.normalize(pt, st, out=z)
        ev[2].record()
        flags = snd.flag_channels(z, 8192, 5.0)
        ev[3].record()
        snd.zero_dm(z, 5.0, count=cnt)
        ev[4].record()
        snd.encode_bits(z, 1.5, out=bits)
        ev[5].record()
        torch.cuda.synchronize()
        if r:  # the first pass warms up
            ms += [ev[i].elapsed_time(ev[i + 1]) for i in range(len(names))]
    ms /= reps
    nflag = int(flags.sum().item())
    return dict(method="front end on raw power", workload=f"{nchan} ch x {n} samples float32 raw power (synthetic)",
                ms={k: round(float(v), 3) for k, v in zip(names, ms)}, total_ms=round(float(ms.sum()), 3),
                flagged_channel_windows=nflag, zero_dm_samples_per_block=int(cnt.item()) // (reps + 1))


def batch_leg(snd, synth, torch, dev, reps=3):
    """48 beams x 1024 ch x 2^16 samples, uneven DM grids (1024-4096 trials, max DM 500-2000), modes
    rotating binary / graded / float with float storage rotating f32 / bf16 / f16: one batched
    execute (shared grids) against one execute per beam."""
    import numpy as np
    specs = [synth.batch_beam(b) for b in range(48)]
    t = time.perf_counter()
    plans = []
    for s_ in specs:
        inp = s_.node_dtype if s_.mode != "graded" else "u8"  # float storage, binary bit rows, graded bytes
        plans.append(snd.Plan(s_.freqs, s_.dms, s_.tsamp_s, s_.nsamp, mode=s_.mode, branching=4, k_leaf=s_.k_leaf,
                              k_int=s_.k_int, node_dtype=s_.node_dtype, in_dtype=inp))
    t_plan = time.perf_counter() - t
    xs = []
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.seed_for(4))
    for s_, p in zip(specs, plans):
        z = torch.randn(s_.nchan, s_.nsamp, device=dev, generator=gen)
        if s_.mode == "float":
            xs.append(z if p.in_dtype == "f32" else snd.cast(z, p.in_dtype))
        elif p.in_dtype == "bits":
            xs.append(snd.encode_bits(z, s_.enc_thresholds[0]))
        else:
            xs.append(snd.encode(z, list(s_.enc_thresholds)))
        del z
    batch = snd.Batch(plans, dev)
    outs = [p.empty_output(dev) for p in plans]
    samples = sum(p.ndm * p.n_out for p in plans)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_batch = timed(lambda: batch.execute(xs, outs))
    ms_single = timed(lambda: [p.execute(x, out=o, workspace=w)
                               for p, x, o, w in zip(plans, xs, outs, batch.workspaces)])
    # tuned against default: launch shapes tuned once per beam class (mode, storage) on its first
    # beam (cached on disk), applied to every beam of the class, the batch timed again
    tw = snd.tune_word
    shapes = [0, tw(xcd_groups=1), tw(xcd_groups=2), tw(xcd_groups=16), tw(lds_quarters_off=1),
              tw(lds_quarters_off=2), tw(leaf_window=1024), tw(leaf_window=512)]
    classes = {}
    for i, p in enumerate(plans):
        classes.setdefault((p.mode, p.node_dtype), []).append(i)
    tuned_rows, best_tune = [], {}
    for key, idx in classes.items():
        s_, p0 = specs[idx[0]], plans[idx[0]]
        kw = dict(mode=s_.mode, branching=4, k_leaf=s_.k_leaf, k_int=s_.k_int, node_dtype=p0.node_dtype,
                  in_dtype=p0.in_dtype)
        best, recs, hit = snd.autotune_cached(s_.freqs, s_.dms, s_.tsamp_s, xs[idx[0]], [(0, 0, t) for t in shapes],
                                              nsamp=s_.nsamp, reps=2, **kw)
        best_tune[key] = best[2]
        ok = [r["ms"] for r in recs if r["ms"] > 0]
        tuned_rows.append(dict(mode=key[0], storage=key[1], beams=len(idx), default_ms=round(recs[0]["ms"], 3),
                               tuned_ms=round(min(ok), 3), tune=snd.tune_fields(best[2]), cache_hit=hit))
        log(f"[bench] batch class {key}: default {recs[0]['ms']:.3f} ms, tuned {min(ok):.3f} ms "
            f"{snd.tune_fields(best[2])}")
    del batch
    torch.cuda.empty_cache()
    plans_t = []
    for s_, p in zip(specs, plans):
        plans_t.append(snd.Plan(s_.freqs, s_.dms, s_.tsamp_s, s_.nsamp, mode=s_.mode, branching=4, k_leaf=s_.k_leaf,
                                k_int=s_.k_int, node_dtype=p.node_dtype, in_dtype=p.in_dtype,
                                tune=best_tune[(p.mode, p.node_dtype)]))
    batch = snd.Batch(plans_t, dev)
    ms_tuned = timed(lambda: batch.execute(xs, outs))
    res = dict(workload="48 beams x 1024 ch x 2^16 samples; DM grids 1024-4096 trials to 500-2000; "
                        "modes binary (bit rows) / graded (u8) / float (f32/bf16/f16); B=4; synthetic N(0,1) "
                        "encoded on the device",
               ms_batched_tuned=round(ms_tuned, 3), tuned_classes=tuned_rows,
               beams=48, grids=batch.n_launches, plan_build_s=round(t_plan, 2),
               dm_time_samples=int(samples), ms_batched=round(ms_batch, 3), ms_per_beam_launches=round(ms_single, 3),
               value_batched=samples / (ms_batch * 1e-3), value_per_beam=samples / (ms_single * 1e-3),
               unit="DM-time samples/s", workspace_gib=round(sum(w.numel() for w in batch.workspaces) / 2**30, 2))
    del xs, outs, batch
    torch.cuda.empty_cache()
    return res


class _ChunkSource:
    """Z-scored 1024-channel chunks on the device for the serving runs: a pool of N(0,1) chunks
    (reused round-robin, so that drawing a chunk costs one device copy) plus dispersed pulses
    from a few pre-built templates, placed at random times per beam."""

    def __init__(self, snd, synth, torch, dev, nchan, chunk, nbeams, seconds, pool=12, ntemplates=6):
        import numpy as np
        self.torch, self.dev, self.T = torch, dev, chunk
        gen = torch.Generator(device=dev)
        gen.manual_seed(synth.seed_for(5))
        self.pool = [torch.randn(nchan, chunk, device=dev, generator=gen) for _ in range(pool)]
        rng = synth.make_rng(synth.seed_for(5, 99))
        freqs = synth.channel_freqs(nchan)
        self.templates = []
        for i in range(ntemplates):
            dm = float(rng.uniform(100.0, 1800.0))
            width = float(np.exp(rng.uniform(np.log(0.5), np.log(5.0))))
            sweep = int(synth.KDM_MS * dm * (freqs.min() ** -2 - freqs.max() ** -2) / (synth.TSAMP_S * 1e3))
            span = sweep + 200
            z = np.zeros((nchan, span), np.float32)
            synth.inject_pulses(z, freqs, synth.TSAMP_S, [synth.Pulse(dm=dm, t0=60.0, width_ms=width,
                                                                      snr=float(rng.uniform(15, 40)))])
            self.templates.append(torch.from_numpy(z).to(dev))
        # one pulse every ~8 s per beam at a random template and phase
        total = int(seconds / (chunk * synth.TSAMP_S) + 2) * chunk
        self.pulses = {}
        for b in range(nbeams):
            n = max(1, int(seconds / 8))
            starts = np.sort(rng.uniform(0, total, n)).astype(np.int64)
            self.pulses[b] = [(int(s0), int(rng.integers(ntemplates))) for s0 in starts]

    def __call__(self, beam, idx):
        z = self.pool[(beam * 7 + idx) % len(self.pool)].clone()
        lo, hi = idx * self.T, (idx + 1) * self.T
        for s0, k in self.pulses.get(beam, ()):
            tpl = self.templates[k]
            a, b = max(lo, s0), min(hi, s0 + tpl.shape[1])
            if a < b:
                z[:, a - lo:b - lo] += tpl[:, a - s0:b - s0]
        return z


class _PlainServer:
    """The plain per-beam form for comparison: each chunk is appended to an explicit overlap
    buffer (the previous max_delay samples + the chunk), the buffer is encoded or cast and
    executed with its own launches, then detected."""

    def __init__(self, snd, torch, kinds, dev):
        self.snd, self.torch, self.dev, self.kinds = snd, torch, dev, kinds
        self.kind_of, self.buf, self.filled, self.out, self.nidx = {}, {}, {}, {}, {}
        self.det = {k: snd.Detector(p, widths=(1, 2, 4, 8, 16, 32, 64), threshold=7.0, device=dev)
                    for k, (p, _) in kinds.items()}
        self.ws = torch.empty(max(p.info["workspace_bytes"] for p, _ in kinds.values()), dtype=torch.uint8,
                              device=dev)

    def admit(self, beam, kind):
        p = self.kinds[kind][0]
        self.kind_of[beam] = kind
        self.buf[beam] = self.torch.zeros(p.nchan, p.nsamp, device=self.dev)
        self.filled[beam] = 0
        self.out[beam] = p.empty_output(self.dev)
        return True

    def evict(self, beam):
        for d in (self.kind_of, self.buf, self.filled, self.out):
            d.pop(beam, None)

    def beams(self):
        return sorted(self.kind_of)

    def next_index(self, beam):
        return self.nidx.get(beam, 0)

    def process(self, ready):
        done = []
        for beam, idx, z in ready:
            p, thr = self.kinds[self.kind_of[beam]]
            buf, T, D = self.buf[beam], z.shape[1], p.max_delay
            self.nidx[beam] = idx + 1
            buf[:, :D] = buf[:, T:T + D].clone()
            buf[:, D:D + T] = z
            self.filled[beam] += T
            if self.filled[beam] < D + T:
                done.append((beam, idx, 0, 0, None))
                continue
            x = self.snd.encode(buf, thr) if thr is not None else self.snd.cast(buf, p.in_dtype)
            p.execute(x, out=self.out[beam], workspace=self.ws)
            done.append((beam, idx, 0, T, self.det[self.kind_of[beam]].run(self.out[beam])))
        return done


def serve_leg(snd, synth, torch, dev, seconds):
    """Streaming service (48 beams of 1024 ch, 8192-sample chunks = 1.13 s, arrivals at a random
    phase with inter-arrival 1.13 s x U(0.8, 1.2); half graded (4-level u8), half BF16 float;
    4096 DMs to 2000, B = 4; history budget for about 44 beams; 40 beams at start, one leaves and
    one joins every 10 s).  Real-time runs of the batched streaming form and of the plain per-beam
    form, then a saturation run of each (all chunks ready at once) for capacity."""
    import numpy as np
    from paper_2606_15361_amd import serve
    T = 8192
    sg, sf = synth.stream_beam(0, T), synth.stream_beam(1, T)
    pg = snd.Plan(sg.freqs, sg.dms, sg.tsamp_s, None, mode="graded", branching=4, chunk=T)
    pf = snd.Plan(sf.freqs, sf.dms, sf.tsamp_s, None, mode="float", branching=4, chunk=T, in_dtype="bf16",
                  node_dtype="bf16")
    kinds = {"graded": (pg, [1.0, 2.0, 3.0, 4.0]), "bf16": (pf, None)}
    budget = 22 * snd.admission_bytes(pg) + 22 * snd.admission_bytes(pf)
    period = synth.chunk_period_s(T)
    src = _ChunkSource(snd, synth, torch, dev, 1024, T, 48, max(seconds, 30.0) + 30.0)
    kind = lambda b: "graded" if b % 2 == 0 else "bf16"
    out = {}
    for form in ("batched_stream", "plain_per_beam"):
        rng = synth.make_rng(synth.seed_for(5, 7))  # the same arrivals for both forms
        if form == "batched_stream":
            server = serve.Server(kinds, budget, batched=True, device=dev)
        else:
            server = _PlainServer(snd, torch, kinds, dev)
        for b in range(40):
            assert server.admit(b, kind(b))
        arr = {b: a for b, a in enumerate(synth.arrival_times(rng, 48, seconds + 5.0, period))}
        # beam i leaves at 10 (i + 1) s; the joining beam cycles through the 48 (after the 8 not
        # yet started, the beams that left first come back)
        joins = [(10.0 * (i + 1), (40 + i) % 48, kind((40 + i) % 48)) for i in range(int(seconds // 10))]
        leaves = [(10.0 * (i + 1), i) for i in range(int(seconds // 10))]
        log(f"[bench] serving ({form}) for {seconds:.0f} s")
        recs, adm = serve.run_schedule(server, arr, src, duration_s=seconds, joins=joins, leaves=leaves, log=log)
        lat = np.array([r["latency"] for r in recs if r["counted"]])
        nout = sum(1 for r in recs if r["counted"])
        out[form] = dict(chunks=len(recs), counted=int(nout),
                         p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3) if lat.size else None,
                         p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3) if lat.size else None,
                         candidates_per_s=round(sum(r["candidates"] for r in recs) / seconds, 3),
                         admissions=[dict(t=a[0], beam=a[1], kind=a[2], admitted=a[3]) for a in adm])
        # saturation: every beam has a chunk ready at once, rounds back to back (after the
        # histories are full), outputs counted as produced
        beams = server.beams()
        nxt = {b: server.next_index(b) for b in beams}
        for r in range(4):  # fill the histories of recently joined beams
            server.process([(b, nxt[b] + r, src(b, nxt[b] + r)) for b in beams])
        torch.cuda.synchronize()
        nround, produced = 6, 0
        t0 = time.perf_counter()
        for r in range(4, 4 + nround):
            res = server.process([(b, nxt[b] + r, src(b, nxt[b] + r)) for b in beams])
            produced += sum(n for _, _, _, n, _ in res)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[form]["saturated_beams"] = len(beams)
        out[form]["saturated_chunks_per_s"] = round(nround * len(beams) / dt, 2)
        out[form]["saturated_dm_time_samples_per_s"] = produced * pg.ndm / dt
        del server
        torch.cuda.empty_cache()
    # offered load: the same 40 beams with their arrival period compressed f times; a form
    # sustains load f while its p99 latency stays within the chunk's real-time duration
    sweep = {}
    for form in ("batched_stream", "plain_per_beam"):
        rows = []
        for f in (1, 5, 10, 15, 20, 22, 24, 26):
            server = (serve.Server(kinds, budget, batched=True, device=dev) if form == "batched_stream"
                      else _PlainServer(snd, torch, kinds, dev))
            for b in range(40):
                assert server.admit(b, kind(b))
            rng = synth.make_rng(synth.seed_for(5, 11))
            dur = 6.0
            arr = {b: a for b, a in enumerate(synth.arrival_times(rng, 40, dur + 1.0, period / f))}
            recs, _ = serve.run_schedule(server, arr, src, duration_s=dur, warm_chunks=5)
            lat = np.array([r["latency"] for r in recs if r["counted"]])
            offered = 40 * f / period
            rows.append(dict(load=f, offered_chunks_per_s=round(offered, 1), chunks=len(recs),
                             served_chunks_per_s=round(len(recs) / dur, 1),
                             p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3) if lat.size else None,
                             p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3) if lat.size else None))
            log(f"[bench] serving sweep {form} load {f}x: {rows[-1]}")
            del server
            torch.cuda.empty_cache()
        ok = [r["load"] for r in rows if r["p99_ms"] is not None and r["p99_ms"] < period * 1e3
              and r["served_chunks_per_s"] >= 0.98 * r["offered_chunks_per_s"]]
        sweep[form] = dict(rows=rows, max_sustained_load=max(ok) if ok else None)
    sweep["note"] = ("40 beams, arrival period 1.1305 s / load, 6 s per point; latency = arrival to candidates "
                     "on the host; sustained = p99 below 1130.5 ms and at least 98 % of the offered chunks served")
    out["load_sweep"] = sweep
    out["workload"] = ("48 beams x 1024 ch, 8192-sample chunks (1.1305 s), arrivals period x U(0.8,1.2); half graded "
                       "u8 / half bf16 float; 4096 DMs to 2000; B=4; history budget ~44 beams; 40 at start, one "
                       "leaves and one joins every 10 s")
    out["seconds"] = seconds
    out["real_time_bound_ms"] = round(period * 1e3, 1)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2606_15361_amd as snd
    import synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del a, b
    spec = synth.workload(2)
    mode = args.mode
    log(f"[bench] generating the 1024 x {spec.nsamp} filterbank")
    z = spec.filterbank()
    zt = torch.from_numpy(z).to(dev)
    if mode == "float":
        x = zt
    node = args.node_dtype
    in_dtype = None
    if mode == "binary" and args.input != "bytes" and node in (None, "bits"):
        in_dtype = "bits"  # spikes as bit rows, straight from the encoder
        x = snd.encode_bits(zt, 2.0)
    elif mode != "float":
        x = snd.encode(zt, [1.0, 2.0, 3.0, 4.0] if mode == "graded" else [2.0])
    if mode == "float" and node in ("bf16", "f16"):
        in_dtype = node
        x = snd.cast(zt, node)
    del zt
    pkw = dict(mode=mode, branching=spec.branching, cluster=spec.cluster, k_leaf=2, k_int=1, cap=255,
               node_dtype=node, in_dtype=in_dtype, generic_kernels=args.generic_kernels)
    tuned = None
    tune = 0
    stage_levels = args.stage_levels
    if not args.no_autotune and not args.stage_levels and not args.generic_kernels:
        # measured choice of the stage schedule: leaves only, level 2 only, leaves and level 2
        # and of the launch shapes (snd_plan_desc.tune); the choice is cached on disk per GPU
        # architecture, mode, storage and tree shape
        tw = snd.tune_word
        cands = [(0, 0, 0), (0b0100, 0, 0), (0b0101, 0, 0), (0, 0, tw(xcd_groups=1)), (0, 0, tw(xcd_groups=2)),
                 (0, 0, tw(xcd_groups=16)), (0, 0, tw(lds_quarters_off=1)), (0, 0, tw(leaf_window=1024))]
        best, tuned, hit = snd.autotune_cached(spec.freqs, spec.dms, spec.tsamp_s, x, cands, reps=1, nsamp=spec.nsamp,
                                               **pkw)
        stage_levels, tune = best[0], best[2]
        for t in tuned:
            t["tune"] = snd.tune_fields(t["tune"])
        log(f"[bench] autotune ({'cached' if hit else 'timed'}): "
            f"{[(hex(t['stage_levels']), round(t['ms'], 2)) for t in tuned]} -> {stage_levels:#x}, tune {tune:#x}")
        torch.cuda.empty_cache()
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, stage_levels=stage_levels, tune=tune, **pkw)
    info = plan.info
    log(f"[bench] plan: {info['n_neurons']} neurons, {info['n_synapses']} synapses, stages {info['stage_rows']}, "
        f"workspace {info['workspace_bytes'] / 2**30:.2f} GiB, built in {info['build_seconds']:.2f} s")
    plan.upload(dev)
    ws = plan.workspace(dev)
    # two output planes: a block's plane stays intact while the next block's tree runs and
    # the host extracts the block's candidates
    outs = [plan.empty_output(dev), plan.empty_output(dev)]
    detector = None
    if not args.no_detect and hasattr(snd, "Detector"):
        detector = snd.Detector(plan, widths=spec.widths, threshold=7.0, device=dev)
    nst = info["n_stages"]
    stream = torch.cuda.current_stream(dev)
    pipeline = detector is not None and not args.serial_detect

    def step(k, evs=None, pending=None):
        """Block k: the tree, then detection.  Pipelined, the detection is only launched here
        and the previous block's candidates are collected (host work) while this block runs."""
        out = outs[k % 2]
        for s in range(nst):
            plan.execute(x, out=out, workspace=ws, stage=s)
            if evs is not None:
                evs[s + 1].record(stream)
        if detector is None:
            return None, None
        if not pipeline:
            cands = detector.run(out)
            if evs is not None:
                evs[nst + 1].record(stream)
            return cands, None
        ticket = detector.launch(out)
        if evs is not None:
            evs[nst + 1].record(stream)
        cands = detector.collect(pending) if pending is not None else None
        return cands, ticket

    pending = None
    for k in range(args.warmup):
        _, pending = step(k, pending=pending)
    if pending is not None:
        detector.collect(pending)
        pending = None
    torch.cuda.synchronize()
    nev = nst + 2
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ncand = 0
    last = None
    for k in range(args.steps):
        events[k][0].record(stream)
        c, pending = step(k, events[k], pending)
        if c is not None:
            last = c
    if pending is not None:
        last = detector.collect(pending)
    if last is not None:
        ncand = len(last)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = np.zeros(nst)
    det_ms = 0.0
    for k in range(args.steps):
        for s in range(nst):
            stage_ms[s] += events[k][s].elapsed_time(events[k][s + 1])
        if detector is not None:
            det_ms += events[k][nst].elapsed_time(events[k][nst + 1])
    stage_ms /= args.steps
    det_ms /= args.steps
    ms_step = wall * 1e3 / args.steps
    samples = spec.dms.size * plan.n_out
    value = samples / (wall / args.steps)
    dom = int(np.argmax(stage_ms))
    alg = info["stage_alg_bytes"][dom]
    achieved = alg / (stage_ms[dom] * 1e-3) / 1e9
    kname = KERNEL_SYMBOL[info["stage_kernel"][dom]]
    node = plan.node_dtype
    wl_key = f"{mode}-{plan.in_dtype}-{node}-stage{dom}-{kname}"
    traffic = measured_traffic(wl_key)
    # LDS: every input of every output row is read once per output sample from LDS by the
    # staged kernels; this is the kernel's own LDS floor, next to the HBM one
    es = {"f32": 4, "bf16": 2, "f16": 2, "u8": 1, "u16": 2, "bits": 0.125}[info["stage_src_dtype"][dom]]
    lds_alg = info["stage_entries"][dom] * plan.n_out * es
    whole_alg = sum(info["stage_alg_bytes"])
    node_es = {"f32": 4, "bf16": 2, "f16": 2, "u8": 1, "u16": 2, "bits": 0.125}[node]
    level_bytes = int(info["n_neurons"] * node_es * 2 * plan.n_out)
    # the type the tree arithmetic runs in: float storage types accumulate in FP32; binary bit
    # rows are evaluated with bitwise logic on 1-bit samples
    dtype_name = {"float": "f32" if node == "f32" else node, "graded": node, "binary": "u1" if node == "bits" else "u8"}[mode]
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DM-time samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": "single NC-shaped beam: 1024 ch 400-416 MHz, 0.138 ms, 2^17 samples, 16 pulses; "
                               "4096 DMs 0-2000; B=4, C=4",
                   "mode": mode, "in_dtype": plan.in_dtype, "node_dtype": node,
                   "n_out": plan.n_out, "stages": nst, "detect": detector is not None,
                   "detect_host_overlapped": pipeline},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{kname} (stage {dom} of {nst}, {info['stage_kernel'][dom]})",
                     "alg_bytes_per_launch": alg, "avg_launch_ms": round(float(stage_ms[dom]), 4)},
        "lds_roofline": {"achieved": lds_alg / (stage_ms[dom] * 1e-3) / 1e9, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                         "frac": lds_alg / (stage_ms[dom] * 1e-3) / 1e9 / LDS_PEAK_GBS,
                         "alg_read_bytes_per_launch": lds_alg},
        "tree_hbm": {"alg_bytes": whole_alg, "ms": round(float(stage_ms.sum()), 4),
                     "achieved": whole_alg / (stage_ms.sum() * 1e-3) / 1e9,
                     "frac": whole_alg / (stage_ms.sum() * 1e-3) / 1e9 / HBM_PEAK_GBS},
        # the level-by-level count (every neuron of every level written once and read once per
        # output sample, in the node storage type), against which a 60 %-of-peak time is quoted;
        # the fused tree keeps levels 1 .. root in registers and moves far fewer bytes
        "level_model": {"bytes": level_bytes, "ms_at_60pct_peak": round(level_bytes / (0.6 * HBM_PEAK_GBS * 1e9) * 1e3, 3),
                        "tree_ms": round(float(stage_ms.sum()), 4),
                        "effective_gbs": level_bytes / (stage_ms.sum() * 1e-3) / 1e9},
        "stage_ms": [round(v, 4) for v in stage_ms],
        "stage_alg_gb": [round(b / 1e9, 3) for b in info["stage_alg_bytes"]],
        "detect_ms": round(det_ms, 4),
        "candidates": ncand,
        "detection": completeness(snd, spec, last, plan.n_out) if last is not None else None,
        "thresholded_cells": detector.npixels if detector is not None else 0,
        "plan": {"neurons": info["n_neurons"], "synapses": info["n_synapses"],
                 "workspace_gib": round(info["workspace_bytes"] / 2**30, 3)},
    }
    if tuned is not None:
        result["autotune"] = dict(cached=hit, candidates=[
            dict(stage_levels=hex(t["stage_levels"]), tune=t["tune"], ms=round(t["ms"], 3),
                 workspace_gib=round(t["workspace_bytes"] / 2**30, 2)) for t in tuned])
    result["config"]["stage_levels"] = hex(stage_levels)
    result["config"]["tune"] = hex(tune)
    if detector is not None:
        # the matched filter's sigma options on the last plane: the standard deviation (the
        # default above) and the median absolute deviation; synchronous runs, host part included
        plane = outs[(args.steps - 1) % 2]
        opt = {}
        for name in ("std", "mad"):
            d2 = snd.Detector(plan, widths=spec.widths, threshold=7.0, device=dev, sigma=name)
            c2 = d2.run(plane)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                c2 = d2.run(plane)
            torch.cuda.synchronize()
            opt[name] = dict(ms=round((time.perf_counter() - t) * 1e3 / 3, 3), candidates=len(c2),
                             detection=completeness(snd, spec, c2, plan.n_out))
            del d2
        result["detect_sigma"] = opt
        # closing and labelling on the host (cells read back) or on the device (candidates only)
        lab = {}
        for where in ("host", "device"):
            d2 = snd.Detector(plan, widths=spec.widths, threshold=7.0, device=dev, label=where)
            c2 = d2.run(plane)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                c2 = d2.run(plane)
            torch.cuda.synchronize()
            lab[where] = dict(ms=round((time.perf_counter() - t) * 1e3 / 3, 3), candidates=len(c2))
            del d2
        result["detect_label"] = lab
    legs = [l for l in args.legs.split(",") if l and l != "none"]
    if "direct" in legs and plan.in_dtype == "bits":
        result["direct"] = {"skipped": "bit input needs the materialised leaf level"}
    elif "direct" in legs:
        log("[bench] direct-dedispersion baseline on the same block")
        ref = outs[(args.steps - 1) % 2]
        result["direct"] = direct_leg(snd, torch, spec, x, pkw, dev, ref)
        result["direct"]["snd_tree_ms"] = round(float(stage_ms.sum()), 3)
        log(f"[bench] direct: {result['direct']['ms']} ms vs tree {result['direct']['snd_tree_ms']} ms")
        if mode == "float":
            result["subband"] = subband_leg(snd, torch, spec, x, pkw, dev, ref)
            result["subband"]["snd_tree_ms"] = round(float(stage_ms.sum()), 3)
            log(f"[bench] sub-band: {result['subband']['ms']} ms")
            result["subband_approx"] = subband_approx_leg(snd, torch, spec, x, dev, ref)
            result["subband_approx"]["snd_tree_ms"] = round(float(stage_ms.sum()), 3)
            log(f"[bench] approximate sub-band: {result['subband_approx']['ms']} ms, "
                f"pulse S/N vs SND {result['subband_approx']['pulse_snr_ratio_vs_snd']}")
    if "fdmt" in legs and mode == "float" and plan.in_dtype == "f32":
        log("[bench] FDMT baseline on the same block")
        torch.cuda.empty_cache()
        result["fdmt"] = fdmt_leg(snd, torch, spec, x, float(stage_ms.sum()))
        log(f"[bench] FDMT: {result['fdmt']['ms']} ms for {result['fdmt']['rows']} rows")
    if "multirate" in legs:
        log("[bench] multi-rate pipeline on the same block")
        del outs, ws, detector
        torch.cuda.empty_cache()
        zt = torch.from_numpy(z).to(dev)
        result["multirate"] = multirate_leg(snd, torch, spec, zt, mode, dev)
        result["multirate"]["single_rate_ms_per_block"] = round(ms_step, 3)
        log(f"[bench] multirate: {result['multirate']['ms_per_block']} ms per block")
        del zt
        outs = ws = detector = None
    if legs:
        del x, outs, ws, detector, plan
        torch.cuda.empty_cache()
    if "trees" in legs:
        log("[bench] trees: every mode and storage, B = 4 and B = 8")
        zt = torch.from_numpy(z).to(dev)
        result["trees"] = trees_leg(snd, torch, spec, zt, dev)
        del zt
        torch.cuda.empty_cache()
    if "completeness" in legs:
        log("[bench] completeness curve: synthetic injections, multi-rate pipeline")
        result["completeness"] = completeness_leg(snd, synth, torch, spec, dev)
        log(f"[bench] completeness: {result['completeness']['total']['overall']}")
    if "frontend" in legs:
        log("[bench] front end on raw power")
        result["frontend"] = frontend_leg(snd, torch, spec, dev)
        log(f"[bench] front end: {result['frontend']['total_ms']} ms per block")
        torch.cuda.empty_cache()
    if "batch" in legs:
        log("[bench] batched leg: 48 beams")
        result["batch"] = batch_leg(snd, synth, torch, dev)
    if "serve" in legs:
        result["serving"] = serve_leg(snd, synth, torch, dev, args.serve_seconds)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample")
        cb, _ = cpu_baseline(spec, mode, args.cpu_sample, args.cpu_sample_all)
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
