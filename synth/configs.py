"""The five benchmark workloads as seeded, synthetic stand-ins for the paper's Northern Cross data.

Instrument shape follows the paper's Northern Cross parameters (Supplementary Table S1:
1024 channels, 408 MHz centre, 16 MHz bandwidth, 0.138 ms sampling).  Every array is
drawn from ``numpy.random.Generator(PCG64(seed))`` with seed ``20260000 + 100 * config + beam``.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .filterbank import (KDM_MS, Pulse, channel_freqs, dm_geometric, dm_linear, inject_pulses, make_rng,
                         noise_filterbank, random_pulses)

TSAMP_S = 0.138e-3


def seed_for(config: int, beam: int = 0) -> int:
    return 20260000 + 100 * config + beam


def sweep_samples(freqs: np.ndarray, dm: float, tsamp_s: float) -> float:
    """Unrounded dispersive sweep across the band in samples (signal model)."""
    return KDM_MS * dm * (float(np.min(freqs)) ** -2 - float(np.max(freqs)) ** -2) / (tsamp_s * 1e3)


@dataclasses.dataclass
class WorkloadSpec:
    name: str
    config: int
    nchan: int
    nsamp: int
    dms: np.ndarray
    branching: int
    cluster: int = 4
    mode: str = "float"            # "binary" | "graded" | "float"
    k_leaf: int = 2
    k_int: int = 2
    cap: int = 255
    enc_thresholds: tuple = ()     # encoder thresholds in sigma (binary: one, graded: several)
    widths: tuple = (1, 2, 4, 8, 16, 32, 64)
    tsamp_s: float = TSAMP_S
    beam: int = 0
    node_dtype: str = "f32"        # tree storage: f32 | bf16 | f16 (float), u8 (graded), bits (binary)
    pulses: list = dataclasses.field(default_factory=list)

    @property
    def freqs(self) -> np.ndarray:
        return channel_freqs(self.nchan)

    @property
    def seed(self) -> int:
        return seed_for(self.config, self.beam)

    def filterbank(self, nsamp: int | None = None) -> np.ndarray:
        """float32 z-scored filterbank [nchan][nsamp] with this workload's pulses injected."""
        n = self.nsamp if nsamp is None else nsamp
        rng = make_rng(self.seed)
        z = noise_filterbank(rng, self.nchan, n)
        inject_pulses(z, self.freqs, self.tsamp_s, [p for p in self.pulses if p.t0 < n])
        return z


def _config1(nsamp: int = 8192) -> WorkloadSpec:
    spec = WorkloadSpec(name="single_beam_binary_64ch", config=1, nchan=64, nsamp=nsamp,
                        dms=dm_linear(64, 0.0, 300.0), branching=2, cluster=4, mode="binary",
                        k_leaf=2, k_int=2, enc_thresholds=(2.0,))
    spec.pulses = [Pulse(dm=150.0, t0=2048.0, width_ms=1.0, snr=20.0, alpha=0.0)]
    return spec


def _config2(nsamp: int = 1 << 17, ndm: int = 4096) -> WorkloadSpec:
    spec = WorkloadSpec(name="nc_float_1024ch_4096dm", config=2, nchan=1024, nsamp=nsamp,
                        dms=dm_linear(ndm, 0.0, 2000.0), branching=4, cluster=4, mode="float",
                        enc_thresholds=())
    rng = make_rng(seed_for(2, 999))
    sweep = sweep_samples(spec.freqs, 2000.0, spec.tsamp_s)
    hi = max(1.0, nsamp - sweep - 200.0)
    spec.pulses = random_pulses(rng, 16, (50.0, 2000.0), (0.3, 10.0), (6.0, 50.0), (-2.0, 2.0), 100.0, hi)
    return spec


def _config3(nsamp: int = 65536, mode: str = "graded", branching: int = 4) -> WorkloadSpec:
    thr = {"binary": (2.0,), "graded": (1.0, 2.0, 3.0, 4.0), "float": ()}[mode]
    spec = WorkloadSpec(name=f"modes_64ch_geometric_{mode}_b{branching}", config=3, nchan=64, nsamp=nsamp,
                        dms=dm_geometric(3000, 2000.0), branching=branching, cluster=4, mode=mode,
                        k_leaf=2, k_int=1, enc_thresholds=thr)
    spec.pulses = [Pulse(dm=150.0, t0=2048.0, width_ms=1.0, snr=20.0, alpha=0.0)]
    return spec


def batch_beam(beam: int, nsamp: int = 65536, nchan: int = 1024) -> WorkloadSpec:
    """One beam of the 48-beam batched workload: uneven DM grids, rotating modes and float storage;
    binary beams carry bit rows (one bit per spike, input and tree), graded beams u8."""
    ndm = 1024 + (3072 * beam) // 47
    dmax = 500.0 + 1500.0 * ((29 * beam) % 48) / 47.0
    mode = ("binary", "graded", "float")[beam % 3]
    node = ("f32", "bf16", "f16")[(beam // 3) % 3] if mode == "float" else ("bits" if mode == "binary" else "u8")
    thr = {"binary": (2.0,), "graded": (1.0, 2.0, 3.0, 4.0), "float": ()}[mode]
    spec = WorkloadSpec(name=f"batch_beam{beam}", config=4, nchan=nchan, nsamp=nsamp,
                        dms=dm_linear(ndm, 0.0, dmax), branching=4, cluster=4, mode=mode,
                        k_leaf=2, k_int=1, enc_thresholds=thr, beam=beam, node_dtype=node)
    rng = make_rng(seed_for(4, 500 + beam))
    sweep = sweep_samples(spec.freqs, dmax, spec.tsamp_s)
    hi = max(101.0, nsamp - sweep - 200.0)
    spec.pulses = random_pulses(rng, 4, (50.0, 0.95 * dmax), (0.3, 10.0), (6.0, 50.0), (-2.0, 2.0), 100.0, hi)
    return spec


def stream_beam(beam: int, chunk: int = 8192, nchan: int = 1024, ndm: int = 4096) -> WorkloadSpec:
    """One beam of the streaming workload: half graded (4-level), half BF16-stored float."""
    mode = "graded" if beam % 2 == 0 else "float"
    thr = (1.0, 2.0, 3.0, 4.0) if mode == "graded" else ()
    return WorkloadSpec(name=f"stream_beam{beam}", config=5, nchan=nchan, nsamp=chunk,
                        dms=dm_linear(ndm, 0.0, 2000.0), branching=4, cluster=4, mode=mode,
                        enc_thresholds=thr, beam=beam, node_dtype="u8" if mode == "graded" else "bf16")


WORKLOADS = {
    1: _config1,
    2: _config2,
    3: _config3,
}


def workload(config: int, **kw) -> WorkloadSpec:
    return WORKLOADS[config](**kw)


def chunk_period_s(chunk: int = 8192, tsamp_s: float = TSAMP_S) -> float:
    return chunk * tsamp_s


def arrival_times(rng: np.random.Generator, nbeams: int, duration_s: float, period_s: float):
    """Per-beam chunk arrival times: random phase, inter-arrival = period * U(0.8, 1.2)."""
    out = []
    for _ in range(nbeams):
        t = rng.uniform(0.0, period_s)
        ts = []
        while t < duration_s:
            ts.append(t)
            t += period_s * rng.uniform(0.8, 1.2)
        out.append(np.array(ts))
    return out

