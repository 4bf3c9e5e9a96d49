"""Seeded noise filterbanks with injected dispersed Gaussian pulses.

Signal model (stand-in for the paper's Northern Cross data, which is not available):
* channel centres of a band of width ``bw`` below ``f_hi``, highest frequency first;
* i.i.d. N(0, 1) noise per channel sample, i.e. an already z-scored filterbank;
* a pulse arrives at the top of the band at sample ``t0`` and at channel frequency f
  ``KDM * DM * (f**-2 - f_top**-2)`` milliseconds later (cold-plasma sweep), with a
  Gaussian profile of the given FWHM, a power-law spectrum ``(f / 408 MHz)**alpha``
  normalised to unit mean square, and an amplitude chosen so that the optimal
  matched-filter S/N ``sqrt(sum_c sum_t s_c(t)**2)`` equals the requested value;
* no scattering and no intra-channel smearing.

The sweep here uses unrounded delays: it describes the sky, not the dedisperser.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf

#: Dispersion constant in MHz^2 ms per (pc cm^-3) used by the signal model.
KDM_MS = 4.148808e6


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def channel_freqs(nchan: int, f_hi: float = 416.0, bw: float = 16.0) -> np.ndarray:
    """Channel centre frequencies in MHz, highest first: f_c = f_hi - (c + 1/2) bw / nchan."""
    c = np.arange(nchan, dtype=np.float64)
    return f_hi - (c + 0.5) * bw / nchan


def dm_linear(n: int, lo: float, hi: float) -> np.ndarray:
    return np.linspace(lo, hi, n, dtype=np.float64)


def dm_geometric(n: int = 3000, top: float = 2000.0, knee: float = 100.0) -> np.ndarray:
    """Grid whose step grows in proportion to (DM + knee): d_k = knee * (r**(k/(n-1)) - 1), d_{n-1} = top."""
    k = np.arange(n, dtype=np.float64)
    r = (top + knee) / knee
    return knee * (r ** (k / (n - 1)) - 1.0)


@dataclasses.dataclass
class Pulse:
    dm: float          # pc cm^-3
    t0: float          # arrival sample at the top of the band (continuous)
    width_ms: float    # Gaussian FWHM in ms
    snr: float         # optimal matched-filter S/N of the injected signal
    alpha: float = 0.0  # spectral index


def noise_filterbank(rng: np.random.Generator, nchan: int, nsamp: int) -> np.ndarray:
    """float32 [nchan][nsamp] of i.i.d. N(0, 1)."""
    return rng.standard_normal((nchan, nsamp), dtype=np.float32)


def _profile(t_centre: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    """Gaussian integrated over each sample [t, t+1) for t in [lo, hi)."""
    edges = np.arange(lo, hi + 1, dtype=np.float64)
    cdf = 0.5 * (1.0 + erf((edges - t_centre) / (sigma * math.sqrt(2.0))))
    return np.diff(cdf)


def inject_pulses(z: np.ndarray, freqs: np.ndarray, tsamp_s: float, pulses, f_top: float | None = None) -> None:
    """Add each pulse to the float32 filterbank ``z`` in place (see the module docstring)."""
    nchan, nsamp = z.shape
    tms = tsamp_s * 1e3
    ftop = float(np.max(freqs)) if f_top is None else f_top
    for p in pulses:
        sig = p.width_ms / (2.0 * math.sqrt(2.0 * math.log(2.0))) / tms
        sig = max(sig, 1e-3)
        half = int(math.ceil(6.0 * sig)) + 2
        a = (freqs / 408.0) ** p.alpha
        a = a / math.sqrt(np.mean(a * a))
        centres = p.t0 + KDM_MS * p.dm * (freqs ** -2 - ftop ** -2) / tms
        prof = []
        energy = 0.0
        for c in range(nchan):
            lo = max(0, int(math.floor(centres[c])) - half)
            hi = min(nsamp, int(math.floor(centres[c])) + half + 1)
            if hi <= lo:
                prof.append((lo, hi, None))
                continue
            g = a[c] * _profile(centres[c], sig, lo, hi)
            energy += float(np.dot(g, g))
            prof.append((lo, hi, g))
        if energy <= 0.0:
            continue
        amp = p.snr / math.sqrt(energy)
        for c, (lo, hi, g) in enumerate(prof):
            if g is not None:
                z[c, lo:hi] += (amp * g).astype(np.float32)


def random_pulse_slots(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """n arrival times in evenly spaced slots of [lo, hi) with +-1/4 slot jitter."""
    slot = (hi - lo) / n
    centres = lo + (np.arange(n) + 0.5) * slot
    return centres + rng.uniform(-0.25, 0.25, size=n) * slot


def random_pulses(rng: np.random.Generator, n: int, dm_range, width_range_ms, snr_range, alpha_range,
                  t_lo: float, t_hi: float):
    """Pulses with DM ~ U, width ~ log-U, S/N ~ U, spectral index ~ U, arrivals in jittered slots."""
    t0 = random_pulse_slots(rng, n, t_lo, t_hi)
    dms = rng.uniform(dm_range[0], dm_range[1], size=n)
    widths = np.exp(rng.uniform(math.log(width_range_ms[0]), math.log(width_range_ms[1]), size=n))
    snrs = rng.uniform(snr_range[0], snr_range[1], size=n)
    alphas = rng.uniform(alpha_range[0], alpha_range[1], size=n)
    return [Pulse(float(d), float(t), float(w), float(s), float(a))
            for d, t, w, s, a in zip(dms, t0, widths, snrs, alphas)]


def random_spikes(rng: np.random.Generator, nchan: int, nsamp: int, p: float) -> np.ndarray:
    """uint8 [nchan][nsamp] of i.i.d. Bernoulli(p) spikes (0/1)."""
    return (rng.random((nchan, nsamp), dtype=np.float32) < p).astype(np.uint8)


def random_levels(rng: np.random.Generator, nchan: int, nsamp: int, hi: int) -> np.ndarray:
    """uint8 [nchan][nsamp] of integer levels uniform on 0..hi."""
    return rng.integers(0, hi + 1, size=(nchan, nsamp), dtype=np.uint8)
