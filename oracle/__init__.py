"""CPU oracle for Spiking Neural Dedispersion -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The product library never loads it, and the oracle never
loads the product library.  The arithmetic lives in ``snd_oracle.c`` (plain C, IEEE
double); this module only marshals numpy arrays through ctypes, plus two closed-form
noise statistics written in Python (``cascade`` and ``binary_snr``).

What pins each function to something other than itself (tests/test_oracle_*.py):

* delays        -- textbook dispersion constant values, the ~42,500-sample sweep at DM 3000 for
                   the Northern Cross band, the printed scrunch band edges, monotonicity, DM 0.
* tree_shape    -- the Northern Cross tree 256 / 32 / 4 / 1 (Table S1).
* snd_recursive, snd_points, snd_dedup
                -- float and uncapped graded equal brute force exactly; graded equals
                   min(brute force, cap) (node values are non-negative, so a clipped child
                   clips its parent); branching-factor invariance; DM 0 row = channel sum;
                   spike-count conservation; binary K = 1 and K = full fan-in reduce to
                   brute force; hand-worked binary cases (tests/golden); the cascade law on
                   Bernoulli spikes; the dedup tree equals the per-DM recursion in all modes.
                   snd_points on its own, at sampled cells of ragged trees: float and graded
                   against brute force, binary K = 1 against 1[brute force >= 1], binary
                   quorums against the dedup tree.
* bruteforce    -- DM 0 row = channel sum; conservation of the summed counts.
* encode        -- fire rates against the normal tail probability; samples exactly at a
                   threshold do not fire, the next float above does (x = 1[z > theta]).
* matched_filter -- the printed noise-floor closed forms (0.8 and ~21), Gaussian noise
                   statistics, optimal boxcar width, constant rows; per-row width counts reduce
                   to the plain filter on the leading widths.
* dm_width_counts -- hand-evaluated widths of the DM-scaled set for the Northern Cross band.
* scrunch_factors -- the printed Northern Cross band edges (289 / 578 / 1157 / 2313).
* scrunch        -- identity at S = 1, constant rows, conservation of the summed samples.
* merge_candidates -- hand-built candidate lists.
* sigma_clip_stats, normalize -- a hand-evaluated clipped outlier; no clipping reduces to the
                   plain mean and standard deviation; the normal tail rate after normalising.
* effective_width -- the printed scrunch band edges (the smearing term equals S dt there),
                   DM 0 and zero-width special cases, a 3-4-5 right triangle.
* match_injections -- hand-worked cases (tests/golden/injection_match.json); all-admissible
                   windows match min(candidates, injections); a one-to-one structure reduces to
                   scipy's linear assignment.
* mad_sigma     -- hand-evaluated rows (odd and even lengths, an outlier), the scale against
                   scipy's normal quantile, Gaussian rows (MAD sigma ~ the standard deviation),
                   robustness to a bright burst.
* zero_dm       -- a broadband spike removed exactly, narrow-band and sub-threshold ones kept,
                   the threshold's closed form on a constant block.
* flag_channels -- a hot channel flagged in its window only, a dead (constant) channel, a
                   clean Gaussian block left alone, a hand-evaluated 5-channel window; the
                   window sigmas equal numpy's population std (pairwise sums) to 1e-12.
* fdmt, fdmt_delays -- the recursion equals the direct sum over the channel delays traced down
                   the split rule (two different computations); the zero-delay row is the channel
                   sum; every traced delay stays within the merge count of the f^-2 law; the
                   split of a sub-band's delay adds up; a spike track along traced delays sums
                   to the channel count (no-smear initialisation: no spike is spread).
* candidates    -- hand-built masks (row gaps 9 / 10, diagonal pairs) and scipy's closing and
                   labelling on padded planes.
* fire_probability, cascade, binary_snr -- Table 1 values.

No function is left "parity unpinned".
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BINARY, GRADED, FLOAT = 0, 1, 2
MODES = {"binary": BINARY, "graded": GRADED, "float": FLOAT}
_IN_U8, _IN_F32, _IN_F64 = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, generic x86-64)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("cluster", C.c_int32), ("branching", C.c_int32),
                ("k_leaf", C.c_int32), ("k_int", C.c_int32), ("cap", C.c_int32), ("root_norm", C.c_int32)]


class _Cand(C.Structure):
    _fields_ = [("k", C.c_int32), ("widx", C.c_int32), ("t", C.c_int64), ("snr", C.c_double),
                ("npix", C.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_delays.argtypes = [C.c_int32, P, C.c_double, C.c_double, C.c_int32, P, P]
        lib.orc_tree_shape.argtypes = [C.c_int32, P, C.c_int32, C.c_int32, P, C.c_int32]
        common = [C.POINTER(_Params), C.c_int32, P, C.c_int64, P, C.c_int32, C.c_int32, P]
        lib.orc_snd_points.argtypes = common + [C.c_int64, P, P, P]
        lib.orc_snd_recursive.argtypes = common + [P]
        lib.orc_snd_dedup.argtypes = common + [P, P, C.c_int32]
        lib.orc_bruteforce.argtypes = [C.c_int32, C.c_int32, C.c_int64, P, C.c_int32, C.c_int32, P, P]
        lib.orc_encode.argtypes = [C.c_int64, P, C.c_int32, P, P]
        lib.orc_encode.restype = None
        lib.orc_matched_filter.argtypes = [C.c_int32, C.c_int64, C.c_int64, P, C.c_int32, P, C.c_double,
                                           P, P, P, P]
        lib.orc_matched_filter_rows.argtypes = [C.c_int32, C.c_int64, C.c_int64, P, C.c_int32, P, P, C.c_double,
                                                P, P, P, P]
        lib.orc_zero_dm.argtypes = [C.c_int32, C.c_int64, P, C.c_double]
        lib.orc_zero_dm.restype = C.c_int64
        lib.orc_flag_channels.argtypes = [C.c_int32, C.c_int64, P, C.c_int64, C.c_double, C.c_double, P, P]
        lib.orc_matched_filter_sigma.argtypes = [C.c_int32, C.c_int64, C.c_int64, P, C.c_int32, P, P, P,
                                                 C.c_double, P, P, P, P]
        lib.orc_dm_width_counts.argtypes = [C.c_int32, P, C.c_double, C.c_double, C.c_int32, P, C.c_int32, P,
                                            C.c_int32, C.c_double, P]
        lib.orc_candidates.argtypes = [C.c_int64, C.c_int64, P, P, C.c_double, C.c_int32, C.c_int64,
                                       C.POINTER(_Cand), C.c_int64]
        lib.orc_candidates.restype = C.c_int64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _input(x: np.ndarray):
    x = np.ascontiguousarray(x)
    if x.dtype == np.uint8:
        return x, _IN_U8
    if x.dtype == np.float32:
        return x, _IN_F32
    return np.ascontiguousarray(x, dtype=np.float64), _IN_F64


def delays(freqs, dms, tsamp_s: float, fref: float = 0.0) -> np.ndarray:
    """int32 [ndm][nchan] integer channel delays in samples."""
    lib = _load()
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.empty((d.size, f.size), dtype=np.int32)
    rc = lib.orc_delays(f.size, _ptr(f), tsamp_s, fref, d.size, _ptr(d), _ptr(out))
    if rc:
        raise ValueError("reference frequency below the highest channel frequency")
    return out


def tree_shape(freqs, cluster: int, branching: int) -> list:
    lib = _load()
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    buf = np.zeros(64, dtype=np.int32)
    n = lib.orc_tree_shape(f.size, _ptr(f), cluster, branching, _ptr(buf), 64)
    if n < 0:
        raise ValueError("bad tree parameters")
    return [int(v) for v in buf[:n]]


def _params(mode, cluster, branching, k_leaf, k_int, cap, root_norm):
    return _Params(MODES[mode] if isinstance(mode, str) else int(mode), cluster, branching, k_leaf, k_int, cap,
                   int(root_norm))


def snd_recursive(x, freqs, delay, *, mode="float", cluster=4, branching=2, k_leaf=2, k_int=2, cap=255,
                  root_norm=False) -> np.ndarray:
    """DM-time plane by the per-DM reference recursion (no sharing)."""
    lib = _load()
    xx, xt = _input(x)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    dl = np.ascontiguousarray(delay, dtype=np.int32)
    nout = xx.shape[1] - int(dl.max())
    y = np.empty((dl.shape[0], nout), dtype=np.float64)
    p = _params(mode, cluster, branching, k_leaf, k_int, cap, root_norm)
    rc = lib.orc_snd_recursive(C.byref(p), f.size, _ptr(f), xx.shape[1], _ptr(xx), xt, dl.shape[0], _ptr(dl), _ptr(y))
    if rc:
        raise ValueError("oracle recursion rejected its arguments")
    return y


def snd_points(x, freqs, delay, ks, ts, *, mode="float", cluster=4, branching=2, k_leaf=2, k_int=2, cap=255,
               root_norm=False) -> np.ndarray:
    """Selected outputs y[k_i, t_i] by the reference recursion."""
    lib = _load()
    xx, xt = _input(x)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    dl = np.ascontiguousarray(delay, dtype=np.int32)
    k = np.ascontiguousarray(ks, dtype=np.int32)
    t = np.ascontiguousarray(ts, dtype=np.int64)
    out = np.empty(k.size, dtype=np.float64)
    p = _params(mode, cluster, branching, k_leaf, k_int, cap, root_norm)
    rc = lib.orc_snd_points(C.byref(p), f.size, _ptr(f), xx.shape[1], _ptr(xx), xt, dl.shape[0], _ptr(dl), k.size,
                            _ptr(k), _ptr(t), _ptr(out))
    if rc:
        raise ValueError("oracle point query out of range")
    return out


def snd_dedup(x, freqs, delay, *, mode="float", cluster=4, branching=2, k_leaf=2, k_int=2, cap=255,
              root_norm=False):
    """(plane, counts) by the shared-pattern tree; counts[l] = (neurons, synapses) at level l."""
    lib = _load()
    xx, xt = _input(x)
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    dl = np.ascontiguousarray(delay, dtype=np.int32)
    nout = xx.shape[1] - int(dl.max())
    y = np.empty((dl.shape[0], nout), dtype=np.float64)
    counts = np.zeros(128, dtype=np.int64)
    p = _params(mode, cluster, branching, k_leaf, k_int, cap, root_norm)
    nl = lib.orc_snd_dedup(C.byref(p), f.size, _ptr(f), xx.shape[1], _ptr(xx), xt, dl.shape[0], _ptr(dl), _ptr(y),
                           _ptr(counts), 64)
    if nl < 0:
        raise ValueError("oracle dedup rejected its arguments")
    return y, [(int(counts[2 * i]), int(counts[2 * i + 1])) for i in range(nl)]


def bruteforce(x, delay, *, mode="float") -> np.ndarray:
    lib = _load()
    xx, xt = _input(x)
    dl = np.ascontiguousarray(delay, dtype=np.int32)
    nout = xx.shape[1] - int(dl.max())
    y = np.empty((dl.shape[0], nout), dtype=np.float64)
    rc = lib.orc_bruteforce(MODES[mode], xx.shape[0], xx.shape[1], _ptr(xx), xt, dl.shape[0], _ptr(dl), _ptr(y))
    if rc:
        raise ValueError("no valid output samples")
    return y


def subband_approx(x, freqs, dms, tsamp_s: float, nsub: int, coarse_step: int) -> np.ndarray:
    """Approximate (coarse-DM) sub-band dedispersion, written out in FP64 (Methods, "Classical
    dedispersion algorithms": the hierarchical baselines).  Sub-bands are runs of nchan / nsub
    channels in the given order; the coarse grid is every coarse_step-th of the sorted distinct
    DMs; fine DM d_k takes the largest coarse DM D_j <= d_k.  With delta the integer delays
    relative to the top frequency (delays()) and c_s the top channel of sub-band s:
        y_k(t) = sum_s sum_{c in s} x_c(t + delta_c(D_j) + delta_{c_s}(d_k) - delta_{c_s}(D_j)),
    for t below the smallest number of samples every term has.  Returns float64 [ndm][n_out].
    Plain loops over DMs and channels: for small cases."""
    x = np.asarray(x, dtype=np.float64)
    f = np.asarray(freqs, dtype=np.float64)
    d = np.asarray(dms, dtype=np.float64)
    nchan, nsamp = x.shape
    m = nchan // nsub
    coarse = np.unique(d)[::coarse_step]
    j = np.searchsorted(coarse, d, side="right") - 1
    dF, dC = delays(f, d, tsamp_s), delays(f, coarse, tsamp_s)
    tops = [s * m + int(np.argmax(f[s * m:(s + 1) * m])) for s in range(nsub)]
    shift = np.empty((d.size, nchan), dtype=np.int64)  # total read offset of each (DM, channel)
    for s in range(nsub):
        extra = dF[:, tops[s]].astype(np.int64) - dC[j, tops[s]]
        for c in range(s * m, (s + 1) * m):
            shift[:, c] = dC[j, c] + extra
    n_out = nsamp - int(shift.max())
    y = np.zeros((d.size, n_out))
    for k in range(d.size):
        for c in range(nchan):
            y[k] += x[c, shift[k, c]:shift[k, c] + n_out]
    return y


def encode(z: np.ndarray, thresholds) -> np.ndarray:
    """uint8 level = number of thresholds exceeded (z > theta), compared in float32."""
    lib = _load()
    zz = np.ascontiguousarray(z, dtype=np.float32)
    th = np.ascontiguousarray(thresholds, dtype=np.float32)
    out = np.empty(zz.shape, dtype=np.uint8)
    lib.orc_encode(zz.size, _ptr(zz), th.size, _ptr(th), _ptr(out))
    return out


def dm_width_counts(freqs, dms, tsamp_s: float, widths, n_base: int, alpha: float, fref: float = 0.0) -> np.ndarray:
    """int32 [ndm]: how many of the increasing widths each DM row uses under the DM-scaled width
    set (base = the first n_base widths, the rest up to alpha * sweep / dt)."""
    lib = _load()
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float64)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    out = np.empty(d.size, dtype=np.int32)
    rc = lib.orc_dm_width_counts(f.size, _ptr(f), tsamp_s, fref, d.size, _ptr(d), w.size, _ptr(w), int(n_base),
                                 float(alpha), _ptr(out))
    if rc:
        raise ValueError("reference frequency below the highest channel frequency")
    return out


def matched_filter(y, widths, *, integer_plane: bool, sigma_min: float = 0.0, row_nw=None, sigma_rows=None):
    """(snr, width_index, mu, sigma) for a DM-time plane y[ndm][nout]; row_nw: per-row number of
    leading widths used (None: all); sigma_rows: per-row sigma to use instead of the standard
    deviation (e.g. mad_sigma), floored by sigma_min like it."""
    lib = _load()
    yy = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    snr = np.empty(yy.shape, dtype=np.float64)
    widx = np.empty(yy.shape, dtype=np.int32)
    mu = np.empty(yy.shape[0], dtype=np.float64)
    sg = np.empty(yy.shape[0], dtype=np.float64)
    rn = None if row_nw is None else np.ascontiguousarray(row_nw, dtype=np.int32)
    si = None if sigma_rows is None else np.ascontiguousarray(sigma_rows, dtype=np.float64)
    rc = lib.orc_matched_filter_sigma(int(integer_plane), yy.shape[0], yy.shape[1], _ptr(yy), w.size, _ptr(w),
                                      None if rn is None else _ptr(rn), None if si is None else _ptr(si), sigma_min,
                                      _ptr(snr), _ptr(widx), _ptr(mu), _ptr(sg))
    if rc:
        raise ValueError("widths must be positive and strictly increasing")
    return snr, widx, mu, sg


# 1 / Phi^-1(3/4): scales a median absolute deviation to the standard deviation of Gaussian
# noise (the correctly rounded double of 1.48260221850560186...)
MAD_SCALE = 1.4826022185056018


def mad_sigma(y) -> np.ndarray:
    """float64 [ndm]: per-row robust sigma, MAD_SCALE times the median absolute deviation (the
    per-row MAD the paper names for graded planes, Methods "Tree activation modes", as an
    alternative sigma for the matched filter).  Both medians are lower medians (element
    floor((n - 1) / 2) of the sorted row); the deviation |y - m| is taken in the plane's own
    type (integers exactly; float32 planes in float32 arithmetic)."""
    y = np.asarray(y)
    out = np.empty(y.shape[0], dtype=np.float64)
    for k in range(y.shape[0]):
        row = y[k].astype(np.int64) if np.issubdtype(y.dtype, np.integer) else y[k]
        r = (row.size - 1) // 2
        m = np.sort(row)[r]
        d = np.abs(row - m)  # int64 or float32 arithmetic, as the row's type
        out[k] = MAD_SCALE * float(np.sort(d)[r])
    return out


def candidates(snr, widx, theta: float, radius: int = 4, n_min: int = 10):
    """List of dicts {k, t, widx, snr, npix}, ordered by (k, t) of the peak pixel."""
    lib = _load()
    s = np.ascontiguousarray(snr, dtype=np.float64)
    w = np.ascontiguousarray(widx, dtype=np.int32)
    cap = 1 << 16
    buf = (_Cand * cap)()
    n = lib.orc_candidates(s.shape[0], s.shape[1], _ptr(s), _ptr(w), theta, radius, n_min, buf, cap)
    if n < 0:
        raise ValueError("candidate extraction failed")
    return [dict(k=buf[i].k, t=buf[i].t, widx=buf[i].widx, snr=buf[i].snr, npix=buf[i].npix)
            for i in range(min(n, cap))]


# --------------------------------------------------------------------------------------
# Closed forms from the paper's noise analysis (Results, "Spike encoding statistics and
# cascade noise analysis").
# --------------------------------------------------------------------------------------
def fire_probability(theta: float) -> float:
    """Per-sample fire probability of the delta encoder on N(0,1) input: erfc(theta/sqrt 2)/2."""
    return 0.5 * math.erfc(theta / math.sqrt(2.0))


def _binom_tail(n: int, p: float, k: int) -> float:
    """P(Bin(n, p) >= k)."""
    if k <= 0:
        return 1.0
    return sum(math.comb(n, i) * p ** i * (1.0 - p) ** (n - i) for i in range(k, n + 1))


def cascade(p0: float, fanins, k_leaf: int, k_int: int) -> list:
    """Noise fire rate per level (Eq. cascade): p1 = P(Bin(C, p0) >= K_L),
    p_{l+1} = P(Bin(B_l, p_l) >= K_I).  fanins = [C, B_1, ..., B_root]."""
    rates = [_binom_tail(fanins[0], p0, k_leaf)]
    for b in fanins[1:]:
        rates.append(_binom_tail(b, rates[-1], k_int))
    return rates


def binary_snr(width: float, p_sig: float, p_noise: float) -> float:
    """Predicted boxcar S/N of a Bernoulli root output (Eq. snr_A)."""
    return math.sqrt(width) * (p_sig - p_noise) / math.sqrt(p_noise * (1.0 - p_noise))


# --------------------------------------------------------------------------------------
# Multi-rate extension (Methods, "Multi-rate extension").
# --------------------------------------------------------------------------------------
K_DM = 4.148808e6  # MHz^2 ms per pc cm^-3 (as in the C part)


def scrunch_factors(freqs, dms, tsamp_s: float, s_max: int = 16) -> np.ndarray:
    """int32 [ndm]: the scrunch factor of each trial DM (Eq. scrunch): the largest power of two
    S <= s_max with S * dt <= tau_smear(d) = K_DM d df / fc^3 (1 when even S = 2 fails).  fc is
    the band centre (mean of the highest and lowest channel frequencies) and df the channel
    spacing; tau_smear and dt in ms, FP64."""
    f = np.asarray(freqs, dtype=np.float64)
    d = np.asarray(dms, dtype=np.float64)
    fc = 0.5 * (f.max() + f.min())
    df = (f.max() - f.min()) / (f.size - 1) if f.size > 1 else 0.0
    dt = tsamp_s * 1e3
    out = np.ones(d.size, dtype=np.int32)
    for i, dm in enumerate(d):
        tau = K_DM * dm * df / (fc * fc * fc)
        s = 1
        while 2 * s <= s_max and 2 * s * dt <= tau:
            s *= 2
        out[i] = s
    return out


def scrunch(z, s: int) -> np.ndarray:
    """float32 [nchan][n // s]: each output sample sums s consecutive input samples, in order, in
    FP32, and scales by the FP32 value of 1/sqrt(s), so that unit-variance input stays unit
    variance.  FP32 on purpose: the spike encoder thresholds the result, and both sides must
    take that decision on the same values."""
    z = np.asarray(z, dtype=np.float32)
    n = z.shape[1] // s
    acc = z[:, 0:n * s:s].copy()
    for j in range(1, s):
        acc = (acc + z[:, j:n * s:s]).astype(np.float32)
    return (acc * np.float32(1.0 / math.sqrt(s))).astype(np.float32)


def merge_candidates(cands, dm_tol: float = 20.0, t_tol_ms: float = 200.0) -> list:
    """Cross-band merge of candidates (dicts with dm, t_ms, snr): in decreasing S/N (ties: lower
    DM, then earlier time) a candidate within |dDM| <= dm_tol and |dt| <= t_tol_ms of an already
    kept candidate is absorbed by it, otherwise it is kept.  Returns the kept ones ordered by
    (t_ms, dm)."""
    order = sorted(range(len(cands)), key=lambda i: (-cands[i]["snr"], cands[i]["dm"], cands[i]["t_ms"]))
    kept = []
    for i in order:
        c = cands[i]
        if any(abs(c["dm"] - q["dm"]) <= dm_tol and abs(c["t_ms"] - q["t_ms"]) <= t_tol_ms for q in kept):
            continue
        kept.append(c)
    return sorted(kept, key=lambda c: (c["t_ms"], c["dm"]))


# --------------------------------------------------------------------------------------
# Front end (Methods, "Input encoding"): two-pass sigma-clip normalisation of raw power.
# --------------------------------------------------------------------------------------
def sigma_clip_stats(p, clip: float = 5.0) -> np.ndarray:
    """float64 [nchan][2] (mu, sigma) per channel: mean and population standard deviation of
    the raw power, then of the power clipped to [mu0 - clip sigma0, mu0 + clip sigma0] (each
    value outside moved to the nearer bound), in FP64."""
    x = np.asarray(p, dtype=np.float64)
    out = np.empty((x.shape[0], 2), dtype=np.float64)
    for c in range(x.shape[0]):
        row = x[c]
        mu0 = row.mean()
        s0 = math.sqrt(((row - mu0) ** 2).mean())
        clipped = np.minimum(np.maximum(row, mu0 - clip * s0), mu0 + clip * s0)
        mu = clipped.mean()
        out[c, 0] = mu
        out[c, 1] = math.sqrt(((clipped - mu) ** 2).mean())
    return out


def normalize(p, stats) -> np.ndarray:
    """float32 z = (P - mu) / sigma per channel, the quotient taken in FP64 and rounded once
    (the encoder then compares it with its thresholds in FP32, as the library does)."""
    x = np.asarray(p, dtype=np.float64)
    st = np.asarray(stats, dtype=np.float64)
    return ((x - st[:, 0:1]) / st[:, 1:2]).astype(np.float32)


# --------------------------------------------------------------------------------------
# Validation against injected pulses (Methods, "Validation methodology").
# --------------------------------------------------------------------------------------
def effective_width(freqs, tsamp_s: float, dms, w_int_ms) -> np.ndarray:
    """float64 [n]: effective width in ms of pulses of intrinsic width w_int_ms at DM dms.
    The paper names the width at the injection DM without a formula; read here as the
    intrinsic width, the smearing inside one channel (Eq. scrunch: K_DM d df / fc^3 with fc the
    band centre and df the channel spacing) and the sampling time added in quadrature."""
    f = np.asarray(freqs, dtype=np.float64)
    fc = 0.5 * (f.max() + f.min())
    df = (f.max() - f.min()) / (f.size - 1) if f.size > 1 else 0.0
    dt = tsamp_s * 1e3
    out = []
    for d, w in zip(np.asarray(dms, dtype=np.float64).ravel(), np.asarray(w_int_ms, dtype=np.float64).ravel()):
        tau = K_DM * d * df / fc ** 3
        out.append(math.sqrt(w * w + tau * tau + dt * dt))
    return np.array(out, dtype=np.float64)


def match_injections(cands, injections, dm_tol: float = 10.0, t_frac: float = 0.5):
    """Greedy one-to-one matching (Methods, "Validation methodology").  cands: dicts with dm,
    t_ms, snr; injections: dicts with dm, t_ms, w_eff_ms.  Candidates go in decreasing S/N
    (equal S/N: list order); each takes, among the injections not yet matched whose DM is
    within dm_tol and whose time is within t_frac * w_eff_ms, the one nearest in time (then
    nearest in DM, then first in the list).  Returns (list: matched candidate index per
    injection or -1, number of injections matched); completeness is the number over the
    injection count."""
    order = sorted(range(len(cands)), key=lambda i: -cands[i]["snr"])  # sorted() is stable
    match = [-1] * len(injections)
    for i in order:
        c = cands[i]
        best = None
        for j, q in enumerate(injections):
            if match[j] >= 0:
                continue
            ddm = abs(c["dm"] - q["dm"])
            dt = abs(c["t_ms"] - q["t_ms"])
            if ddm > dm_tol or dt > t_frac * q["w_eff_ms"]:
                continue
            key = (dt, ddm, j)
            if best is None or key < best:
                best = key
        if best is not None:
            match[best[2]] = i
    return match, sum(1 for m in match if m >= 0)


def zero_dm(z, gamma: float = 5.0):
    """(filtered copy, samples changed): zero-DM subtraction of a z-scored float32 filterbank
    [nchan][n] where the zero-DM S/N exceeds gamma (orc_zero_dm)."""
    lib = _load()
    x = np.array(z, dtype=np.float32, order="C", copy=True)
    n = lib.orc_zero_dm(x.shape[0], x.shape[1], _ptr(x), float(gamma))
    return x, int(n)


def flag_channels(z, window: int, k: float = 5.0, return_sigma: bool = False):
    """(flagged copy, uint8 flags [nwin][nchan][, float64 sigmas [nwin][nchan]]): windowed MAD
    channel flagging of a z-scored float32 filterbank (orc_flag_channels), scale MAD_SCALE."""
    lib = _load()
    x = np.array(z, dtype=np.float32, order="C", copy=True)
    nwin = (x.shape[1] + window - 1) // window
    flags = np.zeros((nwin, x.shape[0]), dtype=np.uint8)
    sig = np.zeros((nwin, x.shape[0]), dtype=np.float64)
    if lib.orc_flag_channels(x.shape[0], x.shape[1], _ptr(x), int(window), float(k), MAD_SCALE, _ptr(flags),
                             _ptr(sig)):
        raise MemoryError("oracle channel flagging")
    return (x, flags, sig) if return_sigma else (x, flags)


# --------------------------------------------------------------------------------------
# FDMT with the no-smear initialisation (Methods, "Classical dedispersion algorithms").
# --------------------------------------------------------------------------------------
def _fdmt_geometry(freqs, chan_bw_mhz: float, tsamp_s: float, dm_max: float):
    """(span(c0, c1), D, ndel(c0, c1)) for channels given as intervals of width chan_bw_mhz
    around descending centres: span is the f^-2 sweep span of channels [c0, c1) (lower edge of
    the last, upper edge of the first), D the band sweep at dm_max in samples rounded up, ndel
    the number of delays a sub-band holds."""
    f = np.asarray(freqs, dtype=np.float64)
    hi = f + 0.5 * chan_bw_mhz
    lo = f - 0.5 * chan_bw_mhz

    def span(c0, c1):
        return 1.0 / (lo[c1 - 1] * lo[c1 - 1]) - 1.0 / (hi[c0] * hi[c0])

    r_band = span(0, f.size)
    D = int(math.ceil(K_DM * dm_max * r_band / (tsamp_s * 1e3)))

    def ndel(c0, c1):
        return min(int(math.ceil(D * span(c0, c1) / r_band)) + 1, D + 1)

    return span, D, ndel


def _fdmt_split(span, ndel, c0, w, d):
    """Delay d of sub-band [c0, c0 + 2w) split over its upper half [c0, c0 + w) and lower half
    [c0 + w, c0 + 2w), in proportion to their f^-2 spans (rounded half to even), each clamped
    to the delays its half holds."""
    du = min(int(np.rint(d * span(c0, c0 + w) / span(c0, c0 + 2 * w))), ndel(c0, c0 + w) - 1)
    dl = min(d - du, ndel(c0 + w, c0 + 2 * w) - 1)
    return du, dl


def fdmt(x, freqs, chan_bw_mhz: float, tsamp_s: float, dm_max: float) -> np.ndarray:
    """float64 [D + 1][n]: FDMT of x [nchan][n] (nchan a power of two) with the no-smear
    initialisation: every initial delay row of a channel is the channel; merging adjacent
    sub-bands, row d of a sub-band is row du of its upper half plus row dl of its lower half
    read du samples later (zero past n), the time reference being each sub-band's upper edge.
    Output row d is the band sweep of d samples."""
    x = np.asarray(x, dtype=np.float64)
    nchan, n = x.shape
    span, D, ndel = _fdmt_geometry(freqs, chan_bw_mhz, tsamp_s, dm_max)
    if D >= n:
        raise ValueError("the band sweep at dm_max does not fit the block")
    # sub-bands of the current width: arrays [ndel][n]
    bands = [np.repeat(x[c][None, :], ndel(c, c + 1), axis=0) for c in range(nchan)]
    w = 1
    while w < nchan:
        merged = []
        for s in range(nchan // (2 * w)):
            c0 = 2 * w * s
            up, low = bands[2 * s], bands[2 * s + 1]
            rows = np.zeros((ndel(c0, c0 + 2 * w), n))
            for d in range(rows.shape[0]):
                du, dl = _fdmt_split(span, ndel, c0, w, d)
                rows[d] = up[du]
                rows[d, : n - du] += low[dl, du:]
            merged.append(rows)
        bands = merged
        w *= 2
    return bands[0]


def fdmt_delays(freqs, chan_bw_mhz: float, tsamp_s: float, dm_max: float, d: int) -> np.ndarray:
    """int64 [nchan]: the sample delay at which FDMT's output row d reads each channel, found by
    following the split rule from the whole band down to single channels (a channel of the
    lower half is read later by the upper half's share of the delay)."""
    f = np.asarray(freqs, dtype=np.float64)
    span, D, ndel = _fdmt_geometry(f, chan_bw_mhz, tsamp_s, dm_max)
    out = np.zeros(f.size, dtype=np.int64)

    def walk(c0, width, dd, base):
        if width == 1:
            out[c0] = base
            return
        w = width // 2
        du, dl = _fdmt_split(span, ndel, c0, w, dd)
        walk(c0, w, du, base)
        walk(c0 + w, w, dl, base + du)

    walk(0, f.size, d, 0)
    return out


def fdmt_row(x, delays) -> np.ndarray:
    """float64 [n]: sum over channels of x_c(t + delays[c]), zero past n (one FDMT output row
    evaluated directly)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    y = np.zeros(n)
    for c, e in enumerate(np.asarray(delays, dtype=np.int64)):
        y[: n - e] += x[c, e:]
    return y

