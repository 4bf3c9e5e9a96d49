"""Validation against injected pulses (Methods, "Validation methodology"): effective widths
and the greedy one-to-one matching of candidates to injections.  Argument marshalling only;
both run in libsnd (host code)."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def effective_width(freqs, tsamp_s: float, dms, w_int_ms) -> np.ndarray:
    """float64 [n] effective widths in ms (snd_effective_width)."""
    f, d, w = _f64(freqs), _f64(dms).ravel(), _f64(w_int_ms).ravel()
    if d.size != w.size:
        raise ValueError("dms and w_int_ms must have the same length")
    out = np.empty(d.size, dtype=np.float64)
    P = C.c_void_p
    capi.check(capi.lib().snd_effective_width(f.size, f.ctypes.data_as(P), float(tsamp_s), d.size, d.ctypes.data_as(P),
                                              w.ctypes.data_as(P), out.ctypes.data_as(P)))
    return out


def match_injections(cand_dm, cand_t_ms, cand_snr, inj_dm, inj_t_ms, inj_weff_ms, dm_tol: float = 10.0,
                     t_frac: float = 0.5):
    """(int32 [n_inj] matched candidate index or -1, number matched) (snd_match_injections)."""
    cd, ct, cs = _f64(cand_dm).ravel(), _f64(cand_t_ms).ravel(), _f64(cand_snr).ravel()
    jd, jt, jw = _f64(inj_dm).ravel(), _f64(inj_t_ms).ravel(), _f64(inj_weff_ms).ravel()
    if not (cd.size == ct.size == cs.size) or not (jd.size == jt.size == jw.size):
        raise ValueError("candidate arrays and injection arrays must each have one length")
    match = np.empty(jd.size, dtype=np.int32)
    n = C.c_int64()
    P = C.c_void_p
    capi.check(capi.lib().snd_match_injections(cd.size, cd.ctypes.data_as(P), ct.ctypes.data_as(P),
                                               cs.ctypes.data_as(P), jd.size, jd.ctypes.data_as(P),
                                               jt.ctypes.data_as(P), jw.ctypes.data_as(P), float(dm_tol),
                                               float(t_frac), match.ctypes.data_as(P), C.byref(n)))
    return match, int(n.value)
