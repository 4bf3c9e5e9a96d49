"""Pins for the oracle's multi-rate extension (Methods, "Multi-rate extension")."""

import math

import numpy as np

import synth


def test_band_edges_of_the_northern_cross(orc):
    # Eq. scrunch with the Northern Cross band (408 MHz centre, 15.625 kHz channels, 0.138 ms):
    # tau_smear(d) = 4.148808e6 d 0.015625 / 408^3 ms = 9.5446e-4 d ms, so S = 2 from
    # d = 0.276 / 9.5446e-4 = 289.2, S = 4 from 578.3, S = 8 from 1156.7, S = 16 from 2313.3:
    # the printed edges 289 / 578 / 1157 / 2313.
    f = synth.channel_freqs(1024)
    dms = [0, 100, 289.0, 289.5, 578.0, 578.5, 1156.5, 1157.0, 2313.0, 2313.5, 3000.0]
    got = orc.scrunch_factors(f, dms, 0.138e-3, s_max=16)
    assert list(got) == [1, 1, 1, 2, 2, 4, 4, 8, 8, 16, 16]
    assert list(orc.scrunch_factors(f, [3000.0], 0.138e-3, s_max=4)) == [4]


def test_scrunch_identity_constants_and_conservation(orc):
    rng = synth.make_rng(5)
    z = rng.standard_normal((3, 101)).astype(np.float32)
    assert np.array_equal(orc.scrunch(z, 1), z)
    c = np.full((2, 64), 0.5, np.float32)
    for s in (2, 4, 8, 16):
        out = orc.scrunch(c, s)
        assert out.shape == (2, 64 // s)
        assert np.allclose(out, 0.5 * math.sqrt(s), rtol=1e-6)
    for s in (2, 3, 8):
        out = orc.scrunch(z, s)
        n = out.shape[1]
        assert n == 101 // s
        # every covered input sample is counted once, no sample twice
        assert np.allclose(out.astype(np.float64).sum(1) * math.sqrt(s), z[:, :n * s].astype(np.float64).sum(1),
                           rtol=1e-5, atol=1e-4)


def test_merge_candidates_hand_cases(orc):
    c = lambda dm, t, snr: dict(dm=dm, t_ms=t, snr=snr)
    # B absorbs A (10 DM, 100 ms apart) and C (20 DM, 100 ms from B); D is 201 ms from B
    cands = [c(100, 1000, 10), c(110, 1100, 12), c(130, 1200, 9), c(110, 1301, 8)]
    got = orc.merge_candidates(cands)
    assert [(g["dm"], g["t_ms"]) for g in got] == [(110, 1100), (110, 1301)]
    # a chain is not transitive: E keeps only what is within reach of the strongest
    cands = [c(0, 0, 20), c(15, 150, 5), c(30, 300, 6)]
    got = orc.merge_candidates(cands)
    assert [(g["dm"], g["t_ms"]) for g in got] == [(0, 0), (30, 300)]
    # ties in S/N: the lower DM is kept
    got = orc.merge_candidates([c(50, 10, 7), c(40, 10, 7)])
    assert [(g["dm"], g["t_ms"]) for g in got] == [(40, 10)]
    assert orc.merge_candidates([]) == []
