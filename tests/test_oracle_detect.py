"""Pins for the oracle's matched filter and candidate extraction."""

import math

import numpy as np
import pytest
from scipy import ndimage

import synth


def test_noise_floor_closed_forms(orc):
    # Methods, matched filtering: with sigma_min = 0.15 a single fire in a W = 64 boxcar
    # gives S/N ~0.8 and a cluster of ~25 fires gives ~21 (row mean ~0 on a sparse plane).
    n = 100000
    y = np.zeros((2, n))
    y[0, 5000] = 1
    y[1, 5000:5025] = 1
    snr, widx, mu, sg = orc.matched_filter(y, [64], integer_plane=True, sigma_min=0.15)
    assert np.all(sg == 0.15)
    assert abs(snr[0].max() - 0.8) < 0.05
    assert abs(snr[1].max() - 21.0) < 0.3
    assert snr[0].argmax() == 5000 - 63


def test_gaussian_noise_snr_statistics(orc):
    # On N(0,1) rows the W-boxcar S/N at any fixed t is N(0,1) (sum of W unit normals scaled
    # by sqrt(W)), so per width the mean is ~0 and the spread ~1.
    rng = synth.make_rng(4)
    y = rng.standard_normal((4, 20000))
    for w in (1, 4, 16):
        snr, _, mu, sg = orc.matched_filter(y, [w], integer_plane=False)
        valid = snr[:, : y.shape[1] - w + 1]
        assert abs(valid.mean()) < 0.05
        assert abs(valid.std() - 1.0) < 0.05
    np.testing.assert_allclose(mu, y.mean(axis=1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(sg, y.std(axis=1), rtol=1e-12)


def test_boxcar_matched_width_is_optimal(orc):
    # A rectangular pulse of width 8 on a quiet row peaks at its start with W = 8.
    y = np.zeros((1, 4096))
    rng = synth.make_rng(5)
    y[0] = rng.standard_normal(4096) * 0.01
    y[0, 1000:1008] += 1.0
    snr, widx, _, _ = orc.matched_filter(y, [1, 2, 4, 8, 16, 32], integer_plane=False)
    assert int(snr[0].argmax()) == 1000
    assert widx[0, 1000] == 3
    assert widx[0, -1] == 0 and widx[0, -40] >= 0  # only W = 1 fits at the last sample


def test_constant_row_has_zero_snr(orc):
    y = np.full((2, 300), 3.0)
    snr, widx, mu, sg = orc.matched_filter(y, [1, 2], integer_plane=True)
    assert np.all(snr == 0) and np.all(sg == 0) and np.all(mu == 3.0)
    with pytest.raises(ValueError):
        orc.matched_filter(y, [2, 2], integer_plane=True)


def _scipy_islands(mask, r):
    pad = 2 * r
    m = np.pad(mask, pad)
    se = np.ones((2 * r + 1, 2 * r + 1), bool)
    closed = ndimage.binary_erosion(ndimage.binary_dilation(m, se), se)[pad:-pad, pad:-pad]
    lab, n = ndimage.label(closed, structure=np.ones((3, 3), bool))
    return lab, n


def test_closing_merges_row_pairs_up_to_gap_nine(orc):
    for gap, expect in ((9, 1), (10, 2)):
        snr = np.zeros((20, 60))
        snr[10, 20] = 8.0
        snr[10, 20 + gap] = 9.0
        widx = np.zeros(snr.shape, np.int32)
        c = orc.candidates(snr, widx, 7.0, radius=4, n_min=1)
        assert len(c) == expect
        if expect == 1:
            assert c[0]["npix"] == gap + 1 and c[0]["t"] == 20 + gap and c[0]["snr"] == 9.0


def test_closing_keeps_diagonal_pairs_apart(orc):
    for d in (2, 3, 5, 8):
        snr = np.zeros((30, 30))
        snr[5, 5] = 8.0
        snr[5 + d, 5 + d] = 8.0
        c = orc.candidates(snr, np.zeros(snr.shape, np.int32), 7.0, radius=4, n_min=1)
        assert len(c) == 2 and all(x["npix"] == 1 for x in c)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_candidates_match_scipy_closing_and_labelling(orc, seed):
    rng = synth.make_rng(100 + seed)
    snr = rng.standard_normal((40, 300)) * 2.0
    snr[12:15, 100:140] += 9.0
    snr[0:2, 0:5] += 9.0            # touches the plane border
    widx = rng.integers(0, 5, size=snr.shape).astype(np.int32)
    theta = 5.0
    lab, n = _scipy_islands(snr >= theta, 4)
    for n_min in (1, 10):
        got = orc.candidates(snr, widx, theta, radius=4, n_min=n_min)
        want = []
        for i in range(1, n + 1):
            pix = np.argwhere(lab == i)
            if len(pix) < n_min:
                continue
            vals = snr[pix[:, 0], pix[:, 1]]
            best = vals.max()
            sel = pix[vals == best]
            k, t = min(map(tuple, sel))
            want.append(dict(k=int(k), t=int(t), widx=int(widx[k, t]), snr=float(best), npix=len(pix)))
        want.sort(key=lambda c: (c["k"], c["t"]))
        assert got == want


def test_binary_snr_prediction_limits(orc):
    # Eq. snr_A grows as sqrt(W) and vanishes when signal and noise rates are equal.
    assert orc.binary_snr(4, 0.5, 0.1) == pytest.approx(2 * orc.binary_snr(1, 0.5, 0.1))
    assert orc.binary_snr(16, 0.2, 0.2) == 0.0
    assert math.isclose(orc.binary_snr(1, 1.0, 0.5), 1.0)


PAPER_WIDTHS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024]


def test_dm_width_counts_northern_cross(orc):
    # Methods, matched filtering, the DM-scaled width set with base {1, 2, 4, 8} and alpha = 0.1,
    # evaluated by hand for the Northern Cross band (channel centres 416 - (c + 1/2) 16/1024 MHz,
    # lowest 400.0078125, highest 415.9921875; dt = 0.138 ms):
    #   sweep / dt = 4.148808e6 * d * (400.0078125^-2 - 415.9921875^-2) / 0.138 = 14.1619 * d
    #   d = 0: 0 -> base only; d = 10: alpha * sweep = 14.16 -> base only; d = 25: 35.4 -> + 16, 32;
    #   d = 50: 70.8 -> + 64; d = 100: 141.6 -> + 128; d = 200: 283.2 -> + 256; d = 400: 566.5
    #   -> + 512; d = 2000: 2832 -> every width up to 1024
    f = synth.channel_freqs(1024)
    dms = [0.0, 10.0, 25.0, 50.0, 100.0, 200.0, 400.0, 2000.0]
    got = orc.dm_width_counts(f, dms, 0.138e-3, PAPER_WIDTHS, 4, 0.1)
    assert list(got) == [4, 4, 6, 7, 8, 9, 10, 11]
    # the sweep at d = 2000 rounds to the band's largest channel delay, 28,324 samples
    assert int(orc.delays(f, [2000.0], 0.138e-3).max()) == 28324
    # no base given: every row keeps every width
    assert list(orc.dm_width_counts(f, dms, 0.138e-3, PAPER_WIDTHS, 0, 0.1)) == [11] * 8


@pytest.mark.parametrize("integer_plane", [True, False])
def test_row_width_counts_reduce_to_the_plain_filter(orc, integer_plane):
    rng = synth.make_rng(41)
    y = rng.integers(0, 5, (6, 700)).astype(np.float64) if integer_plane else rng.standard_normal((6, 700))
    y[2, 300:340] += 3.0
    counts = np.array([1, 3, 5, 7, 2, 7], dtype=np.int32)
    snr, widx, mu, sg = orc.matched_filter(y, PAPER_WIDTHS[:7], integer_plane=integer_plane, row_nw=counts)
    for k, n in enumerate(counts):
        s1, w1, m1, g1 = orc.matched_filter(y[k:k + 1], PAPER_WIDTHS[:n], integer_plane=integer_plane)
        assert np.array_equal(snr[k], s1[0]) and np.array_equal(widx[k], w1[0])
        assert mu[k] == m1[0] and sg[k] == g1[0]


def test_mad_sigma_pins(orc):
    """Robust sigma from the median absolute deviation (lower medians)."""
    from scipy.stats import norm
    # the scale is 1 / Phi^-1(3/4), from scipy's normal quantile
    assert orc.MAD_SCALE == pytest.approx(1.0 / norm.ppf(0.75), rel=2e-16)
    # odd length: median 3, deviations 2 1 0 1 97, their lower median 1
    assert orc.mad_sigma(np.array([[1, 2, 3, 4, 100]], np.uint8))[0] == orc.MAD_SCALE
    # even length: lower median 2 (not 2.5), deviations 1 0 1 8, lower median 1
    assert orc.mad_sigma(np.array([[1.0, 2.0, 3.0, 10.0]], np.float32))[0] == orc.MAD_SCALE
    assert orc.mad_sigma(np.array([[10, 3, 2, 1]], np.uint16))[0] == orc.MAD_SCALE
    # a constant row has MAD 0; a row of two values has the smaller deviation 0
    assert orc.mad_sigma(np.full((1, 7), 5, np.uint8))[0] == 0.0
    # Gaussian rows: the MAD sigma estimates the standard deviation
    rng = np.random.default_rng(3)
    g = (rng.standard_normal((3, 200001)) * np.array([[0.5], [2.0], [7.0]])).astype(np.float32)
    assert np.allclose(orc.mad_sigma(g), [0.5, 2.0, 7.0], rtol=0.01)
    # a bright burst in 2 % of the samples inflates the standard deviation, not the MAD sigma
    b = g[1].copy()
    b[:4000] += 60.0
    _, _, _, sd = orc.matched_filter(b[None, :].astype(np.float64), [1], integer_plane=False)
    assert sd[0] > 4.0
    assert orc.mad_sigma(b[None, :])[0] == pytest.approx(2.0, rel=0.05)
    # the matched filter takes the given sigma, floored by sigma_min
    row = np.array([[0, 0, 1, 0, 0, 3, 0, 0]], np.float64)
    snr, _, mu, sg = orc.matched_filter(row, [1], integer_plane=True, sigma_rows=[0.25], sigma_min=0.5)
    assert sg[0] == 0.5 and mu[0] == 0.5
    assert snr[0, 5] == pytest.approx((3 - 0.5) / 0.5)
