"""Pins for the oracle's front end (Methods, "Input encoding": two-pass sigma-clip normalisation)."""

import math

import numpy as np
import pytest

import synth


def test_clipped_outlier_by_hand(orc):
    # 99 samples of 1 and one of 1000: mu0 = 10.99, sigma0 = sqrt(10000.99 - 10.99^2) = 99.39924;
    # the outlier is moved to mu0 + 5 sigma0 = 507.98622, so mu = (99 + 507.98622) / 100 = 6.0698622
    # and sigma = sqrt((99 + 507.98622^2) / 100 - 6.0698622^2) = 50.444492
    p = np.array([[1.0] * 99 + [1000.0]])
    st = orc.sigma_clip_stats(p, 5.0)
    assert st[0, 0] == pytest.approx(6.0698622, rel=1e-7)
    assert st[0, 1] == pytest.approx(50.444492, rel=1e-7)


def test_no_clipping_is_plain_mean_and_std(orc):
    rng = synth.make_rng(3)
    p = (7.0 + 2.0 * rng.standard_normal((3, 5000))).astype(np.float32)
    x = p.astype(np.float64)
    assert np.all(np.abs(x - x.mean(1, keepdims=True)) < 5 * x.std(1, keepdims=True))
    st = orc.sigma_clip_stats(p, 5.0)
    assert np.allclose(st[:, 0], x.mean(1), rtol=1e-12) and np.allclose(st[:, 1], x.std(1), rtol=1e-12)


def test_normalised_fire_rate_is_the_normal_tail(orc):
    rng = synth.make_rng(4)
    p = (3.0 + 2.0 * rng.standard_normal((2, 200000))).astype(np.float32)
    z = orc.normalize(p, orc.sigma_clip_stats(p, 5.0))
    assert z.dtype == np.float32
    rate = float((z > np.float32(1.5)).mean())
    want = orc.fire_probability(1.5)  # 0.0668
    assert abs(rate - want) < 4 * math.sqrt(want * (1 - want) / z.size)


def test_zero_dm_pins(orc):
    rng = np.random.default_rng(21)
    nchan, n = 64, 500
    z = rng.standard_normal((nchan, n)).astype(np.float32)
    # a broadband spike: +3 in every channel at t = 100, zero-DM S/N about 3 sqrt(64) = 24
    z[:, 100] += 3.0
    # a narrow-band spike of the same total power in one channel: S/N about 192/8 = 24 too, but
    # the subtraction spreads it (it is broadband only in sum)
    z[7, 300] += 192.0
    # a weak broadband excursion: S/N about 0.5 * 8 = 4 < 5, kept
    z[:, 400] += 0.5
    out, changed = orc.zero_dm(z, 5.0)
    zc = z.astype(np.float64)
    snr = np.abs(zc.sum(0)) / 8.0
    assert changed == int((snr > 5.0).sum())
    # at t = 100 the added constant vanishes: the column equals the noise minus its own mean
    noise = zc[:, 100] - 3.0
    assert np.allclose(out[:, 100], noise - noise.mean(), atol=1e-5)
    assert abs(out[:, 100].astype(np.float64).sum()) < 1e-4
    # untouched columns are bit-identical
    keep = snr <= 5.0
    assert keep[400] and np.array_equal(out[:, keep], z[:, keep])
    # closed form of the threshold: a constant block c has S/N |c| sqrt(nchan)
    c = np.full((16, 4), 1.25, np.float32)  # 1.25 * 4 = 5: not above 5
    assert orc.zero_dm(c, 5.0)[1] == 0
    c2 = np.full((16, 4), 1.3, np.float32)
    o2, k2 = orc.zero_dm(c2, 5.0)
    assert k2 == 4 and np.all(o2 == 0.0)


def test_flag_channels_pins(orc):
    rng = np.random.default_rng(22)
    nchan, n, w = 32, 3000, 1000
    z = rng.standard_normal((nchan, n)).astype(np.float32)
    z[5, 1000:2000] *= 10.0      # hot in window 1 only
    z[9, :] = 0.25               # dead channel: sigma 0 in every window
    out, flags = orc.flag_channels(z, w, k=5.0)
    assert flags.shape == (3, nchan)
    assert flags[1, 5] == 1 and flags[0, 5] == 0 and flags[2, 5] == 0
    assert np.all(flags[:, 9] == 1)
    assert flags.sum() == 4  # nothing else in a clean Gaussian block at 5 MADs
    assert np.all(out[5, 1000:2000] == 0.0) and np.array_equal(out[5, :1000], z[5, :1000])
    assert np.all(out[9] == 0.0)
    # hand-evaluated window: channel standard deviations 1, 2, 3, 4 and 50 (values +-s, even
    # length); m = 3, deviations 2 1 0 1 47, MAD = 1, scaled 1.4826: with k = 5 only the
    # channel at 50 (47 > 7.41) is flagged; with k = 1 the channels at 1 and 50 (2 > 1.48)
    s = np.array([1.0, 2.0, 3.0, 4.0, 50.0], np.float32)[:, None]
    h = np.tile(np.array([1.0, -1.0], np.float32), (5, 4)) * s
    assert list(orc.flag_channels(h, 8, k=5.0)[1][0]) == [0, 0, 0, 0, 1]
    assert list(orc.flag_channels(h, 8, k=1.0)[1][0]) == [1, 0, 0, 0, 1]


def test_flag_window_sigma_is_the_population_std(orc):
    # the per-window channel sigma is the population standard deviation of the window's samples
    # (two-pass FP64 sums in time order): numpy's own std, which sums pairwise, agrees to FP64
    # rounding; the last window is ragged
    rng = np.random.default_rng(23)
    nchan, n, w = 9, 2500, 1000
    z = (3.0 + rng.standard_normal((nchan, n)) * rng.uniform(0.5, 4.0, (nchan, 1))).astype(np.float32)
    _, _, sig = orc.flag_channels(z, w, k=5.0, return_sigma=True)
    assert sig.shape == (3, nchan)
    for b in range(3):
        want = z[:, b * w: (b + 1) * w].astype(np.float64).std(axis=1)
        assert np.allclose(sig[b], want, rtol=1e-12, atol=0.0)
