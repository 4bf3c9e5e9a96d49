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
