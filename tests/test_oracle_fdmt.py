"""Pins for the oracle's FDMT with the no-smear initialisation (Methods, "Classical
dedispersion algorithms")."""

import math

import numpy as np
import pytest

import synth

K_DM_MS = 4.148808e6


def _case(nchan=64, n=3000, dm_max=150.0, seed=1):
    # DM 150 sweeps about 2130 samples of 0.138 ms across 400-416 MHz
    f = synth.channel_freqs(nchan)
    bw = 16.0 / nchan
    rng = np.random.default_rng(seed)
    x = (rng.random((nchan, n)) < 0.05).astype(np.float64)
    return f, bw, x, dm_max


def test_recursion_equals_direct_sums_over_traced_delays(orc):
    # two different computations of the same rows: the log2(nchan) merges, and for each row
    # the plain sum over channels at the delays found by following the split rule down
    for nchan in (8, 64):
        f, bw, x, dm = _case(nchan=nchan, n=1500, dm_max=80.0)
        y = orc.fdmt(x, f, bw, 0.138e-3, dm)
        for d in range(y.shape[0]):
            assert np.array_equal(y[d], orc.fdmt_row(x, orc.fdmt_delays(f, bw, 0.138e-3, dm, d))), (nchan, d)


def test_zero_delay_row_is_the_channel_sum_and_shape(orc):
    f, bw, x, dm = _case()
    y = orc.fdmt(x, f, bw, 0.138e-3, dm)
    assert np.array_equal(y[0], x.sum(0))
    # D + 1 rows, D the band sweep at dm_max in samples, from the outer channel edges
    sweep = K_DM_MS * dm * ((f[-1] - bw / 2) ** -2 - (f[0] + bw / 2) ** -2) / 0.138
    assert y.shape == (math.ceil(sweep) + 1, x.shape[1])


def test_traced_delays_follow_the_dispersion_law(orc):
    # row d stands for the DM whose sweep across the band is d samples; each channel is read at
    # that DM's delay of its upper edge below the band's upper edge, up to the rounding of one
    # split per merge (log2 nchan merges)
    for nchan in (16, 64, 256):
        f = synth.channel_freqs(nchan)
        bw = 16.0 / nchan
        dm_max = 200.0
        hi = f + bw / 2
        r_band = (f[-1] - bw / 2) ** -2 - hi[0] ** -2
        D = math.ceil(K_DM_MS * dm_max * r_band / 0.138)
        for d in (1, D // 3, D // 2, D):
            e = orc.fdmt_delays(f, bw, 0.138e-3, dm_max, d)
            ideal = d * (hi ** -2 - hi[0] ** -2) / r_band
            assert e[0] == 0
            assert np.all(np.diff(e) >= 0)  # lower channels are read later
            assert np.max(np.abs(e - ideal)) <= math.log2(nchan), (nchan, d)


def test_no_smear_spike_track_sums_every_channel(orc):
    # spikes placed exactly on row d's track add up to the channel count at the track's start:
    # the no-smear initialisation spreads no spike over other delays
    f, bw, _, dm = _case(nchan=32, n=2000, dm_max=100.0)
    y0 = orc.fdmt(np.zeros((32, 2000)), f, bw, 0.138e-3, dm)
    for d in (0, y0.shape[0] // 2, y0.shape[0] - 1):
        e = orc.fdmt_delays(f, bw, 0.138e-3, dm, d)
        x = np.zeros((32, 2000))
        x[np.arange(32), 100 + e] = 1.0
        y = orc.fdmt(x, f, bw, 0.138e-3, dm)
        assert y[d, 100] == 32.0
        assert y.max() == 32.0


def test_subband_approx_pins():
    """Approximate sub-band dedispersion: with every DM on the coarse grid it is brute-force
    dedispersion; otherwise the rows whose DM lies on the coarse grid still are, and the others
    differ only through the sub-bands' internal sweeps (bounded by the pulse smear)."""
    import oracle as orc
    rng = synth.make_rng(515)
    f = synth.channel_freqs(32)
    dms = np.sort(rng.uniform(0, 80.0, 40))
    d = orc.delays(f, dms, 0.138e-3)
    x = rng.standard_normal((32, int(d.max()) + 400))
    exact = orc.bruteforce(x, d)
    y1 = orc.subband_approx(x, f, dms, 0.138e-3, nsub=4, coarse_step=1)
    assert y1.shape == exact.shape and np.allclose(y1, exact, rtol=0, atol=1e-12)
    y4 = orc.subband_approx(x, f, dms, 0.138e-3, nsub=4, coarse_step=4)
    on_grid = np.isin(dms, np.unique(dms)[::4])
    n = min(y4.shape[1], exact.shape[1])
    assert np.allclose(y4[on_grid, :n], exact[on_grid, :n], rtol=0, atol=1e-12)
    assert not np.allclose(y4[~on_grid, :n], exact[~on_grid, :n])
    # a delta pulse: every sub-band's channels meet at the same time only on the coarse grid;
    # off the grid the channels of a sub-band land within its internal sweep difference
    z = np.zeros((32, int(d.max()) + 400))
    t0 = 150
    k = int(np.flatnonzero(~on_grid)[0])
    for c in range(32):
        z[c, t0 + d[k, c]] = 1.0
    yz = orc.subband_approx(z, f, dms, 0.138e-3, nsub=4, coarse_step=4)
    assert yz[k].sum() == 32.0 and yz[k].max() < 32.0
