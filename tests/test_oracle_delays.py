"""Pins for the oracle's delay table and tree shape (paper values and textbook constants)."""

import numpy as np
import pytest

import synth


def test_textbook_dispersion_constant(orc):
    # Methods, "Incoherent dedispersion": K_DM ~ 4.149e6 MHz^2 ms; the handbook value is
    # 4.148808 ms per unit DM at 1 GHz against an infinitely high reference frequency.
    d = orc.delays([1000.0], [1.0, 10.0, 100.0], 1e-6, fref=1e9)
    assert d[:, 0].tolist() == [4149, 41488, 414881]


def test_nc_sweep_at_dm3000(orc):
    # Methods, hardware mapping: the dispersive sweep at DM 3000 spans about 42,500 native
    # samples for the Northern Cross band (1024 ch, 408 MHz, 16 MHz, 0.138 ms).
    f = synth.channel_freqs(1024)
    d = orc.delays(f, [3000.0], 0.138e-3)
    assert abs(int(d.max()) - 42500) <= 100
    assert d[0, 0] == 0 and d[0, -1] == d.max()


def test_scrunch_band_edges_match_channel_delay(orc):
    # Eq. scrunch with Table S1: the S = 2, 4, 8, 16 bands start at DM 289, 578, 1157, 2313,
    # where the intra-channel smearing K d df / f_c^3 equals S * dt.  The delay between two
    # adjacent channels is twice that smearing, so at each printed edge the integer delay
    # step across the band centre must be 2 S samples (+-1 for rounding).
    f = synth.channel_freqs(1024)
    c = int(np.argmin(np.abs(f - 408.0)))
    for S, dm in ((2, 289.0), (4, 578.0), (8, 1157.0), (16, 2313.0)):
        d = orc.delays(f, [dm], 0.138e-3)[0]
        step = int(d[c + 1] - d[c])
        assert abs(step - 2 * S) <= 1, (S, step)


def test_delay_monotone_and_zero_dm(orc):
    f = synth.channel_freqs(64)
    dms = synth.dm_linear(50, 0.0, 300.0)
    d = orc.delays(f, dms, 0.138e-3)
    assert np.all(d[0] == 0)
    assert np.all(np.diff(d, axis=0) >= 0)      # non-decreasing in DM
    assert np.all(np.diff(d, axis=1) >= 0)      # non-decreasing towards low frequency
    with pytest.raises(ValueError):
        orc.delays(f, dms, 0.138e-3, fref=410.0)


def test_tree_shape_northern_cross(orc):
    # Table S1: C = 4, B = 8 gives leaf + L1 + L2 + root with B_root = 4 for 1024 channels.
    f = synth.channel_freqs(1024)
    assert orc.tree_shape(f, 4, 8) == [256, 32, 4, 1]
    assert orc.tree_shape(f, 4, 4) == [256, 64, 16, 4, 1]
    assert orc.tree_shape(synth.channel_freqs(37), 3, 3) == [13, 5, 2, 1]
    assert orc.tree_shape(synth.channel_freqs(3), 4, 2) == [1]
