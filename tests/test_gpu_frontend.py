"""GPU parity of the front end (two-pass sigma-clip normalisation of raw power, then the
encoders) against the oracle."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


def test_sigma_clip_normalise_and_encode(snd, orc):
    rng = synth.make_rng(31)
    nchan, n = 96, 20000
    # raw power: chi-squared-like (exponential) with per-channel gains and offsets, RFI spikes
    p = (rng.exponential(1.0, (nchan, n)) * rng.uniform(0.5, 3.0, (nchan, 1)) + rng.uniform(0, 10, (nchan, 1)))
    p[5, 100:120] += 500.0
    p[17, ::997] += 80.0
    p[40] = 2.5  # a constant channel: sigma 0
    p[40, 7] = 2.5
    p = p.astype(np.float32)
    want_st = orc.sigma_clip_stats(p, 5.0)
    pt = torch.from_numpy(p).cuda()
    st = snd.channel_stats(pt, 5.0)
    got_st = st.cpu().numpy()
    ok = np.arange(nchan) != 40
    assert np.allclose(got_st[ok], want_st[ok], rtol=1e-12, atol=0.0)
    assert got_st[40, 0] == pytest.approx(2.5) and got_st[40, 1] == 0.0
    # normalise and encode the channels with sigma > 0 from the oracle's statistics: the
    # rasters must agree bit for bit (the same FP64 quotient, the same FP32 comparisons)
    sel = torch.from_numpy(np.flatnonzero(ok)).cuda()
    z = snd.normalize(pt[sel].contiguous(), torch.from_numpy(want_st[ok]).cuda())
    zw = orc.normalize(p[ok], want_st[ok])
    assert np.array_equal(z.cpu().numpy(), zw)
    for thr in ([1.5], [0.75], [1.0, 2.0, 3.0, 4.0]):
        assert np.array_equal(snd.encode(z, thr).cpu().numpy(), orc.encode(zw, thr))
    # with the GPU's own statistics the normalised values agree to FP64 rounding
    z2 = snd.normalize(pt[sel].contiguous(), st[sel].contiguous()).cpu().numpy()
    assert np.max(np.abs(z2 - zw)) <= 1e-5


def _flag_threshold_margin(sig, k):
    """Per window: distance of each channel's |s_c - m| from the flagging threshold
    k * MAD_SCALE * MAD, relative to the threshold (from the oracle's sigmas)."""
    import oracle
    out = np.empty_like(sig)
    for b in range(sig.shape[0]):
        s = sig[b]
        m = np.sort(s)[(s.size - 1) // 2]
        d = np.abs(s - m)
        thr = k * oracle.MAD_SCALE * np.sort(d)[(d.size - 1) // 2]
        out[b] = np.abs(d - thr) / max(thr, np.finfo(np.float64).tiny)
    return out


@pytest.mark.parametrize("nchan,n,window", [(96, 20011, 4096), (1024, 16384, 8192), (7, 1000, 1000)])
def test_flagging_and_zero_dm(snd, orc, nchan, n, window):
    # windowed MAD channel flagging, then zero-DM subtraction, on a z-scored block with RFI.
    # The oracle sums each window in time order, the kernel in its own order: the channel
    # sigmas agree to FP64 rounding (1e-12 relative).  A flag can then differ only for a channel
    # within that rounding of the threshold; no channel of this data comes within 1e-9 of it,
    # so the flags, and with them the zeroed samples, must agree exactly.  Zero-DM subtraction
    # then sums each sample's channels in channel order on both sides: bit-exact.
    rng = synth.make_rng(nchan + window)
    z = rng.standard_normal((nchan, n)).astype(np.float32)
    z[nchan // 3, : min(n, window)] *= 12.0            # hot channel in the first window
    z[nchan // 2, :] = 0.0                              # dead channel
    z[:, n // 2] += 8.0 / np.sqrt(nchan) * 3.0          # broadband spikes (zero-DM S/N ~ 24)
    z[:, n // 3: n // 3 + 5] += 2.0
    z[1, 17] += 40.0                                    # narrow-band spike
    zt = torch.from_numpy(z).cuda()
    flags, sig = snd.flag_channels(zt, window, k=5.0, return_sigma=True)
    want_z, want_f, want_s = orc.flag_channels(z, window, k=5.0, return_sigma=True)
    got_s = sig.cpu().numpy()
    assert np.allclose(got_s, want_s, rtol=1e-12, atol=1e-300)
    assert np.all((got_s == 0) == (want_s == 0))        # the dead channel is exactly 0 on both sides
    assert np.all(_flag_threshold_margin(want_s, 5.0) > 1e-9), "a channel sits on the flag threshold"
    assert np.array_equal(flags.cpu().numpy(), want_f)
    assert np.array_equal(zt.cpu().numpy(), want_z)
    assert want_f[0, nchan // 3] == 1 and np.all(want_f[:, nchan // 2] == 1)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    snd.zero_dm(zt, 5.0, count=cnt)
    want_z2, want_n = orc.zero_dm(want_z, 5.0)
    assert int(cnt.item()) == want_n and want_n >= 1  # at least the strong broadband spike
    assert np.array_equal(zt.cpu().numpy(), want_z2)
