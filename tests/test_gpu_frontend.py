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
