"""GPU parity of the FDMT baseline (no-smear initialisation) against the oracle."""

import sys

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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nchan,n,dm", [(8, 1501, 60.0), (64, 3001, 150.0), (128, 4096, 100.0)])
def test_fdmt_small_exact(snd, orc, nchan, n, dm):
    # spike counts: every partial sum is a small integer, exact in FP32 -> bit-exact
    _say(f"fdmt small nchan={nchan} n={n} dm_max={dm}")
    f = synth.channel_freqs(nchan)
    bw = 16.0 / nchan
    rng = synth.make_rng(nchan)
    x = (rng.random((nchan, n)) < 0.1).astype(np.float32)
    fd = snd.Fdmt(f, bw, 0.138e-3, dm, n)
    y = fd.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    want = orc.fdmt(x, f, bw, 0.138e-3, dm)
    assert y.shape == want.shape and fd.n_delays == want.shape[0]
    assert np.array_equal(y, want.astype(np.float32))
    # Gaussian input: FP32 sums against the FP64 recursion
    g = rng.standard_normal((nchan, n)).astype(np.float32)
    yg = fd.execute(torch.from_numpy(g).cuda()).cpu().numpy()
    wg = orc.fdmt(g, f, bw, 0.138e-3, dm)
    assert np.sqrt(np.mean((yg - wg) ** 2) / np.mean(wg ** 2)) <= 1e-5


def test_fdmt_full_size_sampled_rows(snd, orc):
    # 1024 channels x 2^17 samples up to DM 2000: sampled rows against the direct sum over the
    # channel delays traced down the split rule
    spec = synth.workload(2)
    z = spec.filterbank()
    bw = 16.0 / 1024
    fd = snd.Fdmt(spec.freqs, bw, spec.tsamp_s, 2000.0, spec.nsamp)
    _say(f"fdmt full size: {fd.n_delays} rows, n_out {fd.n_out}, workspace {fd.workspace_bytes / 2**30:.1f} GiB")
    y = fd.execute(torch.from_numpy(z).cuda())
    torch.cuda.synchronize()
    for d in (0, 1, 777, fd.n_delays // 2, fd.n_delays - 1):
        e = orc.fdmt_delays(spec.freqs, bw, spec.tsamp_s, 2000.0, d)
        want = orc.fdmt_row(z, e)[: fd.n_out]
        got = y[d, : fd.n_out].cpu().numpy()
        rel = np.sqrt(np.mean((got - want) ** 2) / np.mean(want ** 2))
        assert rel <= 1e-5, (d, rel)
    del y


def test_fdmt_argument_errors(snd):
    f = synth.channel_freqs(96)
    with pytest.raises(snd.SndError):
        snd.Fdmt(f, 16.0 / 96, 0.138e-3, 100.0, 5000)  # not a power of two
    f = synth.channel_freqs(64)
    with pytest.raises(snd.SndError):
        snd.Fdmt(f, 0.25, 0.138e-3, 3000.0, 1000)  # the sweep does not fit the block


def test_fdmt_dm_zero_is_the_channel_sum(snd, orc):
    f = synth.channel_freqs(16)
    x = synth.make_rng(5).standard_normal((16, 777)).astype(np.float32)
    fd = snd.Fdmt(f, 1.0, 0.138e-3, 0.0, 777)
    assert fd.n_delays == 1 and fd.n_out == 777
    y = fd.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    want = orc.fdmt(x, f, 1.0, 0.138e-3, 0.0)
    assert np.allclose(y, want, rtol=0, atol=1e-5) and np.allclose(want[0], x.astype(np.float64).sum(0))


def test_subband_approx_matches_oracle(snd, orc):
    """Approximate (coarse-DM) sub-band dedispersion: SND plans per sub-band on the coarse grid,
    then the combine kernel, against the oracle's written-out sum (FP32 tolerance); with every DM
    on the coarse grid it is direct dedispersion."""
    rng = synth.make_rng(616)
    f = synth.channel_freqs(64)
    dms = np.sort(rng.uniform(0, 60.0, 150))
    d = orc.delays(f, dms, 0.138e-3)
    nsamp = int(d.max()) + 3000
    x = synth.noise_filterbank(rng, 64, nsamp)
    xt = torch.from_numpy(x).cuda()
    for nsub, step in ((8, 4), (16, 1), (4, 8)):
        sb = snd.SubbandApprox(f, dms, 0.138e-3, nsamp, nsub=nsub, coarse_step=step)
        y = sb.execute(xt).cpu().numpy()
        torch.cuda.synchronize()
        want = orc.subband_approx(x, f, dms, 0.138e-3, nsub, step)
        n = sb.n_out
        assert n <= want.shape[1]
        err = float(np.sqrt(np.mean((y - want[:, :n]) ** 2)) / np.sqrt(np.mean(want[:, :n] ** 2)))
        assert err <= 1e-5, (nsub, step, err)
        if step == 1:
            direct = orc.bruteforce(x, d)
            m = min(n, direct.shape[1])
            assert np.sqrt(np.mean((y[:, :m] - direct[:, :m]) ** 2)) / np.sqrt(np.mean(direct[:, :m] ** 2)) <= 1e-5
