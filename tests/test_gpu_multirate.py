"""GPU parity of the multi-rate pipeline (Methods, "Multi-rate extension") against the oracle:
the time scrunch bit for bit, and per band the re-encoded tree, the S/N and candidates, then
the cross-band merge."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDTHS = [1, 2, 4, 8, 16, 32]


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_scrunch_bit_exact(snd, orc):
    rng = synth.make_rng(12)
    z = rng.standard_normal((37, 1001)).astype(np.float32)
    zt = torch.from_numpy(z).cuda()
    for s in (1, 2, 3, 8, 16, 1001, 1024):
        _say(f"scrunch s={s}")
        got = snd.scrunch(zt, s).cpu().numpy()
        assert np.array_equal(got, orc.scrunch(z, s))


def _oracle_band(orc, z, f, dms, s, tsamp, mode, thr, kw, sigma_min, theta):
    zs = orc.scrunch(z, s)
    x = zs if mode == "float" else orc.encode(zs, thr)
    d = orc.delays(f, dms, tsamp * s)
    plane, _ = orc.snd_dedup(x, f, d, mode=mode, cluster=4, branching=2, **kw)
    snr, widx, _, _ = orc.matched_filter(plane, WIDTHS, integer_plane=mode != "float", sigma_min=sigma_min)
    return x, plane, orc.candidates(snr, widx, theta, radius=4, n_min=10)


@pytest.mark.parametrize("mode,thr,kw,sigma_min", [("binary", [2.0], dict(k_leaf=2, k_int=1), 0.15),
                                                    ("graded", [1.0, 2.0, 3.0, 4.0], {}, 0.0),
                                                    ("float", None, {}, 0.0)])
def test_multirate_pipeline_matches_oracle(snd, orc, mode, thr, kw, sigma_min):
    spec = synth.workload(1)  # 64 channels, 8192 samples, one pulse at DM 150
    z = spec.filterbank()
    dms = np.linspace(0.0, 300.0, 160)  # 1.9 DM steps: the pulse lands within a sample of a trial in every band
    theta = 6.0
    mr = snd.MultiRate(spec.freqs, dms, spec.tsamp_s, z.shape[1], mode=mode, thresholds=thr, widths=WIDTHS,
                       threshold=theta, sigma_min=sigma_min, branching=2, **kw)
    factors = orc.scrunch_factors(spec.freqs, dms, spec.tsamp_s, 16)
    assert np.array_equal(mr.factors, factors) and sorted(set(factors)) == [1, 2, 4, 8, 16]
    zt = torch.from_numpy(z).cuda()
    merged, per_band = mr.run(zt)
    want_all = []
    for bi, b in enumerate(mr.bands):
        s, idx = b["s"], b["idx"]
        _say(f"multirate mode={mode} band S={s}: {idx.size} DMs")
        x, plane, want = _oracle_band(orc, z, spec.freqs, dms[idx], s, spec.tsamp_s, mode, thr, kw, sigma_min, theta)
        xin = mr.band_input(zt, s)
        if mode != "float":
            assert np.array_equal(xin.cpu().numpy(), x)  # re-encoded raster, bit for bit
        y = b["plan"].execute(xin)
        torch.cuda.synchronize()
        yy = y.cpu().numpy()
        if mode == "float":
            assert np.sqrt(np.mean((yy - plane) ** 2)) <= 1e-5 * np.sqrt(np.mean(plane ** 2))
        else:
            assert np.array_equal(yy, plane.astype(yy.dtype))
        got = per_band[bi]
        if mode != "float":
            assert [(c["k"], c["t"], c["npix"]) for c in got] == [(int(idx[w["k"]]), w["t"], w["npix"]) for w in want]
            assert [c["snr"] for c in got] == [w["snr"] for w in want]
        want_all += [dict(dm=float(dms[idx[w["k"]]]), t_ms=w["t"] * s * (spec.tsamp_s * 1e3), snr=w["snr"], k=int(idx[w["k"]]))
                     for w in want]
    want_merged = orc.merge_candidates(want_all)
    if mode != "float":
        assert [(c["k"], c["t_ms"]) for c in merged] == [(c["k"], c["t_ms"]) for c in want_merged]
    # float mode finds the injected pulse (DM 150, sample 2048 at the top of the band) in its
    # S = 16 band; the encoded modes lose most of a 1 ms pulse in 2.2 ms scrunched samples
    if mode == "float":
        assert any(abs(c["dm"] - 150.0) <= 20.0 and abs(c["t_ms"] - 2048 * 0.138) <= 50.0 for c in merged), merged
