"""Reduced-precision storage at the headline size (1024 channels, 4096 DMs, 2^17 samples):
the float tree with the filterbank and tree rows in BF16 or FP16 (FP32 accumulation) against
the FP64 oracle run on the original float32 input -- relative RMS error over sampled rows,
and the S/N of the brightest injected pulses within 1 % of the oracle's."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDTHS = (1, 2, 4, 8, 16, 32, 64)
TOL = {"f32": 1e-5, "bf16": 1e-2, "f16": 1e-2}


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


@pytest.fixture(scope="module")
def beam(orc):
    spec = synth.workload(2)
    z = spec.filterbank()
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    return spec, z, d


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_storage_error_against_fp64_oracle(snd, orc, beam, storage):
    spec, z, d = beam
    zt = torch.from_numpy(z).cuda()
    x = zt if storage == "f32" else snd.cast(zt, storage)
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4, in_dtype=storage,
                 node_dtype=storage)
    y = p.execute(x)
    torch.cuda.synchronize()
    rng = synth.make_rng(31)
    ks = np.repeat(rng.choice(spec.dms.size, 48, replace=False), 512).astype(np.int32)
    t0 = rng.integers(0, p.n_out - 512, 48)
    ts = (t0[:, None] + np.arange(512)[None, :]).ravel().astype(np.int64)
    want = orc.snd_points(z, spec.freqs, d, ks, ts, mode="float", cluster=4, branching=4)
    got = y[torch.from_numpy(ks).long().cuda(), torch.from_numpy(ts).cuda()].double().cpu().numpy()
    err = float(np.sqrt(np.mean((got - want) ** 2)) / np.sqrt(np.mean(want ** 2)))
    _say(f"storage {storage}: rel-RMS {err:.3e} over {ks.size} sampled outputs")
    assert err <= TOL[storage]

    # candidate S/N of the brightest pulses within 1 % of the oracle's own FP64 row
    det = snd.Detector(p, WIDTHS, threshold=7.0)
    cands = det.run(y)
    for pu in sorted(spec.pulses, key=lambda q: -q.snr)[:3]:
        k_true = int(np.argmin(np.abs(spec.dms - pu.dm)))
        near = [c for c in cands if abs(c["k"] - k_true) <= 40 and abs(c["t"] - pu.t0) <= 200]
        assert near, (storage, pu)
        best = max(near, key=lambda c: c["snr"])
        assert abs(best["k"] - k_true) <= 1
        row = orc.snd_points(z, spec.freqs, d, np.full(p.n_out, best["k"], np.int32), np.arange(p.n_out),
                             mode="float", cluster=4, branching=4)
        o_snr, _, _, _ = orc.matched_filter(row[None, :], WIDTHS, integer_plane=False)
        rel = abs(best["snr"] - o_snr[0, best["t"]]) / o_snr[0, best["t"]]
        _say(f"storage {storage}: pulse DM {pu.dm:.1f} S/N {best['snr']:.3f} vs oracle {o_snr[0, best['t']]:.3f} "
             f"({rel:.2e})")
        assert rel <= 0.01
