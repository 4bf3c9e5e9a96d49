"""Pins for the oracle's SND tree: brute force, closed forms, paper values, hand-worked cases."""

import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_case(seed, nchan, ndm, nsamp, dmax=None, shuffle=False):
    # the 16 MHz band at 408 MHz sweeps ~14 samples per unit DM: keep the sweep < nsamp / 2
    dmax = nsamp / 30.0 if dmax is None else dmax
    rng = synth.make_rng(seed)
    f = synth.channel_freqs(nchan)
    dms = rng.uniform(0.0, dmax, size=ndm)
    if not shuffle:
        dms = np.sort(dms)
    dms[min(1, ndm - 1)] = dms[0]  # a duplicate trial
    return rng, f, dms


@pytest.mark.parametrize("nchan,C,B", [(64, 4, 2), (37, 3, 3), (24, 5, 4), (16, 1, 2), (9, 4, 8), (3, 4, 2)])
def test_linear_modes_equal_bruteforce(orc, nchan, C, B):
    # Methods Eq. y_d: direct dedispersion; Results: float SND equals brute force. With
    # integer-valued inputs every FP64 sum is exact, so equality is exact.
    rng, f, dms = _random_case(nchan * 7 + B, nchan, 23, 700, shuffle=True)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, nchan, 700, 5)
    bf = orc.bruteforce(x, d, mode="float")
    for fn in (orc.snd_recursive, lambda *a, **k: orc.snd_dedup(*a, **k)[0]):
        y = fn(x, f, d, mode="float", cluster=C, branching=B)
        assert np.array_equal(y, bf)
        yg = fn(x, f, d, mode="graded", cluster=C, branching=B, cap=65535)
        assert np.array_equal(yg, bf)


def test_float_noninteger_matches_bruteforce(orc):
    rng, f, dms = _random_case(5, 48, 17, 900)
    d = orc.delays(f, dms, 0.138e-3)
    z = synth.noise_filterbank(rng, 48, 900)
    bf = orc.bruteforce(z, d, mode="float")
    y, _ = orc.snd_dedup(z, f, d, mode="float", cluster=4, branching=4)
    assert np.max(np.abs(y - bf)) <= 1e-12 * max(1.0, np.max(np.abs(bf)))
    yn, _ = orc.snd_dedup(z, f, d, mode="float", cluster=4, branching=4, root_norm=True)
    assert np.allclose(yn, bf / math.sqrt(48), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("cap", [1, 3, 15, 255])
def test_graded_is_capped_bruteforce(orc, cap):
    # Mode B clips every node to [0, N] (Methods, tree activation modes).  With non-negative
    # inputs a node that clips hands N to its parent, whose sum is then >= N as well, so
    # the root equals min(direct sum, N) whatever the tree shape.
    rng, f, dms = _random_case(cap, 40, 19, 800)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, 40, 800, 4)
    target = np.minimum(orc.bruteforce(x, d, mode="graded"), cap)
    for B in (2, 3, 8):
        y, _ = orc.snd_dedup(x, f, d, mode="graded", cluster=4, branching=B, cap=cap)
        assert np.array_equal(y, target)
    assert np.array_equal(orc.snd_recursive(x, f, d, mode="graded", cluster=3, branching=2, cap=cap), target)


def test_branching_invariance_float(orc):
    # Results / Methods: DM-time planes are numerically invariant under B in {2,4,8,16}.
    rng, f, dms = _random_case(11, 64, 31, 1200)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, 64, 1200, 3).astype(np.float32)
    ys = [orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=B)[0] for B in (2, 4, 8, 16)]
    for y in ys[1:]:
        assert np.array_equal(y, ys[0])


def test_dm_zero_row_is_channel_sum_and_conservation(orc):
    rng = synth.make_rng(3)
    f = synth.channel_freqs(32)
    dms = np.array([0.0, 10.0, 20.0, 30.0])
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, 32, 1000, 7)
    y, _ = orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=2)
    nout = y.shape[1]
    assert np.array_equal(y[0], x[:, :nout].sum(axis=0).astype(np.float64))
    for k in range(len(dms)):
        total = sum(int(x[c, d[k, c]:d[k, c] + nout].sum()) for c in range(32))
        assert y[k].sum() == total


def test_binary_special_cases_reduce_to_bruteforce(orc):
    rng, f, dms = _random_case(21, 64, 15, 900)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_spikes(rng, 64, 900, 0.3)
    bf = orc.bruteforce(x, d, mode="binary")
    y1, _ = orc.snd_dedup(x, f, d, mode="binary", cluster=4, branching=4, k_leaf=1, k_int=1)
    assert np.array_equal(y1, (bf >= 1).astype(float))
    # 64 = 4 * 4^3: with K equal to every node's fan-in the root fires only when all fire.
    xd = synth.random_spikes(rng, 64, 900, 0.97)
    bfd = orc.bruteforce(xd, d, mode="binary")
    yall, _ = orc.snd_dedup(xd, f, d, mode="binary", cluster=4, branching=4, k_leaf=4, k_int=4)
    assert np.array_equal(yall, (bfd == 64).astype(float))
    assert yall.sum() > 0
    # non-zero input samples count as one spike
    y3, _ = orc.snd_dedup(x * 3, f, d, mode="binary", cluster=4, branching=4, k_leaf=2, k_int=2)
    y4, _ = orc.snd_dedup(x, f, d, mode="binary", cluster=4, branching=4, k_leaf=2, k_int=2)
    assert np.array_equal(y3, y4)


def test_golden_binary_hand_worked(orc):
    g = json.load(open(os.path.join(GOLDEN, "binary_ragged_5ch.json")))
    x = np.array(g["x"], dtype=np.uint8)
    d = np.array(g["delays"], dtype=np.int32)
    for case in g["cases"]:
        kw = dict(mode="binary", cluster=2, branching=2, k_leaf=case["k_leaf"], k_int=case["k_int"])
        y = orc.snd_recursive(x, g["freqs_mhz"], d, **kw)
        assert y.astype(int).tolist() == case["expected"]
        y2, counts = orc.snd_dedup(x, g["freqs_mhz"], d, **kw)
        assert y2.astype(int).tolist() == case["expected"]
        assert [c[0] for c in counts] == [3, 2, 1]


def test_dedup_equals_recursion_all_modes(orc):
    rng, f, dms = _random_case(33, 45, 40, 1500, shuffle=True)
    d = orc.delays(f, dms, 0.138e-3)
    xs = synth.random_spikes(rng, 45, 1500, 0.2)
    xl = synth.random_levels(rng, 45, 1500, 9)
    for mode, x, kw in (("binary", xs, dict(k_leaf=2, k_int=1)), ("binary", xs, dict(k_leaf=1, k_int=2)),
                        ("graded", xl, dict(cap=20)), ("float", xl, {})):
        for B in (2, 3):
            a = orc.snd_recursive(x, f, d, mode=mode, cluster=3, branching=B, **kw)
            b, counts = orc.snd_dedup(x, f, d, mode=mode, cluster=3, branching=B, **kw)
            assert np.array_equal(a, b)
            assert all(n <= len(dms) * 16 for n, _ in counts)
            assert counts[-1][0] <= len(dms)


@pytest.mark.parametrize("nchan,C,B", [(37, 3, 3), (24, 5, 4), (9, 4, 8), (64, 4, 2)])
def test_points_pinned_to_bruteforce_and_dedup(orc, nchan, C, B):
    # orc_snd_points (the checker used on full-size planes) at sampled (k, t) of ragged shapes:
    # float and uncapped graded equal brute force, capped graded equals min(brute force, N),
    # binary with K = 1 everywhere equals 1[brute force >= 1], and binary with a real quorum
    # equals the shared-pattern tree (a separate computation) and the whole-plane recursion.
    rng, f, dms = _random_case(nchan * 13 + B, nchan, 21, 800, shuffle=True)
    d = orc.delays(f, dms, 0.138e-3)
    nout = 800 - int(d.max())
    ks = rng.integers(0, len(dms), 300)
    ts = rng.integers(0, nout, 300)
    ks[:3], ts[:3] = [0, len(dms) - 1, 1], [0, nout - 1, nout - 1]  # the plane's corners
    xl = synth.random_levels(rng, nchan, 800, 6)
    xs = synth.random_spikes(rng, nchan, 800, 0.25)
    bf = orc.bruteforce(xl, d, mode="float")
    bfs = orc.bruteforce(xs, d, mode="binary")
    kw = dict(cluster=C, branching=B)
    assert np.array_equal(orc.snd_points(xl, f, d, ks, ts, mode="float", **kw), bf[ks, ts])
    assert np.array_equal(orc.snd_points(xl, f, d, ks, ts, mode="graded", cap=65535, **kw), bf[ks, ts])
    assert np.array_equal(orc.snd_points(xl, f, d, ks, ts, mode="graded", cap=7, **kw), np.minimum(bf[ks, ts], 7))
    one = orc.snd_points(xs, f, d, ks, ts, mode="binary", k_leaf=1, k_int=1, **kw)
    assert np.array_equal(one, (bfs[ks, ts] >= 1).astype(float))
    for kl, ki in ((2, 1), (2, 2), (1, 2)):
        got = orc.snd_points(xs, f, d, ks, ts, mode="binary", k_leaf=kl, k_int=ki, **kw)
        plane, _ = orc.snd_dedup(xs, f, d, mode="binary", k_leaf=kl, k_int=ki, **kw)
        assert np.array_equal(got, plane[ks, ts])
        rec = orc.snd_recursive(xs, f, d, mode="binary", k_leaf=kl, k_int=ki, **kw)
        assert np.array_equal(got, rec[ks, ts])
    with pytest.raises(ValueError):
        orc.snd_points(xl, f, d, [0], [nout], mode="float", **kw)  # past the valid window


def test_encoder_threshold_is_strict(orc):
    # Methods, "Input encoding": a sample fires when it exceeds the threshold, x = 1[z > theta].
    # A sample exactly at a threshold does not count; the next float above it does.
    thr = [np.float32(0.75), np.float32(1.5), np.float32(2.0)]
    for t in thr:
        up = np.nextafter(t, np.float32(np.inf))
        dn = np.nextafter(t, np.float32(-np.inf))
        z = np.array([[dn, t, up]], dtype=np.float32)
        assert orc.encode(z, [t]).tolist() == [[0, 0, 1]]
    # multi-level: the level is the number of thresholds strictly exceeded
    lv = [1.0, 2.0, 3.0, 4.0]
    z = np.array([[0.0, 1.0, np.nextafter(np.float32(1.0), np.float32(2.0)), 2.0, 3.0, 3.5, 4.0, 4.0001, -5.0]],
                 dtype=np.float32)
    assert orc.encode(z, lv).tolist() == [[0, 0, 1, 1, 2, 3, 3, 4, 0]]


def test_cascade_table1(orc):
    # Table 1: NC tree (C = 4, B = 8, B_root = 4), p0 = p(1.5 sigma); root noise fire rates
    # and the predicted worst-case S/N sqrt((1-p)/p) (Eq. snr_A with p_sig = 1, W = 1).
    p0 = orc.fire_probability(1.5)
    fan = [4, 8, 8, 4]
    table = {(1, 3): 0.24, (2, 2): 2.2e-4, (3, 1): 0.25, (3, 2): 7.7e-15, (4, 1): 5.1e-3}
    for (kl, ki), p in table.items():
        got = orc.cascade(p0, fan, kl, ki)[-1]
        assert abs(got - p) / p < 0.05, (kl, ki, got)
    assert orc.cascade(p0, fan, 2, 1)[-1] > 0.99
    assert orc.cascade(p0, fan, 1, 1)[-1] > 0.999
    assert orc.cascade(p0, fan, 2, 3)[-1] < 1e-15
    pred = {(1, 3): 1.8, (2, 2): 67.5, (3, 1): 1.7, (4, 1): 14.0}
    for (kl, ki), s in pred.items():
        p = orc.cascade(p0, fan, kl, ki)[-1]
        assert abs(orc.binary_snr(1, 1.0, p) - s) / s < 0.03


def test_encoder_fire_rates(orc):
    # Results: p(1.5 sigma) = 6.68e-2; p(2 sigma) = 2.275e-2; graded noise baseline
    # 1024 * p(0.75 sigma) ~ 232 counts.
    assert abs(orc.fire_probability(1.5) - 6.68e-2) < 5e-5
    assert abs(orc.fire_probability(2.0) - 2.275e-2) < 5e-6
    assert abs(1024 * orc.fire_probability(0.75) - 232) < 0.5
    z = synth.noise_filterbank(synth.make_rng(9), 64, 20000)
    x = orc.encode(z, [1.5])
    p = orc.fire_probability(1.5)
    n = x.size
    assert abs(x.mean() - p) < 4 * math.sqrt(p * (1 - p) / n)
    lv = orc.encode(z, [1.0, 2.0, 3.0, 4.0])
    assert lv.max() <= 4
    assert abs((lv >= 2).mean() - orc.fire_probability(2.0)) < 4 * math.sqrt(0.0228 / n)


def test_binary_tree_noise_follows_cascade(orc):
    # Eq. cascade: on i.i.d. Bernoulli(p0) spikes the children of a node cover disjoint
    # channels, so the root fire rate equals the cascade prediction.
    rng = synth.make_rng(17)
    nchan, nsamp = 64, 60000
    f = synth.channel_freqs(nchan)
    d = orc.delays(f, [0.0, 100.0], 0.138e-3)
    x = synth.random_spikes(rng, nchan, nsamp + int(d.max()), 0.3)
    for kl, ki in ((2, 2), (1, 3), (3, 1)):
        y, _ = orc.snd_dedup(x, f, d, mode="binary", cluster=4, branching=4, k_leaf=kl, k_int=ki)
        p = orc.cascade(0.3, [4, 4, 4], kl, ki)[-1]  # 64 ch: 16 leaves -> 4 -> root
        n = y.shape[1]
        for k in range(2):
            assert abs(y[k].mean() - p) < 4.5 * math.sqrt(p * (1 - p) / n) + 1e-12, (kl, ki, y[k].mean(), p)


def test_graded_noise_baseline(orc):
    # Results: the graded root mean on encoded noise is N_f * p(theta): ~232 at 0.75 sigma.
    rng = synth.make_rng(23)
    f = synth.channel_freqs(1024)
    d = orc.delays(f, [0.0, 300.0], 0.138e-3)
    z = synth.noise_filterbank(rng, 1024, int(d.max()) + 3000)
    x = orc.encode(z, [0.75])
    y, _ = orc.snd_dedup(x, f, d, mode="graded", cluster=4, branching=8, cap=65535)
    m = y.mean()
    assert abs(m - 1024 * orc.fire_probability(0.75)) < 1.5


def test_oracle_under_host_sanitizers(tmp_path):
    """The oracle's C compiled with AddressSanitizer and UndefinedBehaviorSanitizer (host gcc)
    and run on a small ragged case in every mode: no memory error, no undefined behaviour, and
    the shared-pattern tree equals the per-DM recursion."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host gcc")
    exe = str(tmp_path / "sanitize_oracle")
    src = os.path.join(os.path.dirname(__file__), "sanitize_oracle.c")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-sanitize-recover=all"]
    san = ["-fsanitize=" + s for s in ("address", "undefined")]
    subprocess.run([gcc] + flags + san + [src, "-o", exe, "-lm"], check=True, capture_output=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized oracle run ok" in r.stdout
