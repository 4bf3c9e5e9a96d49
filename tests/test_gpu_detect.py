"""GPU parity of the boxcar S/N and candidate stage (snd_snr_plane / snd_detect) against the oracle.

Integer planes: row statistics, S/N plane, width index and candidate list are bit-exact
(both sides evaluate the same FP64 expressions on exact integer sums).  Float planes: S/N
within 1e-4 relative (the planes themselves differ at FP32 rounding), candidate S/N within 1 %.
"""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WIDTHS = [1, 2, 4, 8, 16, 32, 64]


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan_for(snd, ndm, n_out, mode):
    # an all-zero DM grid makes n_out = nsamp, so any plane shape can be fed to the detector
    return snd.Plan(synth.channel_freqs(4), np.zeros(ndm), 0.138e-3, n_out, mode=mode, branching=2)


def _cands_equal(got, want):
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert (g["k"], g["t"], g["widx"], g["npix"]) == (w["k"], w["t"], w["widx"], w["npix"])
        assert g["snr"] == w["snr"]


@pytest.mark.parametrize("mode,hi", [("graded", 255), ("graded", 9), ("binary", 1)])
@pytest.mark.parametrize("seed", [1, 2])
def test_integer_plane_bit_exact(snd, orc, mode, hi, seed):
    rng = synth.make_rng(seed)
    ndm, n = 37, 3000 + seed * 333
    if mode == "binary":
        plane = (rng.random((ndm, n)) < 0.02).astype(np.uint8)
        plane[10:14, 1000:1030] = 1
        plane[3, 200:260] = 1
        sigma_min, theta = 0.15, 6.0
    else:
        plane = rng.integers(0, hi + 1, (ndm, n)).astype(np.uint8)
        plane[20:23, 2000:2040] = hi
        sigma_min, theta = 0.0, 5.0
    plane[5] = 3 if mode == "graded" else 1  # constant row: sigma 0 (floored in binary mode)
    p = _plan_for(snd, ndm, n, mode)
    dev = torch.from_numpy(plane).cuda()
    for r, nmin in ((4, 10), (1, 1), (0, 1)):
        _say(f"integer detect mode={mode} hi={hi} seed={seed} r={r} n_min={nmin}")
        det = snd.Detector(p, WIDTHS, threshold=theta, sigma_min=sigma_min, closing_radius=r, n_min=nmin)
        snr, widx = det.snr_plane(dev)
        mu, sg = det.row_stats()
        o_snr, o_widx, o_mu, o_sg = orc.matched_filter(plane.astype(np.float64), WIDTHS, integer_plane=True,
                                                       sigma_min=sigma_min)
        assert np.array_equal(mu.cpu().numpy(), o_mu) and np.array_equal(sg.cpu().numpy(), o_sg)
        assert np.array_equal(snr.cpu().numpy(), o_snr.astype(np.float32))
        assert np.array_equal(widx.cpu().numpy().astype(np.int32), o_widx)
        got = det.run(dev)
        want = orc.candidates(o_snr, o_widx, theta, radius=r, n_min=nmin)
        _cands_equal(got, want)
        assert det.npixels == int((o_snr >= theta).sum())


@pytest.mark.parametrize("mode,hi,widths,theta,sigma_min", [
    ("graded", 255, WIDTHS, 5.0, 0.0),
    ("graded", 9, [1, 2, 8, 32, 128, 256], 5.0, 0.0),
    ("graded", 255, [1, 2, 4, 8, 16, 32, 64, 256], 4.5, 0.0),
    ("binary", 1, WIDTHS, 2.0, 0.15),        # bounds at or below zero: every cell is tested exactly
    ("graded", 255, [1, 3, 5, 7], 4.0, 0.0),  # odd widths: the general path
    ("graded", 255, [2, 4, 8], 4.0, 0.0),     # first width not 1: the general path
])
def test_integer_plane_multi_tile_bit_exact(snd, orc, mode, hi, widths, theta, sigma_min):
    """u8 planes several S/N tiles long with a ragged last tile: the paired 16-bit bound tests
    (widths 1 and even widths up to 256) and the general path give the oracle's S/N plane, cell
    count and candidates."""
    rng = synth.make_rng(hi + len(widths))
    ndm, n = 19, 3 * 4096 + 777
    if mode == "binary":
        plane = (rng.random((ndm, n)) < 0.03).astype(np.uint8)
        plane[4:7, 5000:5040] = 1
        plane[8] = 0  # an all-zero row: sigma floored
    else:
        plane = rng.integers(0, hi + 1, (ndm, n)).astype(np.uint8)
        plane[11:13, 8190:8300] = hi  # a pulse across a tile boundary
        plane[2, 4096 - 20:4096 + 20] = hi
    plane[5] = 1 if mode == "binary" else 3  # constant row
    p = _plan_for(snd, ndm, n, mode)
    dev = torch.from_numpy(plane).cuda()
    _say(f"multi-tile integer detect mode={mode} hi={hi} widths={widths} theta={theta}")
    det = snd.Detector(p, widths, threshold=theta, sigma_min=sigma_min, closing_radius=1, n_min=1)
    o_snr, o_widx, o_mu, o_sg = orc.matched_filter(plane.astype(np.float64), widths, integer_plane=True,
                                                   sigma_min=sigma_min)
    snr, widx = det.snr_plane(dev)
    assert np.array_equal(snr.cpu().numpy(), o_snr.astype(np.float32))
    assert np.array_equal(widx.cpu().numpy().astype(np.int32), o_widx)
    got = det.run(dev)
    want = orc.candidates(o_snr, o_widx, theta, radius=1, n_min=1)
    _cands_equal(got, want)
    assert det.npixels == int((o_snr >= theta).sum()) > 0


def test_float_plane_within_tolerance(snd, orc):
    rng = synth.make_rng(8)
    ndm, n = 24, 5000
    plane = rng.standard_normal((ndm, n)).astype(np.float32)
    plane[7:10, 3000:3008] += 4.0
    p = _plan_for(snd, ndm, n, "float")
    dev = torch.from_numpy(plane).cuda()
    det = snd.Detector(p, WIDTHS, threshold=6.0)
    snr, widx = det.snr_plane(dev)
    o_snr, o_widx, _, _ = orc.matched_filter(plane.astype(np.float64), WIDTHS, integer_plane=False)
    s = snr.cpu().numpy()
    assert np.max(np.abs(s - o_snr)) <= 1e-4 * max(1.0, np.abs(o_snr).max())
    got = det.run(dev)
    want = orc.candidates(o_snr, o_widx, 6.0, radius=4, n_min=10)
    assert [(g["k"], g["t"], g["npix"]) for g in got] == [(w["k"], w["t"], w["npix"]) for w in want]
    for g, w in zip(got, want):
        assert abs(g["snr"] - w["snr"]) <= 0.01 * abs(w["snr"])


def test_launch_collect_matches_run(snd, orc):
    # the asynchronous pair gives the candidates of snd_detect, with later device work queued
    # between launch and collect; a stage buffer too small for the cells falls back to run()
    rng = synth.make_rng(21)
    ndm, n = 40, 6000
    planes = []
    for j in range(3):
        pl = rng.standard_normal((ndm, n)).astype(np.float32)
        pl[5 + 9 * j:8 + 9 * j, 1000 + 700 * j:1012 + 700 * j] += 5.0
        planes.append(torch.from_numpy(pl).cuda())
    p = _plan_for(snd, ndm, n, "float")
    det = snd.Detector(p, WIDTHS, threshold=6.0)
    want = [det.run(pl) for pl in planes]
    npx = []
    for pl in planes:
        det.run(pl)
        npx.append(det.npixels)
    tickets = [det.launch(pl) for pl in planes]  # three launches queued before any collect
    got = [det.collect(t) for t in tickets]
    for g, w, m in zip(got, want, npx):
        assert g == w and len(w) >= 1
    o_snr, o_widx, _, _ = orc.matched_filter(planes[0].cpu().numpy().astype(np.float64), WIDTHS,
                                             integer_plane=False)
    assert [(c["k"], c["t"]) for c in got[0]] == [(c["k"], c["t"]) for c in orc.candidates(o_snr, o_widx, 6.0)]
    small = det.launch(planes[1], stage_cells=max(1, npx[1] // 2))
    assert det.collect(small) == want[1]


def test_capacity_error(snd):
    from paper_2606_15361_amd import SndError
    plane = np.full((8, 500), 1.0, np.float32)
    plane[:, ::2] = 5.0
    p = _plan_for(snd, 8, 500, "float")
    det = snd.Detector(p, [1], threshold=0.5, max_pixels=10)
    with pytest.raises(SndError):
        det.run(torch.from_numpy(plane).cuda())


def test_config1_pulse_recovery_all_modes(snd, orc):
    # Fig. 4 precedent: all three modes localise a bright injected pulse at the right DM/time.
    spec = synth.workload(1)
    z = spec.filterbank()
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    true_k = int(np.argmin(np.abs(spec.dms - spec.pulses[0].dm)))
    for mode, thr, kw, smin in (("float", None, {}, 0.0), ("graded", [1.0, 2.0, 3.0, 4.0], {}, 0.0),
                                ("binary", [2.0], dict(k_leaf=2, k_int=1), 0.2)):
        _say(f"config1 recovery mode={mode}")
        x = z if thr is None else orc.encode(z, thr)
        p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode=mode, branching=2, **kw)
        y = p.execute(torch.from_numpy(x).cuda())
        det = snd.Detector(p, WIDTHS, threshold=6.0, sigma_min=smin)
        cands = det.run(y)
        want_plane, _ = orc.snd_dedup(x, spec.freqs, d, mode=mode, cluster=4, branching=2, **kw)
        o_snr, o_widx, _, _ = orc.matched_filter(want_plane, WIDTHS, integer_plane=mode != "float", sigma_min=smin)
        want = orc.candidates(o_snr, o_widx, 6.0)
        if mode != "float":
            _cands_equal(cands, want)
        best = max(cands, key=lambda c: c["snr"])
        wbest = max(want, key=lambda c: c["snr"])
        assert abs(best["k"] - true_k) <= 1, (mode, best, true_k)
        # the peak boxcar [t, t + W) lies at the arrival time, up to the sweep residual of one
        # DM trial across the band (~2.4 DM x 14 samples per DM unit / 2) and the pulse width
        t0 = spec.pulses[0].t0
        assert best["t"] - 24 <= t0 < best["t"] + best["width"] + 24, (mode, best)
        assert abs(best["snr"] - wbest["snr"]) <= 0.01 * wbest["snr"]


def test_config2_pulse_recovery_float(snd, orc):
    # Full-size 1024-channel beam: each bright injected pulse is found within one DM trial,
    # and its S/N matches the oracle's S/N (own FP64 plane row, own statistics) within 1 %.
    spec = synth.workload(2)
    z = spec.filterbank()
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4)
    y = p.execute(torch.from_numpy(z).cuda())
    det = snd.Detector(p, WIDTHS, threshold=7.0)
    cands = det.run(y)
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    checked = 0
    for pu in sorted(spec.pulses, key=lambda q: -q.snr)[:3]:
        k_true = int(np.argmin(np.abs(spec.dms - pu.dm)))
        near = [c for c in cands if abs(c["k"] - k_true) <= 40 and abs(c["t"] - pu.t0) <= 200]
        assert near, (pu, k_true)
        best = max(near, key=lambda c: c["snr"])
        assert abs(best["k"] - k_true) <= 1, (pu, best, k_true)
        # the oracle's own row at the candidate DM, matched-filtered in FP64
        k = best["k"]
        ks = np.full(p.n_out, k, np.int32)
        row = orc.snd_points(z, spec.freqs, d, ks, np.arange(p.n_out), mode="float", cluster=4, branching=4)
        o_snr, o_widx, _, _ = orc.matched_filter(row[None, :], WIDTHS, integer_plane=False)
        assert abs(best["snr"] - o_snr[0, best["t"]]) <= 0.01 * o_snr[0, best["t"]]
        assert abs(float(o_snr[0].max()) - best["snr"]) <= 0.01 * best["snr"]
        checked += 1
    assert checked == 3
    # completeness under the paper's matching rule (|dDM| <= 10, |dt| <= 0.5 W_eff, greedy in
    # decreasing S/N): the library's host matching agrees with the oracle's on these candidates,
    # and the three brightest pulses are matched
    tms = spec.tsamp_s * 1e3
    pulses = [q for q in spec.pulses if 0 <= q.t0 < p.n_out]
    weff = snd.effective_width(spec.freqs, spec.tsamp_s, [q.dm for q in pulses], [q.width_ms for q in pulses])
    ct = [(c["t"] + 0.5 * (c["width"] - 1)) * tms for c in cands]
    match, n = snd.match_injections([c["dm"] for c in cands], ct, [c["snr"] for c in cands], [q.dm for q in pulses],
                                    [q.t0 * tms for q in pulses], weff)
    want, wn = orc.match_injections([dict(dm=c["dm"], t_ms=t, snr=c["snr"]) for c, t in zip(cands, ct)],
                                    [dict(dm=q.dm, t_ms=q.t0 * tms, w_eff_ms=w) for q, w in zip(pulses, weff)])
    assert list(match) == want and n == wn
    for j in sorted(range(len(pulses)), key=lambda j: -pulses[j].snr)[:3]:
        assert match[j] >= 0, (pulses[j], weff[j])
    _say(f"config2 float: {n} of {len(pulses)} injected pulses matched")


PAPER_WIDTHS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024]


@pytest.mark.parametrize("integer_plane", [True, False])
def test_dm_scaled_width_set(snd, orc, integer_plane):
    # the paper's width set: {1, 2, 4, 8} in every row, 16..1024 up to 0.1 x the row's sweep
    f = synth.channel_freqs(1024)
    dms = np.array([0.0, 10.0, 25.0, 50.0, 100.0, 200.0, 400.0, 2000.0])
    n = 5000
    dmax = int(orc.delays(f, dms, 0.138e-3).max())
    p = snd.Plan(f, dms, 0.138e-3, dmax + n, mode="graded" if integer_plane else "float", branching=4)
    assert p.n_out == n
    rng = synth.make_rng(77)
    if integer_plane:
        plane = rng.integers(0, 6, (dms.size, n)).astype(np.uint8)
        plane[6, 1000:1400] = 5  # a wide pulse: only rows with the wide widths catch it whole
        plane[2, 3000:3030] = 5
    else:
        plane = rng.standard_normal((dms.size, n)).astype(np.float32)
        plane[6, 1000:1400] += 1.0
        plane[2, 3000:3030] += 3.0
    counts = orc.dm_width_counts(f, dms, 0.138e-3, PAPER_WIDTHS, 4, 0.1)
    assert list(counts) == [4, 4, 6, 7, 8, 9, 10, 11]
    det = snd.Detector(p, PAPER_WIDTHS, threshold=6.0, n_base_widths=4, width_alpha=0.1)
    dev = torch.from_numpy(plane).cuda()
    snr, widx = det.snr_plane(dev)
    o_snr, o_widx, _, _ = orc.matched_filter(plane.astype(np.float64), PAPER_WIDTHS, integer_plane=integer_plane,
                                             row_nw=counts)
    w = widx.cpu().numpy().astype(np.int32)
    if integer_plane:
        assert np.array_equal(snr.cpu().numpy(), o_snr.astype(np.float32)) and np.array_equal(w, o_widx)
    else:
        assert np.max(np.abs(snr.cpu().numpy() - o_snr)) <= 1e-4 * max(1.0, np.abs(o_snr).max())
    assert np.all(w < counts[:, None])  # no row uses a width outside its set
    got = det.run(dev)
    want = orc.candidates(o_snr, o_widx, 6.0, radius=4, n_min=10)
    assert [(c["k"], c["t"], c["npix"]) for c in got] == [(c["k"], c["t"], c["npix"]) for c in want]
    assert any(c["k"] == 6 for c in got)


@pytest.mark.parametrize("mode,hi,cap", [("graded", 255, 255), ("graded", 9, 255), ("binary", 1, 255),
                                         ("graded", 3000, 4000)])
def test_mad_sigma_integer_planes_bit_exact(snd, orc, mode, hi, cap):
    # sigma from the median absolute deviation: exact medians on both sides, so the row
    # statistics, the S/N plane and the candidates are bit-exact
    rng = synth.make_rng(11 + hi)
    ndm, n = 29, 4001 + hi % 7
    dt = np.uint16 if cap > 255 else np.uint8
    if mode == "binary":
        plane = (rng.random((ndm, n)) < 0.03).astype(dt)
        plane[6:9, 1500:1540] = 1
        smin, theta = 0.2, 6.0
    else:
        plane = rng.integers(0, hi + 1, (ndm, n)).astype(dt)
        plane[12:15, 2500:2530] = hi
        plane[20, :80] = hi  # a burst that inflates the standard deviation, not the MAD
        smin, theta = 0.0, 5.0
    plane[4] = 2 if mode == "graded" else 0  # constant row: MAD 0
    p = snd.Plan(synth.channel_freqs(4), np.zeros(ndm), 0.138e-3, n, mode=mode, branching=2, cap=cap)
    _say(f"MAD detect mode={mode} hi={hi} cap={cap} plane dtype={p.info['out_dtype']}")
    dev = torch.from_numpy(plane).cuda()
    det = snd.Detector(p, WIDTHS, threshold=theta, sigma_min=smin, sigma="mad")
    snr, widx = det.snr_plane(dev)
    mu, sg = det.row_stats()
    o_sig = orc.mad_sigma(plane)
    o_snr, o_widx, o_mu, o_sg = orc.matched_filter(plane.astype(np.float64), WIDTHS, integer_plane=True,
                                                   sigma_min=smin, sigma_rows=o_sig)
    assert np.array_equal(mu.cpu().numpy(), o_mu) and np.array_equal(sg.cpu().numpy(), o_sg)
    assert np.array_equal(snr.cpu().numpy(), o_snr.astype(np.float32))
    assert np.array_equal(widx.cpu().numpy().astype(np.int32), o_widx)
    _cands_equal(det.run(dev), orc.candidates(o_snr, o_widx, theta))


def test_mad_sigma_float_plane(snd, orc):
    # float planes: the deviation is one FP32 subtraction on both sides, so sigma is bit-exact;
    # the S/N is within the float tolerance of the oracle's FP64 evaluation
    rng = synth.make_rng(17)
    ndm, n = 21, 6003
    plane = (rng.standard_normal((ndm, n)) * rng.uniform(0.5, 30.0, (ndm, 1)) + rng.uniform(-5, 5, (ndm, 1)))
    plane = plane.astype(np.float32)
    plane[9:11, 4000:4010] += 40.0
    plane[15, :150] += 500.0  # burst
    plane[3] = 0.0
    plane[3, ::2] = -0.0  # signed zeros: MAD 0, sigma 0, S/N 0
    plane[18, :] = np.float32(1e-3)
    plane[18, ::3] = np.float32(-2e30)  # a third of the row far below: the median stays 1e-3
    p = _plan_for(snd, ndm, n, "float")
    dev = torch.from_numpy(plane).cuda()
    det = snd.Detector(p, WIDTHS, threshold=6.0, sigma="mad")
    snr, widx = det.snr_plane(dev)
    mu, sg = det.row_stats()
    o_sig = orc.mad_sigma(plane)
    assert np.array_equal(sg.cpu().numpy(), o_sig)
    assert o_sig[3] == 0.0 and o_sig[18] == 0.0  # rows 3 and 18: MAD 0, so S/N 0 throughout
    o_snr, o_widx, _, _ = orc.matched_filter(plane.astype(np.float64), WIDTHS, integer_plane=False, sigma_rows=o_sig)
    s = snr.cpu().numpy()
    assert np.max(np.abs(s - o_snr)) <= 1e-4 * max(1.0, np.abs(o_snr).max())


@pytest.mark.parametrize("mode,hi", [("graded", 255), ("graded", 9), ("binary", 1), ("float", 0)])
def test_label_on_device_matches_host_and_oracle(snd, orc, mode, hi):
    # closing and labelling on the device: the same candidates as the host path and the oracle
    rng = synth.make_rng(23 + hi)
    ndm, n = 41, 5003
    if mode == "binary":
        plane = (rng.random((ndm, n)) < 0.02).astype(np.uint8)
        plane[10:14, 1000:1030] = 1
        plane[0:3, 0:40] = 1            # islands on the plane's edges
        plane[ndm - 2:, n - 30:] = 1
        smin, theta = 0.15, 6.0
    elif mode == "graded":
        plane = rng.integers(0, hi + 1, (ndm, n)).astype(np.uint8)
        plane[20:23, 2000:2040] = hi
        plane[0, :50] = hi
        smin, theta = 0.0, 5.0
    else:
        plane = rng.standard_normal((ndm, n)).astype(np.float32)
        plane[7:10, 3000:3008] += 4.0
        plane[ndm - 1, n - 20:] += 5.0
        smin, theta = 0.0, 4.0
    p = _plan_for(snd, ndm, n, mode)
    dev = torch.from_numpy(plane).cuda()
    integer = mode != "float"
    o_snr, o_widx, _, _ = orc.matched_filter(plane.astype(np.float64), WIDTHS, integer_plane=integer, sigma_min=smin)
    for r, nmin in ((4, 10), (1, 1), (0, 1), (6, 3)):
        _say(f"device labelling mode={mode} hi={hi} r={r} n_min={nmin}")
        host = snd.Detector(p, WIDTHS, threshold=theta, sigma_min=smin, closing_radius=r, n_min=nmin).run(dev)
        devc = snd.Detector(p, WIDTHS, threshold=theta, sigma_min=smin, closing_radius=r, n_min=nmin,
                            label="device").run(dev)
        assert [(c["k"], c["t"], c["widx"], c["npix"], c["snr"]) for c in devc] == \
               [(c["k"], c["t"], c["widx"], c["npix"], c["snr"]) for c in host]
        if integer:
            _cands_equal(devc, orc.candidates(o_snr, o_widx, theta, radius=r, n_min=nmin))
    # more closed runs than the run tables hold: a capacity error, not a fault
    det = snd.Detector(p, WIDTHS, threshold=theta, sigma_min=smin, closing_radius=4, n_min=1, label="device",
                       max_pixels=int((o_snr >= theta).sum()))
    try:
        det.run(dev)
    except snd.SndError as e:
        assert e.status == -5


def test_label_on_device_full_size_float(snd, orc):
    spec = synth.workload(2)
    z = spec.filterbank()
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4)
    y = p.execute(torch.from_numpy(z).cuda())
    host = snd.Detector(p, WIDTHS, threshold=7.0).run(y)
    devc = snd.Detector(p, WIDTHS, threshold=7.0, label="device").run(y)
    _say(f"full-size float: {len(host)} candidates on the host, {len(devc)} on the device")
    assert [(c["k"], c["t"], c["widx"], c["npix"], c["snr"]) for c in devc] == \
           [(c["k"], c["t"], c["widx"], c["npix"], c["snr"]) for c in host]


def test_detect_edge_cases_both_labelling_paths(snd, orc):
    # no cell above threshold, a single cell, and single-sample rows (MAD of one value is 0)
    ndm, n = 9, 700
    p = _plan_for(snd, ndm, n, "graded")
    zero = torch.zeros((ndm, n), dtype=torch.uint8, device="cuda")
    for where in ("host", "device"):
        det = snd.Detector(p, WIDTHS, threshold=5.0, label=where)
        assert det.run(zero) == [] and det.npixels == 0
    one = np.zeros((ndm, n), np.uint8)
    one[4, 350] = 200
    dev = torch.from_numpy(one).cuda()
    o_snr, o_widx, _, _ = orc.matched_filter(one.astype(np.float64), WIDTHS, integer_plane=True)
    want = orc.candidates(o_snr, o_widx, 5.0, radius=4, n_min=1)
    for where in ("host", "device"):
        _cands_equal(snd.Detector(p, WIDTHS, threshold=5.0, n_min=1, label=where).run(dev), want)
    p1 = _plan_for(snd, 3, 1, "graded")
    d1 = snd.Detector(p1, [1], threshold=5.0, sigma="mad")
    d1.run(torch.tensor([[3], [0], [9]], dtype=torch.uint8, device="cuda"))
    mu, sg = d1.row_stats()
    assert np.array_equal(sg.cpu().numpy(), [0.0, 0.0, 0.0]) and np.array_equal(mu.cpu().numpy(), [3.0, 0.0, 9.0])


@pytest.mark.parametrize("scaled", [False, True])
def test_batched_detection_equals_per_beam(snd, orc, scaled):
    """snd_detect_batch_*: planes of four beams with different plans (graded u8, float f32,
    binary u8, graded u16; different DM grids and lengths) detected in shared grids give each
    beam the candidates and cell counts of its own detection."""
    beams = [("graded", dict(cap=255), 64, 120, 60.0, 9000), ("float", {}, 96, 200, 80.0, 12000),
             ("binary", dict(k_leaf=2, k_int=1), 64, 77, 40.0, 7000), ("graded", dict(cap=4095), 128, 150, 100.0, 8000)]
    rng = synth.make_rng(404)
    plans, planes = [], []
    for mode, kw, nchan, ndm, dmax, nsamp in beams:
        f = synth.channel_freqs(nchan)
        dms = np.sort(rng.uniform(0, dmax, ndm))
        z = synth.noise_filterbank(rng, nchan, nsamp)
        synth.inject_pulses(z, f, 0.138e-3, [synth.Pulse(dm=dmax * 0.6, t0=nsamp / 3.0, width_ms=2.0, snr=60.0)])
        x = z if mode == "float" else orc.encode(z, [1.0, 2.0, 3.0, 4.0] if mode == "graded" else [2.0])
        p = snd.Plan(f, dms, 0.138e-3, nsamp, mode=mode, branching=4, **kw)
        planes.append(p.execute(torch.from_numpy(np.ascontiguousarray(x)).cuda()))
        plans.append(p)
    torch.cuda.synchronize()
    kw = dict(widths=(1, 2, 4, 8, 16, 32), threshold=6.0, sigma_min=0.15, n_min=3)
    if scaled:
        kw.update(n_base_widths=2, width_alpha=0.1)
    bd = snd.BatchDetector(**kw)
    got = bd.collect(bd.launch(plans, planes, stage_cells=1 << 16))
    total = 0
    for i, (p, y) in enumerate(zip(plans, planes)):
        d = snd.Detector(p, **kw)
        want = d.run(y)
        assert got[i] == want, i
        assert bd.npixels[i] == d.npixels, i
        total += len(want)
    assert total > 0
