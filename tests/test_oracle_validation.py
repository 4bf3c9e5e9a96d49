"""Pins for the oracle's validation helpers (Methods, "Validation methodology"): effective
widths of injected pulses and the greedy one-to-one matching of candidates to injections."""

import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_effective_width_smearing_term_meets_the_printed_band_edges(orc):
    # with zero intrinsic width and the sampling term removed in quadrature, what remains is
    # the smearing inside one channel; Eq. scrunch puts S dt = that smearing at the printed
    # Northern Cross band edges 289 / 578 / 1157 / 2313 (S = 2, 4, 8, 16)
    f = synth.channel_freqs(1024)
    dt = 0.138
    edges = [289.0, 578.0, 1157.0, 2313.0]
    w = orc.effective_width(f, dt * 1e-3, edges, [0.0] * 4)
    tau = np.sqrt(w * w - dt * dt)
    for t, s in zip(tau, (2, 4, 8, 16)):
        assert t == pytest.approx(s * dt, rel=2e-3)


def test_effective_width_special_cases(orc):
    f = synth.channel_freqs(1024)
    # DM 0: only the intrinsic width and the sampling time
    assert orc.effective_width(f, 0.138e-3, [0.0], [0.0])[0] == pytest.approx(0.138, rel=1e-15)
    assert orc.effective_width(f, 0.138e-3, [0.0], [2.0])[0] == pytest.approx(math.hypot(2.0, 0.138), rel=1e-15)
    # a 3-4-5 triangle: choose the DM whose smearing is 4 ms and a negligible sampling time
    fc = 0.5 * (f.max() + f.min())
    df = (f.max() - f.min()) / (f.size - 1)
    d4 = 4.0 * fc ** 3 / (4.148808e6 * df)
    assert orc.effective_width(f, 1e-12, [d4], [3.0])[0] == pytest.approx(5.0, rel=1e-12)
    # never below any of its terms, and growing with DM
    w = orc.effective_width(f, 0.138e-3, [10.0, 500.0, 3000.0], [0.5, 0.5, 0.5])
    assert np.all(w >= 0.5) and np.all(np.diff(w) > 0)


def test_match_injections_hand_worked(orc):
    g = json.load(open(os.path.join(GOLDEN, "injection_match.json")))
    for case in g["cases"]:
        cands = [dict(dm=c[0], t_ms=c[1], snr=c[2]) for c in case["candidates"]]
        injs = [dict(dm=q[0], t_ms=q[1], w_eff_ms=q[2]) for q in case["injections"]]
        match, n = orc.match_injections(cands, injs, g["dm_tol"], g["t_frac"])
        assert match == case["expected"], case["name"]
        assert n == sum(1 for m in case["expected"] if m >= 0)


def test_match_injections_all_admissible_and_none_admissible(orc):
    rng = synth.make_rng(41)
    for nc, ni in ((0, 3), (3, 0), (5, 3), (3, 5), (7, 7)):
        cands = [dict(dm=float(rng.uniform(0, 5)), t_ms=float(rng.uniform(0, 1)), snr=float(rng.uniform(6, 30)))
                 for _ in range(nc)]
        injs = [dict(dm=float(rng.uniform(0, 5)), t_ms=float(rng.uniform(0, 1)), w_eff_ms=10.0) for _ in range(ni)]
        match, n = orc.match_injections(cands, injs, dm_tol=10.0, t_frac=0.5)
        # every pair admissible: one to one, so min(n_cand, n_inj) injections are matched, each
        # by a different candidate
        assert n == min(nc, ni)
        used = [m for m in match if m >= 0]
        assert len(used) == len(set(used))
        # every pair far apart: nothing matches
        far = [dict(q, dm=q["dm"] + 100.0) for q in injs]
        assert orc.match_injections(cands, far, dm_tol=10.0, t_frac=0.5) == ([-1] * ni, 0)


def test_match_injections_reduces_to_linear_assignment(orc):
    # injections far apart, each candidate admissible for at most one of them and at most one
    # candidate per injection: greedy matching and an optimal assignment (scipy) find the same
    # pairs
    from scipy.optimize import linear_sum_assignment
    rng = synth.make_rng(43)
    injs = [dict(dm=100.0 * (k + 1), t_ms=1000.0 * (k + 1), w_eff_ms=2.0) for k in range(12)]
    cands = []
    for k in rng.permutation(12)[:8]:
        cands.append(dict(dm=injs[k]["dm"] + float(rng.uniform(-5, 5)), t_ms=injs[k]["t_ms"] + float(rng.uniform(-0.9, 0.9)),
                          snr=float(rng.uniform(6, 40))))
    cands.append(dict(dm=50.0, t_ms=5.0, snr=99.0))  # admissible for none
    match, n = orc.match_injections(cands, injs)
    cost = np.ones((len(cands), len(injs)))
    for i, c in enumerate(cands):
        for j, q in enumerate(injs):
            if abs(c["dm"] - q["dm"]) <= 10.0 and abs(c["t_ms"] - q["t_ms"]) <= 1.0:
                cost[i, j] = 0.0
    r, col = linear_sum_assignment(cost)
    want = {int(j): int(i) for i, j in zip(r, col) if cost[i, j] == 0.0}
    assert n == len(want) == 8
    assert {j: m for j, m in enumerate(match) if m >= 0} == want
