"""The serving loop (serve.Server) through the C ABI: budgeted admission, device-side encoding,
batched pushes and per-chunk detection find an injected pulse at its DM, and the batched and
per-beam forms of the server agree."""

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


def test_server_admission_detection_and_forms_agree(snd):
    from paper_2606_15361_amd import serve
    spec = synth.workload(1)
    T = 2048
    pg = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=T)
    pf = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="float", branching=2, chunk=T, in_dtype="bf16",
                  node_dtype="bf16")
    kinds = {"graded": (pg, [1.0, 2.0, 3.0, 4.0]), "bf16": (pf, None)}
    budget = 2 * snd.admission_bytes(pg) + snd.admission_bytes(pf)
    total = 6 * T
    z = synth.noise_filterbank(synth.make_rng(5), 64, total)
    # a bright pulse at DM 150 whose sweep lies inside the fifth chunk's output window
    synth.inject_pulses(z, spec.freqs, spec.tsamp_s, [synth.Pulse(dm=150.0, t0=4 * T + 900.0 - pg.max_delay,
                                                                  width_ms=1.0, snr=40.0)])
    zt = torch.from_numpy(z).cuda()
    results = {}
    for batched in (True, False):
        srv = serve.Server(kinds, budget, batched=batched, n_min=3, device="cuda")
        assert srv.admit(0, "graded") and srv.admit(1, "bf16") and srv.admit(2, "graded")
        assert not srv.admit(3, "bf16")  # over the history budget
        got = {}
        for i in range(6):
            res = srv.process([(b, i, zt[:, i * T:(i + 1) * T]) for b in (0, 1, 2)])
            torch.cuda.synchronize()
            for b, idx, t0, n, cands in res:
                got[(b, idx)] = (t0, n, None if cands is None else [(c["k"], c["t"], round(c["snr"], 6)) for c in cands],
                                 srv.out[b][:, :n].float().cpu().numpy().copy())
        results[batched] = got
    for key, (t0, n, cands, y) in results[True].items():
        t0b, nb, cb, yb = results[False][key]
        assert (t0, n, cands) == (t0b, nb, cb) and np.array_equal(y, yb), key
    k_true = int(np.argmin(np.abs(spec.dms - 150.0)))
    hits = [(b, idx, c) for (b, idx), (t0, n, cands, _) in results[True].items() if cands for c in cands]
    print("candidates (beam, chunk, (k, t, snr)):", hits, "true k", k_true)
    assert {b for b, _, _ in hits} == {0, 1, 2}
    for b in (0, 1, 2):  # the brightest candidate of each beam is the pulse, in the fifth chunk
        bb, idx, c = max((h for h in hits if h[0] == b), key=lambda h: h[2][2])
        assert idx == 4 and abs(c[0] - k_true) <= 2 and abs(c[1] - 900) <= 40, (b, idx, c)
