"""GPU tests of the streaming form (snd_stream_* through the C ABI): chunked output equals the
oracle (and the plain execute) on the concatenated input for any chunk sizes, chunk-index gaps
reset a beam, admission follows the budget, and a checkpoint restores a beam exactly."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP32_TOL = 1e-5
REDUCED_TOL = 1e-2


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(y):
    if y.dtype == torch.uint16:
        y = y.view(torch.int16).to(torch.int32) & 0xFFFF
    elif y.dtype in (torch.bfloat16, torch.float16):
        y = y.float()
    return y.cpu().numpy()


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def chunk_lengths(rng, total, chunk):
    """Random chunk sizes in 1..chunk (some single samples, some full chunks) summing to total."""
    out = []
    while sum(out) < total:
        r = rng.random()
        L = 1 if r < 0.1 else (chunk if r < 0.4 else int(rng.integers(1, chunk + 1)))
        out.append(min(L, total - sum(out)))
    return out


def run_stream(snd, st, beam, plan, xt, lengths, first_idx=0, ws=None):
    """Push xt [nchan][N] in chunks; returns the concatenated outputs and the per-push (t0, n)."""
    out = plan.empty_output("cuda")
    ws = plan.workspace("cuda") if ws is None else ws
    pieces, meta = [], []
    pos = 0
    for i, L in enumerate(lengths):
        (t0, n, status), = st.push([(beam, first_idx + i, xt[:, pos:pos + L], out)], workspace=ws)
        assert status == 0
        torch.cuda.synchronize()
        if n:
            pieces.append(to_np(out[:, :n]))
        meta.append((t0, n))
        pos += L
    return (np.concatenate(pieces, axis=1) if pieces else np.zeros((plan.ndm, 0))), meta


CASES = [("binary", dict(k_leaf=2, k_int=1), "u8"), ("graded", dict(cap=15), "u8"), ("graded", dict(cap=300), "u8"),
         ("float", {}, "f32"), ("float", dict(node_dtype="bf16"), "bf16")]


@pytest.mark.parametrize("mode,kw,inp", CASES)
def test_stream_equals_oracle_any_chunks(snd, orc, mode, kw, inp):
    spec = synth.workload(1)
    rng = synth.make_rng(4242)
    chunk = 1000
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode=mode, branching=2, chunk=chunk,
                    in_dtype=inp, **kw)
    total = plan.max_delay + 3 * chunk + 357
    z = spec.filterbank(total)
    if mode == "binary":
        x = orc.encode(z, [2.0])
    elif mode == "graded":
        x = orc.encode(z, [1.0, 2.0, 3.0, 4.0])
    else:
        x = z
    okw = {k: v for k, v in kw.items() if k != "node_dtype"}
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    if inp == "bf16":
        xt = snd.cast(xt, "bf16")
    want, _ = orc.snd_dedup(x, spec.freqs, d, mode=mode, cluster=4, branching=2, **okw)
    # the plain execute on the whole input, same plan parameters
    plain_plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, total, mode=mode, branching=2, in_dtype=inp, **kw)
    plain = to_np(plain_plan.execute(xt))
    st = snd.Stream(1 << 34)
    st.admit(0, plan)
    lengths = chunk_lengths(rng, total, chunk)
    _say(f"stream mode={mode} {kw} in={inp} chunks={len(lengths)} total={total}")
    y, meta = run_stream(snd, st, 0, plan, xt, lengths)
    assert y.shape == want.shape
    # outputs appear exactly when their sweep has arrived, contiguous in time
    S = np.cumsum(lengths)
    emitted = np.maximum(0, S - plan.max_delay)
    assert [m[1] for m in meta] == list(np.diff(np.concatenate([[0], emitted])))
    assert [m[0] for m in meta] == list(np.concatenate([[0], emitted[:-1]]))
    assert np.array_equal(y, plain)  # bit-identical to the plain form
    if mode == "float" and inp == "f32" and "node_dtype" not in kw:
        assert rel_rms(y, want) <= FP32_TOL
    elif mode == "float":
        assert rel_rms(y, want) <= REDUCED_TOL
    else:
        assert np.array_equal(y, want.astype(y.dtype))
    assert st.state(0) == dict(received=total, next_chunk=len(lengths), emitted=total - plan.max_delay)


def test_stream_gap_resets_history(snd):
    spec = synth.workload(1)
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=2048)
    x = torch.from_numpy(synth.random_levels(synth.make_rng(3), 64, 6 * 2048, 4)).cuda()
    out = plan.empty_output("cuda")
    ws = plan.workspace("cuda")
    st = snd.Stream(1 << 34)
    st.admit(5, plan)
    for i in range(2):
        st.push([(5, 10 + i, x[:, 2048 * i:2048 * (i + 1)], out)], workspace=ws)
    # chunk 12 is lost: chunk 13 restarts the history
    (t0, n, status), = st.push([(5, 13, x[:, 2048 * 3:2048 * 4], out)], workspace=ws)
    assert status == -7 and (t0, n) == (0, 0)
    assert st.state(5) == dict(received=2048, next_chunk=14, emitted=0)
    rest, _ = run_stream(snd, st, 5, plan, x[:, 2048 * 4:], [2048, 2048], first_idx=14)
    fresh = snd.Stream(1 << 34)
    fresh.admit(0, plan)
    ref, _ = run_stream(snd, fresh, 0, plan, x[:, 2048 * 3:], [2048, 2048, 2048])
    assert np.array_equal(rest, ref)
    # a repeated index is a gap too
    (_, _, status), = st.push([(5, 15, x[:, :2048], out)], workspace=ws)
    assert status == -7


def test_stream_admission_by_budget_and_multi_beam_push(snd):
    spec = synth.workload(1)
    pg = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=1024)
    pf = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="float", branching=2, chunk=1024,
                  in_dtype="bf16", node_dtype="bf16")
    hg, hf = snd.admission_bytes(pg), snd.admission_bytes(pf)
    assert hg > snd.history_bytes(pg) and hf > snd.history_bytes(pf)  # ring + batched-push workspace share
    st = snd.Stream(2 * hg + hf)
    st.admit(0, pg)
    st.admit(1, pf)
    st.admit(2, pg)
    with pytest.raises(snd.SndError) as ei:
        st.admit(3, pg)
    assert ei.value.status == -5
    assert st.usage() == dict(budget=2 * hg + hf, used=2 * hg + hf, n_beams=3)
    st.evict(2)
    st.admit(3, pg)
    assert st.beams() == [0, 1, 3]
    rng = synth.make_rng(11)
    N = pg.max_delay + 3 * 1024
    xg = torch.from_numpy(synth.random_levels(rng, 64, N, 4)).cuda()
    x3 = torch.from_numpy(synth.random_levels(rng, 64, N, 4)).cuda()
    xf = snd.cast(torch.from_numpy(synth.noise_filterbank(rng, 64, N)).cuda(), "bf16")
    ws = torch.empty(max(pg.info["workspace_bytes"], pf.info["workspace_bytes"]), dtype=torch.uint8, device="cuda")
    outs = {b: p.empty_output("cuda") for b, p in ((0, pg), (1, pf), (3, pg))}
    got = {0: [], 1: [], 3: []}
    srcs = {0: xg, 1: xf, 3: x3}
    for i in range(N // 1024 + 1):
        lo, hi = 1024 * i, min(N, 1024 * (i + 1))
        if lo >= N:
            break
        res = st.push([(b, i, srcs[b][:, lo:hi], outs[b]) for b in (0, 1, 3)], workspace=ws)
        torch.cuda.synchronize()
        for b, (t0, n, status) in zip((0, 1, 3), res):
            assert status == 0
            if n:
                got[b].append(to_np(outs[b][:, :n]))
    for b, p in ((0, pg), (1, pf), (3, pg)):
        plain = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, N, mode=p.mode, branching=2, in_dtype=p.in_dtype,
                         node_dtype=p.node_dtype)
        assert np.array_equal(np.concatenate(got[b], axis=1), to_np(plain.execute(srcs[b])))


def test_stream_checkpoint_restores_beam(snd):
    spec = synth.workload(1)
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="float", branching=2, chunk=1500)
    x = torch.from_numpy(synth.noise_filterbank(synth.make_rng(8), 64, plan.max_delay + 6000)).cuda()
    a = snd.Stream(1 << 34)
    a.admit(0, plan)
    first = [1500] * 4
    run_stream(snd, a, 0, plan, x, first)
    ck = a.export(0)
    b = snd.Stream(1 << 34)
    b.admit(9, plan)
    b.restore(9, ck)
    assert b.state(9) == a.state(0)
    rest = x[:, sum(first):]
    lens = [1500] * (rest.shape[1] // 1500) + ([rest.shape[1] % 1500] if rest.shape[1] % 1500 else [])
    ya, _ = run_stream(snd, a, 0, plan, rest, lens, first_idx=4)
    yb, _ = run_stream(snd, b, 9, plan, rest, lens, first_idx=4)
    assert np.array_equal(ya, yb) and ya.shape[1] > 0
    other = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="float", branching=2, chunk=1000)
    c = snd.Stream(1 << 34)
    c.admit(0, other)
    with pytest.raises(snd.SndError):
        c.restore(0, ck)  # ring shape differs


def test_stream_full_size_graded_chunk(snd, orc):
    """1024 channels, 4096 DMs to 2000, 8192-sample chunks (the serving beams' shape): the
    streamed output of the first complete chunks equals the plain execute on the same samples,
    and the oracle's recursion at 600 sampled (DM, time) cells, bit for bit."""
    spec = synth.workload(2)
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=4, chunk=8192)
    assert plan.info["stage_kernel"][0] == "anchored"
    T = 8192
    nchunks = (plan.max_delay + T - 1) // T + 2
    N = nchunks * T
    z = torch.from_numpy(spec.filterbank(N)).cuda()
    x = snd.encode(z, [1.0, 2.0, 3.0, 4.0])
    del z
    st = snd.Stream(1 << 36)
    st.admit(0, plan)
    _say(f"full-size stream: {nchunks} chunks of {T}, max_delay {plan.max_delay}")
    y, meta = run_stream(snd, st, 0, plan, x, [T] * nchunks)
    assert y.shape[1] == N - plan.max_delay
    plain = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, N, mode="graded", branching=4)
    assert np.array_equal(y, to_np(plain.execute(x)))
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    r = synth.make_rng(77)
    ks, ts = r.integers(0, plan.ndm, 600), r.integers(0, y.shape[1], 600)
    want = orc.snd_points(x.cpu().numpy(), spec.freqs, d, ks, ts, mode="graded", cluster=4, branching=4)
    assert np.array_equal(y[ks, ts], want.astype(y.dtype))


def test_batched_push_equals_per_beam_push(snd):
    """snd_stream_push_batched (shared grids across beams) gives the outputs of the per-beam
    push, through history fill, steady state and a chunk gap."""
    spec = synth.workload(1)
    plans = [snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=1024),
             snd.Plan(spec.freqs, spec.dms[:40], spec.tsamp_s, None, mode="float", branching=4, chunk=1024,
                      in_dtype="bf16", node_dtype="bf16"),
             snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="binary", branching=2, chunk=800, k_leaf=2,
                      k_int=1)]
    rng = synth.make_rng(77)
    N = 9 * 1024
    srcs = [torch.from_numpy(synth.random_levels(rng, 64, N, 4)).cuda(),
            snd.cast(torch.from_numpy(synth.noise_filterbank(rng, 64, N)).cuda(), "bf16"),
            torch.from_numpy(synth.random_spikes(rng, 64, N, 0.3)).cuda()]
    a, b = snd.Stream(1 << 34), snd.Stream(1 << 34)
    for i, p in enumerate(plans):
        a.admit(10 + i, p)
        b.admit(10 + i, p)
    ws = torch.empty(max(p.info["workspace_bytes"] for p in plans), dtype=torch.uint8, device="cuda")
    oa = [p.empty_output("cuda") for p in plans]
    ob = [p.empty_output("cuda") for p in plans]
    idx = [0, 0, 0]
    pos = [0, 0, 0]
    gaps = 0
    for step in range(9):
        items_a, items_b = [], []
        for i, p in enumerate(plans):
            L = min(p.n_out, N - pos[i]) if step % 3 else max(1, p.n_out // 3)
            if L <= 0:
                continue
            if step == 5 and i == 1:
                idx[i] += 1  # a lost chunk on one beam
            items_a.append((10 + i, idx[i], srcs[i][:, pos[i]:pos[i] + L], oa[i]))
            items_b.append((10 + i, idx[i], srcs[i][:, pos[i]:pos[i] + L], ob[i]))
            idx[i] += 1
            pos[i] += L
        ra = a.push(items_a, workspace=ws)
        rb = b.push(items_b, batched=True)
        torch.cuda.synchronize()
        assert ra == rb
        gaps += sum(1 for _, _, st in ra if st == -7)
        for (bid, _, _, _), (t0, n, status) in zip(items_a, ra):
            i = bid - 10
            if n:
                assert torch.equal(oa[i][:, :n], ob[i][:, :n]), (step, i)
    assert gaps == 1


def test_stream_bit_input_any_chunks(snd, orc):
    """Binary beams fed rows of bits: each chunk (any length, any bit offset in the ring) is
    merged into a ring of bits, and the output equals the plain execute on the whole bit
    input and the oracle, through per-beam and batched pushes and a checkpoint restore."""
    from bitrows import pack_bits
    spec = synth.workload(1)
    rng = synth.make_rng(5151)
    chunk = 1000
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="binary", branching=4, chunk=chunk,
                    in_dtype="bits", node_dtype="bits", k_leaf=2, k_int=1)
    assert plan.info["stage_kernel"][0] == "anchored_bits"
    total = plan.max_delay + 5 * chunk + 357
    x = orc.encode(spec.filterbank(total), [2.0])
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    want, _ = orc.snd_dedup(x, spec.freqs, d, mode="binary", cluster=4, branching=4, k_leaf=2, k_int=1)
    plain_plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, total, mode="binary", branching=4, in_dtype="bits",
                          node_dtype="bits", k_leaf=2, k_int=1)
    plain = to_np(plain_plan.execute(torch.from_numpy(pack_bits(x)).cuda()))
    assert np.array_equal(plain, want.astype(plain.dtype))
    lengths = chunk_lengths(rng, total, chunk)
    _say(f"bit stream chunks={len(lengths)} total={total} max_delay={plan.max_delay}")
    a, b = snd.Stream(1 << 34), snd.Stream(1 << 34)
    a.admit(0, plan)
    b.admit(0, plan)
    ws = plan.workspace("cuda")
    oa, ob = plan.empty_output("cuda"), plan.empty_output("cuda")
    ya, yb, yc = [], [], []
    c = oc = None
    pos = 0
    half = len(lengths) // 2
    for i, L in enumerate(lengths):
        xb = torch.from_numpy(pack_bits(x[:, pos:pos + L])).cuda()
        (t0, n, s1), = a.push([(0, i, xb, oa, L)], workspace=ws)
        (u0, m, s2), = b.push([(0, i, xb, ob, L)], batched=True)
        assert (t0, n, s1) == (u0, m, s2) and s1 == 0
        if c is not None:
            (v0, k, s3), = c.push([(0, i, xb, oc, L)], workspace=ws)
            assert (v0, k, s3) == (t0, n, s1)
        torch.cuda.synchronize()
        if n:
            ya.append(to_np(oa[:, :n]))
            yb.append(to_np(ob[:, :n]))
            if c is not None:
                yc.append(to_np(oc[:, :n]))
        pos += L
        if i == half:  # checkpoint the beam into a new stream, which then runs alongside
            c = snd.Stream(1 << 34)
            c.admit(0, plan)
            c.restore(0, a.export(0))
            oc = plan.empty_output("cuda")
    y = np.concatenate(ya, axis=1)
    assert np.array_equal(y, plain)
    assert np.array_equal(np.concatenate(yb, axis=1), plain)
    tail = np.concatenate(yc, axis=1)
    assert np.array_equal(tail, plain[:, plain.shape[1] - tail.shape[1]:])
    assert a.state(0) == dict(received=total, next_chunk=len(lengths), emitted=total - plan.max_delay)
