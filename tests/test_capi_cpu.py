"""Host-side checks of libsnd: it loads, exports every declared symbol, and its plan
(delays, shared-pattern counts, validation) agrees with the oracle.  No device calls."""

import ctypes as C
import os

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def snd():
    import paper_2606_15361_amd as m
    return m


def test_library_exports_every_declared_symbol(snd):
    from paper_2606_15361_amd import _capi
    names = _capi.declared_symbols(os.path.join(ROOT, "include", "snd.h"))
    assert "snd_execute" in names and "snd_plan_create" in names
    L = _capi.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_library_exports_no_undeclared_c_symbol(snd):
    """Every unmangled function the library defines is one the header declares (internal
    helpers have internal linkage or live in the C++ namespace)."""
    import shutil
    import subprocess
    from paper_2606_15361_amd import _capi
    if not shutil.which("nm"):
        pytest.skip("nm not available")
    names = set(_capi.declared_symbols(os.path.join(ROOT, "include", "snd.h")))
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    funcs = {ln.split()[-1] for ln in out.splitlines() if len(ln.split()) == 3 and ln.split()[1] == "T"}
    extra = sorted(n for n in funcs if not n.startswith("_Z") and n not in names)
    assert not extra, extra


@pytest.mark.parametrize("nchan,ndm,C_,B,dmax", [(64, 64, 4, 2, 300.0), (37, 29, 3, 3, 40.0), (24, 17, 5, 4, 30.0),
                                                 (9, 5, 4, 8, 10.0), (3, 4, 4, 2, 10.0), (1, 3, 1, 2, 50.0)])
def test_plan_matches_oracle_counts(snd, orc, nchan, ndm, C_, B, dmax):
    f = synth.channel_freqs(nchan)
    rng = synth.make_rng(nchan + ndm)
    dms = rng.uniform(0, dmax, ndm)
    dms[-1] = dms[0]
    od = orc.delays(f, dms, 0.138e-3)
    nsamp = int(od.max()) + 50
    for mode in ("binary", "graded", "float"):
        p = snd.Plan(f, dms, 0.138e-3, nsamp, mode=mode, branching=B, cluster=C_)
        assert np.array_equal(p.delays(), od)
        assert p.n_out == nsamp - od.max()
        x = np.zeros((nchan, nsamp), np.uint8)
        _, counts = orc.snd_dedup(x, f, od, mode=mode, cluster=C_, branching=B)
        assert p.info["neurons_per_level"] == [c[0] for c in counts]
        assert p.info["synapses_per_level"] == [c[1] for c in counts]
        assert p.info["nodes_per_level"] == orc.tree_shape(f, C_, B)


def test_config2_plan_shape(snd):
    spec = synth.workload(2)
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4)
    assert p.info["neurons_per_level"] == [49722, 207270, 65356, 16384, 4096]
    assert p.info["n_synapses"] == 1371312
    assert p.n_out == 102748
    assert p.info["n_stages"] == 2
    assert p.info["build_seconds"] < 3.0
    # float mode: every final-stage row is one sum, whatever the tree's shape
    assert p.info["stage_kernel"] == ["anchored", "group_lin"]
    b8 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=8)
    assert b8.info["stage_kernel"] == ["anchored", "group_lin"]
    # graded u8 rows with level-1 nodes of 4 or 8 inputs: levels on packed 16-bit counts
    pg = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=4)
    assert pg.info["stage_kernel"] == ["anchored", "group_pack"]
    g8 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=8)
    assert g8.info["stage_kernel"] == ["anchored", "group_pack"]
    g2 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=2)
    assert g2.info["stage_kernel"] == ["anchored", "group_fast"]
    g16 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=4, cap=4095)
    assert g16.node_dtype == "u16" and g16.info["stage_kernel"] == ["anchored", "group_fast"]
    pb = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="binary", branching=4, node_dtype="u8")
    assert pb.info["stage_kernel"] == ["anchored", "group_fast"]
    h8 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=8, node_dtype="bf16",
                  in_dtype="bf16")
    assert h8.info["stage_kernel"] == ["anchored", "group_lin"]  # 16-bit float rows are one sum too
    h4 = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4, node_dtype="f16")
    assert h4.info["stage_kernel"] == ["anchored", "group_lin"]
    # a ragged tree (1000 channels: the last leaf and node groups are short) has irregular
    # level-1 nodes and takes the general row-group kernel in the activated modes
    rag = snd.Plan(synth.channel_freqs(1000), synth.dm_linear(512, 0, 500), spec.tsamp_s, 20000, mode="graded",
                   branching=4)
    assert rag.info["stage_kernel"] == ["anchored", "group_lds"]
    ragf = snd.Plan(synth.channel_freqs(1000), synth.dm_linear(512, 0, 500), spec.tsamp_s, 20000, mode="float",
                    branching=4)
    assert ragf.info["stage_kernel"] == ["anchored", "group_lin"]
    g = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4, generic_kernels=True)
    assert g.info["stage_kernel"] == ["generic", "generic"]
    every = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, 40000, mode="graded", branching=4, stage_levels=0b1111)
    assert every.info["n_stages"] == 5 and every.info["stage_rows"] == [49722, 207270, 65356, 16384, 4096]


def test_plan_validation_errors(snd):
    from paper_2606_15361_amd import SndError, _capi
    f = synth.channel_freqs(16)
    dms = np.array([0.0, 5.0])
    ok = dict(mode="graded", branching=2, cluster=4)
    snd.Plan(f, dms, 0.138e-3, 500, **ok)
    bad = [
        (dict(dms=np.array([-1.0])), _capi.ERR_INVALID),
        (dict(nsamp=10), _capi.ERR_INVALID),
        (dict(fref=410.0), _capi.ERR_INVALID),
        (dict(branching=1), _capi.ERR_INVALID),
        (dict(cluster=0), _capi.ERR_INVALID),
        (dict(mode="binary", k_leaf=0), _capi.ERR_INVALID),
        (dict(cap=0), _capi.ERR_INVALID),
        (dict(cap=70000), _capi.ERR_INVALID),
        (dict(mode="float", in_dtype="u8"), _capi.ERR_UNSUPPORTED),
        (dict(node_dtype="f32"), _capi.ERR_UNSUPPORTED),
        (dict(cap=300, node_dtype="u8"), _capi.ERR_UNSUPPORTED),
        (dict(stage_levels=1 << 3), _capi.ERR_INVALID),
        (dict(in_dtype="bits"), _capi.ERR_UNSUPPORTED),
        (dict(mode="binary", in_dtype="bits", node_dtype="u8"), _capi.ERR_UNSUPPORTED),
        (dict(mode="binary", in_dtype="bits", cluster=16), _capi.ERR_UNSUPPORTED),
        (dict(mode="binary", in_dtype="bits", stage_levels=0x80000000), _capi.ERR_UNSUPPORTED),
        (dict(mode="binary", in_dtype="bits", generic_kernels=True), _capi.ERR_UNSUPPORTED),
    ]
    for kw, code in bad:
        args = dict(ok)
        dd = kw.pop("dms", dms)
        ns = kw.pop("nsamp", 500)
        args.update(kw)
        with pytest.raises(SndError) as ei:
            snd.Plan(f, dd, 0.138e-3, ns, **args)
        assert ei.value.status == code, kw


def test_bit_input_plans(snd):
    """Bit input: leaf stage on bit rows, bit-row final stage; streamed through a ring of bits."""
    from paper_2606_15361_amd import SndError, _capi
    f = synth.channel_freqs(64)
    dms = synth.dm_linear(40, 0, 60)
    p = snd.Plan(f, dms, 0.138e-3, 2000, mode="binary", branching=4, in_dtype="bits")
    assert p.info["stage_kernel"] == ["anchored_bits", "group_bits"]
    assert p.info["stage_src_dtype"] == ["bits", "bits"]
    u = snd.Plan(f, dms, 0.138e-3, 2000, mode="binary", branching=4)
    # same tree; the input read is 1/8 of the byte input's
    assert p.info["n_neurons"] == u.info["n_neurons"] and p.info["stage_entries"] == u.info["stage_entries"]
    assert u.info["stage_alg_bytes"][0] - p.info["stage_alg_bytes"][0] == 64 * 2000 - 64 * 2000 // 8
    # a stream keeps one bit per sample: ring of whole words, rows padded to 256 bytes
    q = snd.Plan(f, dms, 0.138e-3, None, mode="binary", branching=4, in_dtype="bits", chunk=512)
    nb = C.c_int64()
    _capi.check(_capi.lib().snd_stream_history_bytes(q.handle, C.byref(nb)))
    ring = -(-(q.info["max_delay"] + q.n_out) // 32) * 32
    assert nb.value == 64 * (-(-ring // 2048) * 2048) // 8
    with pytest.raises(SndError) as ei:
        snd.Plan(f, dms, 0.138e-3, 2000, mode="binary", branching=4, in_dtype="bits", cluster=16)
    assert ei.value.status == _capi.ERR_UNSUPPORTED
    # pushes of bit chunks: lengths and pitches in bits, whole 32-bit words per row, 4-byte
    # aligned rows; checked before any device work (admission records the buffer only)
    L = _capi.lib()
    h = C.c_void_p()
    _capi.check(L.snd_stream_create(1 << 34, C.byref(h)))
    _capi.check(L.snd_stream_admit(h, 3, q.handle, C.c_void_p(1 << 20), nb.value))
    item = _capi.StreamItem()
    item.beam_id, item.chunk_idx, item.chunk_len = 3, 0, 300
    item.d_chunk, item.chunk_pitch = 1 << 24, 320
    item.d_out, item.out_pitch = 1 << 28, q.n_out
    rc = L.snd_stream_push(h, 1, C.byref(item), None, 0, None)
    assert rc == _capi.ERR_STATE  # the arguments pass; the plan's tables are not uploaded
    for pitch, ptr in ((300, 1 << 24), (330, 1 << 24), (320, (1 << 24) + 2)):
        item.chunk_pitch, item.d_chunk = pitch, ptr
        assert L.snd_stream_push(h, 1, C.byref(item), None, 0, None) == _capi.ERR_INVALID, (pitch, ptr)
    item.chunk_pitch, item.d_chunk, item.chunk_len = 1024, 1 << 24, q.n_out + 1
    assert L.snd_stream_push(h, 1, C.byref(item), None, 0, None) == _capi.ERR_INVALID  # longer than n_out
    L.snd_stream_destroy(h)
    # bit input pitch must be whole words; encoder pitch likewise
    buf = (C.c_uint8 * 256)()
    rc = _capi.lib().snd_encode_bits(C.cast(buf, C.c_void_p), 100, 0, 1, 100, C.c_float(1.0),
                                     C.cast(buf, C.c_void_p), 112, None)
    assert rc == _capi.ERR_INVALID


def test_stage_variants_are_consistent_plans(snd):
    f = synth.channel_freqs(64)
    dms = synth.dm_linear(40, 0, 60)
    base = snd.Plan(f, dms, 0.138e-3, 2000, mode="float", branching=2)
    top = base.info["n_levels"] - 1
    none = snd.Plan(f, dms, 0.138e-3, 2000, mode="float", branching=2, stage_levels=0x80000000)
    assert none.info["n_stages"] == 1 and none.info["workspace_bytes"] == 0
    assert none.info["stage_entries"] == [40 * 64]
    every = snd.Plan(f, dms, 0.138e-3, 2000, mode="float", branching=2, stage_levels=(1 << top) - 1)
    assert every.info["n_stages"] == top + 1
    # per-level schedule: every stage input is one synapse of the shared-pattern tree
    assert every.info["stage_entries"][:-1] == every.info["synapses_per_level"][:-1]
    assert base.info["stage_entries"] == [base.info["synapses_per_level"][0], 40 * base.info["nodes_per_level"][0]]


def test_execute_requires_upload(snd):
    from paper_2606_15361_amd import SndError, _capi
    p = snd.Plan(synth.channel_freqs(8), [0.0, 1.0], 0.138e-3, 100, mode="float", branching=2)
    buf = (C.c_uint8 * 1024)()
    rc = _capi.lib().snd_execute(p.handle, C.cast(buf, C.c_void_p), 100, C.cast(buf, C.c_void_p), 100,
                                 None, 0, None)
    assert rc == _capi.ERR_STATE
    assert "upload" in _capi.lib().snd_last_error().decode()
    with pytest.raises(SndError):
        _capi.check(rc)


def test_streaming_plan_and_admission_host_logic(snd):
    """Streaming plans (chunk > 0), history sizing and admission by budget; no device work
    (admission only records the caller's buffer, so any 256-byte aligned address serves)."""
    import ctypes as C
    from paper_2606_15361_amd import SndError, _capi
    L = _capi.lib()
    f = synth.channel_freqs(64)
    dms = synth.dm_linear(64, 0, 300)
    p = snd.Plan(f, dms, 0.138e-3, None, mode="graded", branching=2, chunk=1000)
    assert p.n_out == 1000 and p.nsamp == p.max_delay + 1000
    assert p.max_delay == 4186
    nb = snd.history_bytes(p)
    assert nb == 64 * ((p.max_delay + 1000 + 255) // 256 * 256)  # u8 ring rows padded to 256 bytes
    pf = snd.Plan(f, dms, 0.138e-3, None, mode="float", branching=2, chunk=1000, node_dtype="bf16", in_dtype="bf16")
    assert snd.history_bytes(pf) == 64 * ((2 * (pf.max_delay + 1000) + 255) // 256 * 256)

    na = snd.admission_bytes(p)
    h = C.c_void_p()
    assert L.snd_stream_create(0, C.byref(h)) == _capi.ERR_INVALID
    _capi.check(L.snd_stream_create(2 * na + na // 2, C.byref(h)))
    fake = C.c_void_p(1 << 20)
    assert L.snd_stream_admit(h, 0, p.handle, C.c_void_p((1 << 20) + 8), nb) == _capi.ERR_INVALID  # misaligned
    assert L.snd_stream_admit(h, 0, p.handle, fake, nb - 1) == _capi.ERR_NOMEM
    used = C.c_int64()
    _capi.check(L.snd_stream_usage(h, None, C.byref(used), None))
    assert used.value == 0
    assert L.snd_stream_admit(h, 0, p.handle, fake, nb) == _capi.OK  # tables are needed only to push
    # a plan without the input-anchored first stage cannot stream
    g = snd.Plan(f, dms, 0.138e-3, None, mode="graded", branching=2, chunk=1000, generic_kernels=True)
    assert L.snd_stream_admit(h, 1, g.handle, fake, nb) == _capi.ERR_UNSUPPORTED
    # budget: the third beam of this size does not fit
    assert L.snd_stream_admit(h, 2, p.handle, fake, 3 * nb) == _capi.OK
    assert L.snd_stream_admit(h, 3, p.handle, fake, nb) == _capi.ERR_CAPACITY
    _capi.check(L.snd_stream_usage(h, None, C.byref(used), None))
    assert used.value == 2 * na
    small_budget = C.c_void_p()
    _capi.check(L.snd_stream_create(na - 1, C.byref(small_budget)))
    assert L.snd_stream_admit(small_budget, 0, p.handle, fake, nb) == _capi.ERR_CAPACITY
    assert "budget" in L.snd_last_error().decode()
    # unknown beams
    assert L.snd_stream_evict(h, 7) == _capi.ERR_STATE
    item = _capi.StreamItem()
    item.beam_id = 7
    assert L.snd_stream_push(h, 1, C.byref(item), None, 0, None) == _capi.ERR_STATE
    assert L.snd_stream_push(h, 0, None, None, 0, None) == _capi.OK
    L.snd_stream_destroy(h)
    L.snd_stream_destroy(small_budget)
    with pytest.raises(SndError):
        snd.Plan(f, dms, 0.138e-3, None, mode="graded", branching=2, chunk=-5)


def test_batch_grouping_and_errors_host_logic(snd):
    """Batched execution groups stage launches by kernel class; argument errors are caught on
    the host before any device work."""
    import ctypes as C
    from paper_2606_15361_amd import _capi
    L = _capi.lib()
    f = synth.channel_freqs(64)
    mk = lambda n, hi, **kw: snd.Plan(f, synth.dm_linear(n, 0, hi), 0.138e-3, 6000, branching=2, **kw)
    plans = [mk(40, 100, mode="graded"), mk(64, 300, mode="graded"), mk(20, 50, mode="binary"),
             mk(33, 120, mode="float"), mk(33, 120, mode="float", node_dtype="bf16", in_dtype="bf16")]
    # stage 0: anchored graded / binary / float f32 / float bf16 -> 4 classes; final stage the same
    # split (the two graded plans share one grid per stage)
    nb, nl = snd.records_bytes(plans)
    assert nl == 8 and nb % 256 == 0 and nb > 0
    nb1, nl1 = snd.records_bytes(plans[:1])
    assert nl1 == 2
    hs = (C.c_void_p * 1)(plans[0].handle.value)
    ptr = (C.c_void_p * 1)(1 << 20)
    pitch = (C.c_int64 * 1)(6000)
    wsb = (C.c_int64 * 1)(plans[0].info["workspace_bytes"])
    rc = L.snd_batch_execute(1, hs, ptr, pitch, ptr, pitch, ptr, wsb, None, C.c_void_p(1 << 20), nb1, None, None)
    assert rc == _capi.ERR_STATE  # tables not uploaded
    assert L.snd_batch_execute(0, hs, ptr, pitch, ptr, pitch, ptr, wsb, None, C.c_void_p(1 << 20), nb1, None,
                               None) == _capi.ERR_INVALID
    assert L.snd_batch_execute(1, hs, ptr, pitch, ptr, pitch, ptr, wsb, None, C.c_void_p((1 << 20) + 4), nb1, None,
                               None) == _capi.ERR_INVALID  # misaligned records


def test_autotune_argument_errors(snd):
    import ctypes as C
    from paper_2606_15361_amd import _capi
    from paper_2606_15361_amd.plan import make_desc
    L = _capi.lib()
    f = synth.channel_freqs(16)
    d, _f, _d, _, _ = make_desc(f, [0.0, 5.0], 0.138e-3, 500, mode="graded", branching=2, chunk=100)
    c = (_capi.TuneCandidate * 1)()
    best = C.c_int32()
    buf = C.c_void_p(1 << 20)
    rc = L.snd_autotune(C.byref(d), c, 1, buf, 500, buf, 500, buf, 1 << 20, buf, 1 << 20, 1, C.byref(best), None)
    assert rc == _capi.ERR_INVALID and "whole block" in L.snd_last_error().decode()
    d.chunk = 0
    assert L.snd_autotune(C.byref(d), c, 0, buf, 500, buf, 500, buf, 1 << 20, buf, 1 << 20, 1, C.byref(best),
                          None) == _capi.ERR_INVALID


def test_bit_row_packing_layout():
    """The tests' bit-row packing follows the BITS layout: bit i of word w is sample 32 w + i."""
    from bitrows import pack_bits
    rng = np.random.default_rng(3)
    x = (rng.random((3, 301)) < 0.4).astype(np.uint8)
    w = pack_bits(x).view(np.uint32)
    assert w.shape == (3, 12)  # 301 samples -> 10 words, padded to a multiple of 4
    for c in range(3):
        for t in range(w.shape[1] * 32):
            bit = (int(w[c, t // 32]) >> (t % 32)) & 1
            assert bit == (x[c, t] if t < 301 else 0)


def test_multirate_host_logic_matches_the_oracle(snd, orc):
    """Scrunch factors and the cross-band merge are host code: compared with the oracle here."""
    f = synth.channel_freqs(1024)
    dms = np.concatenate([np.linspace(0, 3000, 801), [289.0, 289.5, 578.0, 578.5, 1157.0, 2313.5]])
    for s_max in (1, 2, 16):
        assert np.array_equal(snd.scrunch_factors(f, dms, 0.138e-3, s_max), orc.scrunch_factors(f, dms, 0.138e-3, s_max))
    f64 = synth.channel_freqs(64)
    assert np.array_equal(snd.scrunch_factors(f64, dms[:200], 0.138e-3), orc.scrunch_factors(f64, dms[:200], 0.138e-3))
    rng = np.random.default_rng(8)
    for trial in range(20):
        n = int(rng.integers(0, 40))
        cands = [dict(dm=float(rng.integers(0, 200)), t_ms=float(rng.integers(0, 2000)),
                      snr=float(rng.integers(6, 12)), band=0, k=i, width=1, t=0, npix=1) for i in range(n)]
        got = snd.merge_candidates(cands)
        want = orc.merge_candidates(cands)
        assert [(g["dm"], g["t_ms"], g["snr"], g["k"]) for g in got] == [(w["dm"], w["t_ms"], w["snr"], w["k"])
                                                                         for w in want]


def test_validation_host_logic_matches_the_oracle(snd, orc):
    """Effective widths and injection matching are host code: compared with the oracle here,
    on the hand-worked cases and on random ones with ties in S/N, time and DM."""
    import json
    f = synth.channel_freqs(1024)
    dms = np.linspace(0, 3000, 301)
    ws = np.linspace(0.1, 20, 301)
    assert np.allclose(snd.effective_width(f, 0.138e-3, dms, ws), orc.effective_width(f, 0.138e-3, dms, ws),
                       rtol=1e-15, atol=0.0)
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "injection_match.json")))
    for case in g["cases"]:
        c = np.array(case["candidates"], dtype=np.float64).reshape(-1, 3)
        q = np.array(case["injections"], dtype=np.float64).reshape(-1, 3)
        match, n = snd.match_injections(c[:, 0], c[:, 1], c[:, 2], q[:, 0], q[:, 1], q[:, 2], g["dm_tol"], g["t_frac"])
        assert list(match) == case["expected"], case["name"]
    rng = np.random.default_rng(12)
    for trial in range(40):
        nc, ni = int(rng.integers(0, 30)), int(rng.integers(0, 12))
        # coarse values so that ties and bounds occur
        c = np.stack([rng.integers(0, 40, nc) * 1.0, rng.integers(0, 20, nc) * 0.5, rng.integers(6, 10, nc) * 1.0], 1)
        q = np.stack([rng.integers(0, 40, ni) * 1.0, rng.integers(0, 20, ni) * 0.5, rng.integers(0, 8, ni) * 1.0], 1)
        match, n = snd.match_injections(c[:, 0], c[:, 1], c[:, 2], q[:, 0], q[:, 1], q[:, 2], 5.0, 0.5)
        want, wn = orc.match_injections([dict(dm=a, t_ms=b, snr=s) for a, b, s in c],
                                        [dict(dm=a, t_ms=b, w_eff_ms=w) for a, b, w in q], 5.0, 0.5)
        assert list(match) == want and n == wn
    with pytest.raises(snd.SndError):
        snd.match_injections([1.0], [1.0], [float("nan")], [1.0], [1.0], [1.0])
    with pytest.raises(snd.SndError):
        snd.match_injections([1.0], [1.0], [7.0], [1.0], [1.0], [-1.0])
    with pytest.raises(snd.SndError):
        snd.effective_width(f, 0.138e-3, [-1.0], [1.0])


def test_new_entry_points_reject_bad_arguments(snd):
    """Front-end, FDMT and detector-descriptor checks fail before any device call."""
    from paper_2606_15361_amd import _capi
    L = _capi.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails its argument checks
    P = C.c_void_p
    # zero-DM: null filterbank, pitch below nsamp, negative gamma
    assert L.snd_zero_dm(None, 100, 4, 100, 5.0, None, None) == _capi.ERR_INVALID
    assert L.snd_zero_dm(fake, 50, 4, 100, 5.0, None, None) == _capi.ERR_INVALID
    assert L.snd_zero_dm(fake, 100, 4, 100, -1.0, None, None) == _capi.ERR_INVALID
    # channel flagging: the sigma buffer is required; nchan, window, k and flags pitch checked
    assert L.snd_flag_channels(fake, 100, 4, 100, 10, 5.0, None, None, 0, None) == _capi.ERR_INVALID
    assert L.snd_flag_channels(fake, 100, 9000, 100, 10, 5.0, fake, None, 0, None) == _capi.ERR_INVALID
    assert L.snd_flag_channels(fake, 100, 4, 100, 0, 5.0, fake, None, 0, None) == _capi.ERR_INVALID
    assert L.snd_flag_channels(fake, 100, 4, 100, 10, -2.0, fake, None, 0, None) == _capi.ERR_INVALID
    assert L.snd_flag_channels(fake, 100, 4, 100, 10, 5.0, fake, fake, 3, None) == _capi.ERR_INVALID
    # FDMT: channel count a power of two, descending frequencies, the sweep inside the block
    f = np.ascontiguousarray(synth.channel_freqs(64))
    h = P()
    assert L.snd_fdmt_create(48, f.ctypes.data_as(P), 0.25, 0.138e-3, 100.0, 4096, C.byref(h)) == _capi.ERR_INVALID
    fa = np.ascontiguousarray(f[::-1])
    assert L.snd_fdmt_create(64, fa.ctypes.data_as(P), 0.25, 0.138e-3, 100.0, 4096, C.byref(h)) == _capi.ERR_INVALID
    assert L.snd_fdmt_create(64, f.ctypes.data_as(P), 0.25, 0.138e-3, 3000.0, 1000, C.byref(h)) == _capi.ERR_INVALID
    assert L.snd_fdmt_create(64, f.ctypes.data_as(P), 0.25, 0.138e-3, 100.0, 4096, C.byref(h)) == _capi.OK
    nd = C.c_int64()
    assert L.snd_fdmt_query(h, C.byref(nd), None, None, None, None) == _capi.OK and nd.value > 1
    # execute before upload is a state error, not a device call
    assert L.snd_fdmt_execute(h, fake, 4096, fake, 4096, fake, 1 << 40, None) == _capi.ERR_STATE
    assert L.snd_fdmt_destroy(h) == _capi.OK
    # detector descriptor: sigma_estimator must be 0 or 1
    p = snd.Plan(synth.channel_freqs(4), np.zeros(3), 0.138e-3, 100, mode="graded", branching=2)
    w = np.array([1, 2], np.int32)
    d = _capi.DetectDesc()
    d.widths = w.ctypes.data_as(C.POINTER(C.c_int32))
    d.nwidths, d.threshold, d.sigma_min, d.closing_radius, d.n_min, d.max_pixels = 2, 6.0, 0.0, 4, 10, 100
    d.sigma_estimator = 2
    nb = C.c_int64()
    assert L.snd_detect_workspace(p.handle, C.byref(d), C.byref(nb)) == _capi.ERR_INVALID
    d.sigma_estimator = 1
    assert L.snd_detect_workspace(p.handle, C.byref(d), C.byref(nb)) == _capi.OK


def _fake_device_ptr():
    # a 256-byte aligned address that admission records but never dereferences
    return C.c_void_p(0x7F0000000000)


def test_stream_admission_charges_ring_and_workspace(snd):
    """Admission charges a beam's history ring plus its share of a batched push's workspace, so
    a budget that admits a set of beams also holds a batched push of all of them (host-only
    accounting: admission touches no device memory)."""
    from paper_2606_15361_amd import _capi
    spec = synth.workload(1)
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=1024)
    ring = snd.history_bytes(p)
    ws = (p.info["workspace_bytes"] + 255) // 256 * 256
    assert ws > 0 and snd.admission_bytes(p) == ring + ws
    lib = _capi.lib()
    for budget, want in ((ring + ws - 1, _capi.ERR_CAPACITY), (ring, _capi.ERR_CAPACITY), (ring + ws, _capi.OK)):
        h = C.c_void_p()
        assert lib.snd_stream_create(budget, C.byref(h)) == _capi.OK
        assert lib.snd_stream_admit(h, 0, p.handle, _fake_device_ptr(), ring) == want
        b, u, n = C.c_int64(), C.c_int64(), C.c_int32()
        assert lib.snd_stream_usage(h, C.byref(b), C.byref(u), C.byref(n)) == _capi.OK
        assert (u.value, n.value) == ((ring + ws, 1) if want == _capi.OK else (0, 0))
        if want == _capi.OK:
            assert lib.snd_stream_evict(h, 0) == _capi.OK
            assert lib.snd_stream_usage(h, C.byref(b), C.byref(u), C.byref(n)) == _capi.OK and u.value == 0
        lib.snd_stream_destroy(h)


def test_stream_import_rejects_inconsistent_checkpoints(snd):
    """A checkpoint header whose state the beam cannot be in is rejected before anything is
    copied: emitted must be max(0, received - max_delay), and a beam with nothing received has
    emitted 0 and next chunk -1.  A push on a plan whose tables were never uploaded is refused."""
    from paper_2606_15361_amd import _capi
    spec = synth.workload(1)
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, None, mode="graded", branching=2, chunk=1024)
    lib = _capi.lib()
    h = C.c_void_p()
    assert lib.snd_stream_create(1 << 40, C.byref(h)) == _capi.OK
    assert lib.snd_stream_admit(h, 7, p.handle, _fake_device_ptr(), snd.history_bytes(p)) == _capi.OK
    nb = C.c_int64()
    assert lib.snd_stream_export_bytes(h, 7, C.byref(nb)) == _capi.OK
    ring = snd.history_bytes(p)
    assert nb.value == 64 + ring
    md = p.max_delay
    ring_len = md + p.n_out
    es, pitch = 1, (ring_len + 255) // 256 * 256
    assert 64 * pitch == ring

    def header(received, emitted, next_chunk, magic=0x31564548444e53, rl=ring_len):
        buf = np.zeros(nb.value, dtype=np.uint8)
        buf[:64] = np.frombuffer(np.array([magic, received, emitted, next_chunk, rl, pitch, es, 64],
                                          dtype=np.int64).tobytes(), dtype=np.uint8)
        return buf

    bad = [header(10 * md, 0, 5),                  # received far above emitted: outputs past n_out
           header(md + 100, 99, 5),                # emitted one short
           header(md + 100, 101, 5),               # emitted one over
           header(50, 0, -1),                      # samples received but no chunk index
           header(0, 0, 3),                        # nothing received but an expected index
           header(-5, 0, -1),
           header(md + 100, 100, 0),
           header(md + 100, 100, 5, magic=1),      # not a checkpoint
           header(md + 100, 100, 5, rl=ring_len + 1)]  # another ring shape
    for buf in bad:
        rc = lib.snd_stream_import(h, 7, buf.ctypes.data_as(C.c_void_p), buf.size, None)
        assert rc == _capi.ERR_INVALID, buf[:64].view(np.int64)
    short = header(md + 100, 100, 5)[:100]
    assert lib.snd_stream_import(h, 7, short.ctypes.data_as(C.c_void_p), short.size, None) == _capi.ERR_INVALID
    r, nx, e = C.c_int64(), C.c_int64(), C.c_int64()
    assert lib.snd_stream_beam_state(h, 7, C.byref(r), C.byref(nx), C.byref(e)) == _capi.OK
    assert (r.value, nx.value, e.value) == (0, -1, 0)  # nothing restored
    # a push before the plan's tables are uploaded: STATE, before any copy or launch
    it = (_capi.StreamItem * 1)()
    it[0].beam_id, it[0].chunk_idx, it[0].chunk_len, it[0].chunk_pitch = 7, 0, 1024, 1024
    it[0].d_chunk, it[0].d_out, it[0].out_pitch = 0x7F0000100000, 0x7F0000200000, p.n_out
    assert lib.snd_stream_push(h, 1, it, _fake_device_ptr(), 1 << 40, None) == _capi.ERR_STATE
    lib.snd_stream_destroy(h)


def test_noalloc_detect_rejects_workspaces_beyond_the_scratch(snd):
    """snd_detect_launch_noalloc refuses, before touching any device, a descriptor whose
    workspace exceeds its fixed device array."""
    import numpy as np
    from paper_2606_15361_amd import _capi as capi
    spec = synth.workload(1)
    plan = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=2)
    w = np.array([1, 2, 4], dtype=np.int32)
    desc = capi.DetectDesc()
    desc.widths = w.ctypes.data_as(C.POINTER(C.c_int32))
    desc.nwidths, desc.threshold, desc.closing_radius, desc.n_min = 3, 5.0, 4, 1
    desc.max_pixels = 1 << 24
    stage = (C.c_uint8 * 512)()
    rc = capi.lib().snd_detect_launch_noalloc(plan.handle, C.c_void_p(1 << 20), plan.n_out, C.byref(desc),
                                              C.cast(stage, C.c_void_p), 512, None)
    assert rc == capi.ERR_NOMEM
    assert b"static scratch" in capi.lib().snd_last_error()


def test_tune_word_plans(snd):
    """Launch-shape choices (snd_plan_desc.tune): every field builds a plan of the same kernels
    and counts; a smaller LDS batch budget makes more batches; unknown bits and a leaf window
    the LDS cannot hold are refused."""
    from paper_2606_15361_amd import SndError, tune_word, tune_fields
    spec = synth.workload(2)
    base = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=4)
    for kw in (dict(xcd_groups=1), dict(xcd_groups=64), dict(lds_quarters_off=2), dict(leaf_window=512),
               dict(leaf_window=1024, xcd_groups=4, lds_quarters_off=1)):
        t = tune_word(**kw)
        assert {k: v for k, v in tune_fields(t).items() if v} == {k: v for k, v in kw.items() if v}
        p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=4, tune=t)
        assert p.info["stage_kernel"] == base.info["stage_kernel"]
        assert p.info["neurons_per_level"] == base.info["neurons_per_level"] and p.n_out == base.n_out
        if kw.get("lds_quarters_off"):
            assert p.info["stage_batches"][1] > base.info["stage_batches"][1]
    with pytest.raises(SndError) as e:
        snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="graded", branching=4, tune=1 << 12)
    assert e.value.status == -1
    with pytest.raises(SndError) as e:  # 4 channels x (4096 + spread) f32 samples exceed 64 KB
        snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="float", branching=4,
                 tune=tune_word(leaf_window=4096))
    assert e.value.status == -2
    with pytest.raises(ValueError):
        tune_word(xcd_groups=3)
