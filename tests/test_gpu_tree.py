"""GPU parity of the SND tree (libsnd through its C ABI) against the CPU oracle.

Integer modes must be bit-exact; float32 within rel-RMS 1e-5 of the FP64 oracle (bit-exact on
small-integer inputs); BF16/FP16 storage within rel-RMS 1e-2 of the FP64 oracle on the
original float32 input.
"""

import sys

import numpy as np
import pytest

import synth
from bitrows import pack_bits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STAGE_NONE = 0x80000000
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


def gpu_run(plan, x, stage_by_stage=False):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    if stage_by_stage:
        out = plan.empty_output(xt.device)
        for s in range(plan.info["n_stages"]):
            plan.execute(xt, out=out, stage=s)
        y = out
    else:
        y = plan.execute(xt)
    torch.cuda.synchronize()
    return to_np(y)


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / max(np.sqrt(np.mean(b ** 2)), 1e-300))


def _inputs(rng, mode, nchan, nsamp):
    if mode == "binary":
        return synth.random_spikes(rng, nchan, nsamp, 0.3)
    if mode == "graded":
        return synth.random_levels(rng, nchan, nsamp, 4)
    return synth.noise_filterbank(rng, nchan, nsamp)


def _case(nchan, ndm, seed, extra=1037):
    rng = synth.make_rng(seed)
    f = synth.channel_freqs(nchan)
    dms = rng.uniform(0, 40.0, ndm)
    dms[-1] = dms[0]
    dms[0] = 0.0
    return rng, f, dms, extra


SHAPES = [(64, 4, 2), (37, 3, 3), (24, 5, 4), (16, 1, 2), (9, 4, 8), (3, 4, 2), (1, 1, 2)]


@pytest.mark.parametrize("nchan,C_,B", SHAPES)
@pytest.mark.parametrize("mode,kw", [("binary", dict(k_leaf=2, k_int=2)), ("binary", dict(k_leaf=1, k_int=2)),
                                     ("graded", dict(cap=255)), ("graded", dict(cap=7)), ("float", {})])
def test_parity_small(snd, orc, nchan, C_, B, mode, kw):
    rng, f, dms, extra = _case(nchan, 33, nchan * 31 + B)
    d = orc.delays(f, dms, 0.138e-3)
    nsamp = int(d.max()) + extra
    x = _inputs(rng, mode, nchan, nsamp)
    want, _ = orc.snd_dedup(x, f, d, mode=mode, cluster=C_, branching=B, **kw)
    ys = []
    nlev = len(orc.tree_shape(f, C_, B))
    variants = [(0, False, None), (0, True, None), (STAGE_NONE, False, None)]
    if mode == "binary":
        variants.append((0, False, "u8"))  # byte rows next to the default bit rows
    if nlev > 2:
        variants += [((1 << (nlev - 1)) - 1, False, None), ((1 << (nlev - 1)) - 1, True, None)]
    for sl, generic, node in variants:
        _say(f"case nchan={nchan} C={C_} B={B} mode={mode} {kw} stage_levels={sl:#x} generic={generic} node={node}")
        p = snd.Plan(f, dms, 0.138e-3, nsamp, mode=mode, cluster=C_, branching=B, stage_levels=sl,
                     generic_kernels=generic, node_dtype=node, **kw)
        if not generic and sl == 0 and nlev > 1:
            assert p.info["stage_kernel"][0] == "anchored", p.info["stage_kernel"]
            assert p.info["stage_kernel"][1] in ("group_lds", "group_fast", "group_bits", "group_lin"), \
                p.info["stage_kernel"]
        y = gpu_run(p, x, stage_by_stage=(sl == 0))
        assert y.shape == want.shape
        if mode == "float":
            assert rel_rms(y, want) <= FP32_TOL
        else:
            assert np.array_equal(y, want.astype(y.dtype))
        ys.append(y)
    if mode == "binary":
        # bit input (rows of bits straight from the encoder) where the tree takes bit rows
        try:
            pb = snd.Plan(f, dms, 0.138e-3, nsamp, mode=mode, cluster=C_, branching=B, in_dtype="bits", **kw)
        except snd.SndError as e:
            assert e.status == -2 and snd.Plan(f, dms, 0.138e-3, nsamp, mode=mode, cluster=C_, branching=B,
                                              **kw).node_dtype == "u8"
        else:
            _say(f"case nchan={nchan} C={C_} B={B} mode={mode} {kw} bit input")
            if nlev > 1:
                assert pb.info["stage_kernel"] == ["anchored_bits", "group_bits"], pb.info["stage_kernel"]
            y = gpu_run(pb, pack_bits(x), stage_by_stage=True)
            assert np.array_equal(y, want.astype(y.dtype))
            ys.append(y)
    for y in ys[1:]:
        if mode == "float":
            # float mode fixes no FP32 summation order: each schedule's plane is within the float
            # tolerance of the others (every one already is of the FP64 oracle)
            assert rel_rms(y, ys[0]) <= FP32_TOL
        else:
            assert np.array_equal(y, ys[0])  # identical whatever levels are materialised


def test_float_small_integer_input_is_exact(snd, orc):
    rng, f, dms, extra = _case(48, 40, 7)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, 48, int(d.max()) + extra, 3).astype(np.float32)
    want, _ = orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=4)
    p = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="float", branching=4)
    assert np.array_equal(gpu_run(p, x), want.astype(np.float32))
    pn = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="float", branching=4, root_norm=True)
    wn, _ = orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=4, root_norm=True)
    assert rel_rms(gpu_run(pn, x), wn) <= FP32_TOL


@pytest.mark.parametrize("node,B", [("f32", 4), ("bf16", 4), ("f16", 4), ("bf16", 8), ("f16", 3)])
def test_float_storage_small_integers_exact(snd, orc, node, B):
    """Small-integer float input (levels -3..4): leaf sums (|v| <= 16) are exact in bf16 and f16
    and the roots exact in FP32, so every storage type must reproduce the FP64 oracle bit for bit.  300 DMs
    fill five 64-row groups of the one-sum final stage (the last one partly), and 2600 output
    samples make two full 1024-sample tiles and a ragged one; random DMs give inputs of both
    dword phases on 16-bit rows."""
    rng, f, dms, _ = _case(96, 300, 11 + B)
    d = orc.delays(f, dms, 0.138e-3)
    x = (synth.random_levels(rng, 96, int(d.max()) + 2600, 7).astype(np.float32) - 3.0)
    want, _ = orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=B)
    p = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="float", branching=B, node_dtype=node)
    assert p.info["stage_kernel"] == ["anchored", "group_lin"], p.info["stage_kernel"]
    _say(f"small integers node={node} B={B} n_out={p.n_out}")
    assert p.n_out == x.shape[1] - int(d.max())
    y = gpu_run(p, x)
    assert np.array_equal(y, want.astype(np.float32))
    # the same leaf plane through the generic kernels
    pg = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="float", branching=B, node_dtype=node, generic_kernels=True)
    assert np.array_equal(gpu_run(pg, x), y)


@pytest.mark.parametrize("node", ["f32", "bf16", "f16"])
def test_float_rows_sum_error_bound(snd, orc, node):
    """Element-wise bound on the final stage's FP32 arithmetic.  One channel of every cluster of
    four carries values +-m 2^e (m < 256, e in -10..7), the others zero, so every leaf is exact in
    bf16 and f16 storage while the 128-input roots span 2^29 in magnitude and round.  Whatever the
    association, n roundings of at most one unit in the last place (round to nearest: half of
    one; the bf16 kernel's paired dots: one) keep |y - exact| <= n 2^-23 sum|x| with n = 128
    inputs per root; a dropped or foreign sample, or a non-sample half in a dot, breaks it.  300
    DMs and 2600 output samples: five 64-row groups, two full 1024-sample tiles and a ragged one."""
    rng, f, dms, _ = _case(512, 300, 71)
    d = orc.delays(f, dms, 0.138e-3)
    nsamp = int(d.max()) + 2600
    m = rng.integers(1, 256, (512, nsamp)).astype(np.float64)
    e = rng.integers(-10, 8, (512, nsamp)).astype(np.float64)
    x = (np.where(rng.random((512, nsamp)) < 0.5, -1.0, 1.0) * m * np.exp2(e)).astype(np.float32)
    x[np.arange(512) % 4 != 0] = 0.0
    want, _ = orc.snd_dedup(x, f, d, mode="float", cluster=4, branching=4)
    absum, _ = orc.snd_dedup(np.abs(x), f, d, mode="float", cluster=4, branching=4)
    p = snd.Plan(f, dms, 0.138e-3, nsamp, mode="float", branching=4, node_dtype=node)
    assert p.info["stage_kernel"] == ["anchored", "group_lin"], p.info["stage_kernel"]
    _say(f"float rows error bound node={node} n_out={p.n_out}")
    y = gpu_run(p, x).astype(np.float64)
    err = np.abs(y - want)
    bound = 128 * 2.0 ** -23 * absum
    assert np.all(np.isfinite(y))
    assert np.all(err <= bound), (float(np.max(err / np.maximum(bound, 1e-300))), np.argwhere(err > bound)[:5])
    assert np.any(err > 0)  # the roots do round


@pytest.mark.parametrize("nchan,B,cap,levels", [(1024, 4, 255, 4), (1024, 4, 3, 4), (256, 8, 255, 4),
                                                (512, 8, 7, 6), (64, 4, 2, 2), (4096, 4, 15, 4),
                                                (4096, 8, 255, 4)])
def test_graded_packed_levels_exact(snd, orc, nchan, B, cap, levels):
    """Graded u8 rows with level-1 nodes of 4 or 8 inputs run the packed kernel (two 16-bit
    counts per dword); small caps clip at every level.  Bit-exact against the oracle and the
    generic kernels, over 300 DMs (32-row groups over 1024-sample tiles at four inputs per node
    and depth <= 4, else 64-row groups over 512 samples; the last group partial in both) and
    2600 output samples (a ragged last tile in both)."""
    rng, f, dms, _ = _case(nchan, 300, 17 + B + cap)
    d = orc.delays(f, dms, 0.138e-3)
    x = synth.random_levels(rng, nchan, int(d.max()) + 2600, levels)
    want, _ = orc.snd_dedup(x, f, d, mode="graded", cluster=4, branching=B, cap=cap)
    p = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="graded", branching=B, cap=cap)
    assert p.info["stage_kernel"] == ["anchored", "group_pack"], p.info["stage_kernel"]
    _say(f"packed graded nchan={nchan} B={B} cap={cap} n_out={p.n_out}")
    y = gpu_run(p, x)
    assert np.array_equal(y, want.astype(y.dtype))
    pg = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode="graded", branching=B, cap=cap, generic_kernels=True)
    assert np.array_equal(gpu_run(pg, x), y)


@pytest.mark.parametrize("B,top,cap", [(4, 63, 255), (4, 64, 255), (4, 63, 100), (8, 31, 255), (8, 32, 60)])
def test_graded_packed_byte_sums_at_the_bound(snd, orc, B, top, cap):
    """The packed kernel adds a level-1 node's inputs as four bytes per dword when the leaf
    stage's largest value m has F1 m < 256 (F1 = B here), and as 16-bit counts otherwise.  The
    first F1 clusters carry leaves of exactly `top` over most of the block, so their level-1 node
    reaches F1 top: 252 or 248 on the byte path, 256 on the other.  The workspace starts filled
    with 0xFF, so row padding past the valid length holds the largest bytes.  Bit-exact against
    the oracle and the generic kernels, with a ragged last tile."""
    rng, f, dms, _ = _case(256, 300, 29 + B + top)
    d = orc.delays(f, dms, 0.138e-3)
    nsamp = int(d.max()) + 2600
    hi = (top - 3) // 4 if B == 4 else (top - 3) // 4 // 2 * 2
    x = synth.random_levels(rng, 256, nsamp, min(hi, 15))
    q, r = divmod(top, 4)  # channel values of one cluster summing to top
    per_cluster = [q + (1 if k < r else 0) for k in range(4)]
    for c in range(4 * B):
        x[c, 50:nsamp - 50] = per_cluster[c % 4]
    want, _ = orc.snd_dedup(x, f, d, mode="graded", cluster=4, branching=B, cap=cap)
    p = snd.Plan(f, dms, 0.138e-3, nsamp, mode="graded", branching=B, cap=cap)
    assert p.info["stage_kernel"] == ["anchored", "group_pack"], p.info["stage_kernel"]
    _say(f"packed byte sums B={B} top={top} cap={cap} n_out={p.n_out}")
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ws = p.workspace(xt.device)
    ws.fill_(255)
    out = p.empty_output(xt.device)
    p.execute(xt, out=out, workspace=ws)
    torch.cuda.synchronize()
    y = to_np(out)
    assert np.array_equal(y, want.astype(y.dtype))
    pg = snd.Plan(f, dms, 0.138e-3, nsamp, mode="graded", branching=B, cap=cap, generic_kernels=True)
    assert np.array_equal(gpu_run(pg, x), y)


@pytest.mark.parametrize("mode,node", [("float", "f32"), ("float", "bf16"), ("graded", "u8"), ("binary", "bits"),
                                       ("binary", "u8")])
def test_tune_variants_identical(snd, orc, mode, node):
    """Every launch shape of snd_plan_desc.tune (leaf window, XCD dealing, LDS batch budget)
    computes the same plane bit for bit, equal to the oracle's (float: within FP32 tolerance; f32
    rows bit for bit while the final stage keeps its kernel)."""
    rng, f, dms, _ = _case(256, 300, 23)
    d = orc.delays(f, dms, 0.138e-3)
    x = _inputs(rng, mode, 256, int(d.max()) + 3000)
    kw = dict(k_leaf=2, k_int=1) if mode == "binary" else {}
    want, _ = orc.snd_dedup(x, f, d, mode=mode, cluster=4, branching=4, **kw)
    tw = snd.tune_word
    base = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode=mode, branching=4, node_dtype=node, **kw)
    y0 = gpu_run(base, x)
    if mode == "float":
        assert rel_rms(y0, want) <= (FP32_TOL if node == "f32" else REDUCED_TOL)
    else:
        assert np.array_equal(y0, want.astype(y0.dtype))
    for t in (tw(xcd_groups=1), tw(xcd_groups=2), tw(xcd_groups=16), tw(lds_quarters_off=1), tw(lds_quarters_off=3),
              tw(leaf_window=512), tw(leaf_window=1024), tw(leaf_window=2048, xcd_groups=4, lds_quarters_off=2)):
        _say(f"tune mode={mode} node={node} tune={t:#x}")
        p = snd.Plan(f, dms, 0.138e-3, x.shape[1], mode=mode, branching=4, node_dtype=node, tune=t, **kw)
        y = gpu_run(p, x)
        if mode == "float" and (node != "f32" or p.info["stage_kernel"] != base.info["stage_kernel"]):
            # the one-sum kernel on 16-bit rows adds each batch's inputs grouped by dword phase,
            # so other batch boundaries associate differently; and a budget too small for its
            # batches moves the stage to a kernel that sums in the tree's association: the same
            # plane within FP32 rounding
            assert rel_rms(y, y0) <= FP32_TOL, snd.tune_fields(t)
        else:
            assert np.array_equal(y, y0), snd.tune_fields(t)


def test_encoder_parity(snd, orc):
    spec = synth.workload(1)
    z = spec.filterbank()
    zt = torch.from_numpy(z).cuda()
    for thr in ([2.0], [1.0, 2.0, 3.0, 4.0], [0.75]):
        _say(f"encode thresholds={thr}")
        a = to_np(snd.encode(zt, thr))
        b = to_np(snd.encode(zt.t().contiguous(), thr, time_major=True))
        want = orc.encode(z, thr)
        assert np.array_equal(a, want) and np.array_equal(b, want)


def test_encoder_bits_parity(snd, orc):
    spec = synth.workload(1)
    z = spec.filterbank()
    zt = torch.from_numpy(z).cuda()
    for thr, n in ((2.0, z.shape[1]), (0.75, z.shape[1]), (1.0, 1000), (1.5, 1)):
        _say(f"encode_bits threshold={thr} nsamp={n}")
        want = pack_bits(orc.encode(z[:, :n], [thr]))
        a = snd.encode_bits(zt[:, :n], thr).cpu().numpy()
        b = snd.encode_bits(zt[:, :n].t().contiguous(), thr, time_major=True).cpu().numpy()
        assert np.array_equal(a, want) and np.array_equal(b, want)


def test_encoders_at_exact_thresholds(snd, orc):
    # samples exactly at a threshold do not fire (x = 1[z > theta]); the float just above does
    rng = synth.make_rng(77)
    thr = [0.75, 1.5, 2.0, 3.0]
    t32 = np.array(thr, dtype=np.float32)
    vals = np.concatenate([t32, np.nextafter(t32, np.float32(np.inf)), np.nextafter(t32, np.float32(-np.inf))])
    z = rng.choice(vals, size=(5, 4100)).astype(np.float32)
    zt = torch.from_numpy(z).cuda()
    for th in ([2.0], [1.0, 2.0, 3.0, 4.0], [0.75, 1.5]):
        _say(f"encode at exact thresholds {th}")
        want = orc.encode(z, th)
        assert np.array_equal(to_np(snd.encode(zt, th)), want)
        assert np.array_equal(to_np(snd.encode(zt.t().contiguous(), th, time_major=True)), want)
    for th in thr:
        want = pack_bits(orc.encode(z, [th]))
        assert np.array_equal(snd.encode_bits(zt, th).cpu().numpy(), want)
        assert np.array_equal(snd.encode_bits(zt.t().contiguous(), th, time_major=True).cpu().numpy(), want)


@pytest.mark.parametrize("kl,ki", [(2, 2), (2, 1)])
def test_config1_binary_exact(snd, orc, kl, ki):
    spec = synth.workload(1)
    z = spec.filterbank()
    x = to_np(snd.encode(torch.from_numpy(z).cuda(), list(spec.enc_thresholds)))
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    want, counts = orc.snd_dedup(x, spec.freqs, d, mode="binary", cluster=4, branching=2, k_leaf=kl, k_int=ki)
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="binary", branching=2, k_leaf=kl, k_int=ki)
    assert p.info["n_neurons"] == sum(c[0] for c in counts) == 1984
    assert p.node_dtype == "bits" and p.info["stage_kernel"] == ["anchored", "group_bits"]
    assert np.array_equal(gpu_run(p, x), want.astype(np.uint8))
    pb = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="binary", branching=2, k_leaf=kl, k_int=ki,
                  node_dtype="u8")
    assert pb.info["stage_kernel"] == ["anchored", "group_fast"]
    assert np.array_equal(gpu_run(pb, x), want.astype(np.uint8))
    if len(spec.enc_thresholds) == 1:  # bit input from the bit encoder
        xb = snd.encode_bits(torch.from_numpy(z).cuda(), spec.enc_thresholds[0])
        pi = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode="binary", branching=2, k_leaf=kl,
                      k_int=ki, in_dtype="bits")
        assert pi.info["stage_kernel"] == ["anchored_bits", "group_bits"]
        y = pi.execute(xb)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(y), want.astype(np.uint8))


@pytest.mark.parametrize("B", [2, 4, 8])
@pytest.mark.parametrize("mode", ["binary", "graded", "float"])
def test_config3_modes_exact(snd, orc, B, mode):
    # the 64-channel geometric 3000-trial grid, n_out shortened to keep the oracle fast
    spec = synth.workload(3, mode=mode, branching=B)
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    nsamp = int(d.max()) + 1500
    z = spec.filterbank(nsamp)
    if mode == "float":
        x = z
    else:
        x = orc.encode(z, list(spec.enc_thresholds))
    kw = dict(k_leaf=spec.k_leaf, k_int=spec.k_int) if mode == "binary" else {}
    for cap in ((255, 15) if mode == "graded" else (255,)):
        _say(f"config3 mode={mode} B={B} cap={cap}")
        want, _ = orc.snd_dedup(x, spec.freqs, d, mode=mode, cluster=4, branching=B, cap=cap, **kw)
        p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, nsamp, mode=mode, branching=B, cap=cap, **kw)
        y = gpu_run(p, x)
        if mode == "float":
            assert rel_rms(y, want) <= FP32_TOL
        else:
            assert np.array_equal(y, want.astype(y.dtype))


@pytest.mark.parametrize("node,inp", [("bf16", "f32"), ("f16", "f32"), ("bf16", "bf16"), ("f16", "f16")])
def test_reduced_precision_storage(snd, orc, node, inp):
    rng, f, dms, extra = _case(64, 50, 99)
    d = orc.delays(f, dms, 0.138e-3)
    z = synth.noise_filterbank(rng, 64, int(d.max()) + extra)
    want, _ = orc.snd_dedup(z, f, d, mode="float", cluster=4, branching=4)
    p = snd.Plan(f, dms, 0.138e-3, z.shape[1], mode="float", branching=4, in_dtype=inp, node_dtype=node)
    zt = torch.from_numpy(z).cuda()
    xin = zt if inp == "f32" else snd.cast(zt, inp)
    if inp != "f32":
        ref = xin.float().cpu() if inp == "bf16" else xin.float().cpu()
        cpu_cast = zt.cpu().to(torch.bfloat16 if inp == "bf16" else torch.float16).float()
        assert torch.equal(ref, cpu_cast)  # round-to-nearest-even like torch's own cast
    y = p.execute(xin)
    torch.cuda.synchronize()
    err = rel_rms(to_np(y), want)
    _say(f"storage node={node} in={inp} rel_rms={err:.3e}")
    assert err <= REDUCED_TOL


def test_edge_cases(snd, orc):
    f = synth.channel_freqs(40)
    rng = synth.make_rng(5)
    # all-zero DM grid: no delay, n_out = nsamp; duplicate rows identical
    x = synth.random_levels(rng, 40, 300, 4)
    p = snd.Plan(f, [0.0, 0.0, 0.0], 0.138e-3, 300, mode="graded", branching=2, cap=6)
    y = gpu_run(p, x)
    assert y.shape == (3, 300)
    assert np.array_equal(y[0], np.minimum(x.sum(0), 6)) and np.array_equal(y[0], y[2])
    # single DM, single channel
    p1 = snd.Plan([400.0], [100.0], 0.138e-3, 70, mode="float", branching=2, cluster=1)
    x1 = rng.standard_normal((1, 70)).astype(np.float32)
    assert np.array_equal(gpu_run(p1, x1), x1[:, :70])
    # unsorted DMs: rows follow the caller's order
    dms = np.array([30.0, 0.0, 15.0, 30.0])
    d = orc.delays(f, dms, 0.138e-3)
    x2 = synth.random_spikes(rng, 40, int(d.max()) + 600, 0.4)
    p2 = snd.Plan(f, dms, 0.138e-3, x2.shape[1], mode="binary", branching=3, k_leaf=1, k_int=2)
    want, _ = orc.snd_dedup(x2, f, d, mode="binary", cluster=4, branching=3, k_leaf=1, k_int=2)
    y2 = gpu_run(p2, x2)
    assert np.array_equal(y2, want.astype(np.uint8)) and np.array_equal(y2[0], y2[3])
    # a pitched input (extra columns) gives the same answer
    xt = torch.zeros((40, x2.shape[1] + 77), dtype=torch.uint8, device="cuda")
    xt[:, : x2.shape[1]] = torch.from_numpy(x2).cuda()
    y3 = to_np(p2.execute(xt))
    assert np.array_equal(y3, y2)


def test_bad_arguments_raise(snd):
    p = snd.Plan(synth.channel_freqs(8), [0.0, 2.0], 0.138e-3, 200, mode="float", branching=2)
    with pytest.raises(ValueError):
        p.execute(torch.zeros((8, 100), device="cuda"))
    with pytest.raises(TypeError):
        p.execute(torch.zeros((8, 200), dtype=torch.uint8, device="cuda"))


def test_determinism(snd):
    rng, f, dms, extra = _case(128, 64, 3)
    p = snd.Plan(f, dms, 0.138e-3, 4000, mode="float", branching=4)
    z = synth.noise_filterbank(rng, 128, 4000)
    a = gpu_run(p, z)
    b = gpu_run(p, z)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("mode", ["float", "graded", "binary", "binary-bits"])
def test_config2_full_size_sampled(snd, orc, mode):
    # The benchmarked workload (1024 ch, 4096 DM, 2^17 samples, B = 4) at full size, checked
    # on sampled outputs against the oracle's per-point recursion.
    spec = synth.workload(2)
    _say(f"config2 full size mode={mode}: generating input")
    z = spec.filterbank()
    d = orc.delays(spec.freqs, spec.dms, spec.tsamp_s)
    zt = torch.from_numpy(z).cuda()
    bit_input = mode == "binary-bits"
    mode = "binary" if bit_input else mode
    if mode == "float":
        x, xin = z, zt
    else:
        xin = snd.encode(zt, [1.0, 2.0, 3.0, 4.0] if mode == "graded" else [2.0])
        x = to_np(xin)
    if bit_input:
        xin = snd.encode_bits(zt, 2.0)
        assert np.array_equal(xin[:, :64].cpu().numpy(), pack_bits(x[:, :2048]))
    p = snd.Plan(spec.freqs, spec.dms, spec.tsamp_s, spec.nsamp, mode=mode, branching=4,
                 in_dtype="bits" if bit_input else None)
    if mode == "binary":
        assert p.info["stage_kernel"] == ["anchored_bits" if bit_input else "anchored", "group_bits"]
    _say(f"config2 mode={mode}: executing on the GPU")
    y = p.execute(xin)
    torch.cuda.synchronize()
    rng = synth.make_rng(77)
    n = 3000
    ks = rng.integers(0, spec.dms.size, n)
    ts = rng.integers(0, p.n_out, n)
    ks[:4] = [0, spec.dms.size - 1, 0, spec.dms.size - 1]
    ts[:4] = [0, 0, p.n_out - 1, p.n_out - 1]
    got = to_np(y[torch.from_numpy(ks).cuda(), torch.from_numpy(ts).cuda()])
    want = orc.snd_points(x, spec.freqs, d, ks, ts, mode=mode, cluster=4, branching=4)
    if mode == "float":
        assert rel_rms(got, want) <= FP32_TOL
    else:
        assert np.array_equal(got, want.astype(got.dtype))
    # DM 0 row is the plain channel sum
    if mode == "graded":
        row0 = to_np(y[0, :2000])
        assert np.array_equal(row0, np.minimum(x[:, :2000].astype(np.int64).sum(0), 255))
