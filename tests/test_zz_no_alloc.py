"""snd_detect_launch_noalloc through the C ABI: the same staged cells and candidates as
snd_detect_launch with a caller workspace, on two calls in a row, the second on a smaller plane
(the library's fixed device array then still holds the first call's contents)."""

import ctypes as C
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[no-alloc] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def snd():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2606_15361_amd as m
    return m


def _desc(capi, widths):
    d = capi.DetectDesc()
    d.widths = widths.ctypes.data_as(C.POINTER(C.c_int32))
    d.nwidths = widths.size
    d.threshold = 3.0
    d.sigma_min = 0.0
    d.closing_radius = 2
    d.n_min = 1
    d.max_pixels = 200000
    return d


def _staged(capi, plan, desc, stage, nb):
    """(thresholded-cell count, staged cells sorted by (k, t), candidates) of a completed launch."""
    count = int(np.frombuffer(bytes(stage[:4].numpy()), dtype=np.uint32)[0])
    cells = stage[capi.DETECT_STAGE_HEADER: capi.DETECT_STAGE_HEADER + 24 * count].numpy().copy()
    rec = cells.view(np.dtype([("k", "<i4"), ("t", "<i4"), ("snr", "<f8"), ("widx", "<i4"), ("pad", "<i4")]))
    rec = np.sort(rec[["k", "t", "snr", "widx"]], order=("k", "t"))
    buf = (capi.Candidate * 4096)()
    cnt, npx = C.c_int64(), C.c_int64()
    capi.check(capi.lib().snd_detect_collect(plan.handle, C.byref(desc), C.c_void_p(stage.data_ptr()), nb, buf, 4096,
                                             C.byref(cnt), C.byref(npx)))
    assert npx.value == count
    cands = [(buf[i].dm_index, buf[i].t, buf[i].width, buf[i].snr, buf[i].npix) for i in range(cnt.value)]
    return count, rec, cands


def test_noalloc_launch_equals_workspace_launch(snd):
    from paper_2606_15361_amd import _capi as capi
    lib = capi.lib()
    spec = synth.workload(1)
    z = spec.filterbank()
    widths = np.array([1, 2, 4, 8, 16], dtype=np.int32)
    cases = [("64 DMs x 8192 samples", spec.dms, spec.nsamp), ("24 DMs x 4096 samples", spec.dms[:24] * 0.5, 4096)]
    stream = torch.cuda.current_stream()
    sh = C.c_void_p(stream.cuda_stream)
    for name, dms, nsamp in cases:
        _say(f"plane {name}")
        plan = snd.Plan(spec.freqs, dms, spec.tsamp_s, nsamp, mode="float", branching=2)
        plane = plan.execute(torch.from_numpy(z[:, :nsamp]).cuda())
        desc = _desc(capi, widths)
        need = C.c_int64()
        capi.check(lib.snd_detect_workspace(plan.handle, C.byref(desc), C.byref(need)))
        assert need.value <= capi.DETECT_NOALLOC_MAX_BYTES
        ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        nb = capi.DETECT_STAGE_HEADER + 24 * desc.max_pixels
        st_ref = torch.zeros(nb, dtype=torch.uint8, pin_memory=True)
        st_new = torch.zeros(nb, dtype=torch.uint8, pin_memory=True)
        capi.check(lib.snd_detect_launch(plan.handle, C.c_void_p(plane.data_ptr()), plane.stride(0), C.byref(desc),
                                         C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(st_ref.data_ptr()), nb, sh))
        torch.cuda.synchronize()
        want = _staged(capi, plan, desc, st_ref, nb)
        capi.check(lib.snd_detect_launch_noalloc(plan.handle, C.c_void_p(plane.data_ptr()), plane.stride(0),
                                                 C.byref(desc), C.c_void_p(st_new.data_ptr()), nb, sh))
        torch.cuda.synchronize()
        got = _staged(capi, plan, desc, st_new, nb)
        _say(f"{name}: {want[0]} cells, {len(want[2])} candidates")
        assert want[0] >= 20 and len(want[2]) >= 1
        assert got[0] == want[0]
        assert np.array_equal(got[1], want[1])
        assert got[2] == want[2]
