"""ctypes declarations of include/snd.h.  Argument marshalling only."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnd.so")

MAX_LEVELS = 32
STAGE_NONE = 0x80000000

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_NOMEM, ERR_HIP, ERR_CAPACITY, ERR_STATE, ERR_GAP = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "SND_OK", -1: "SND_ERR_INVALID", -2: "SND_ERR_UNSUPPORTED", -3: "SND_ERR_NOMEM",
                -4: "SND_ERR_HIP", -5: "SND_ERR_CAPACITY", -6: "SND_ERR_STATE", -7: "SND_ERR_GAP"}
MODE_BINARY, MODE_GRADED, MODE_FLOAT = 0, 1, 2
DT_U8, DT_U16, DT_F32, DT_BF16, DT_F16, DT_BITS = 1, 2, 3, 4, 5, 6


DETECT_STAGE_HEADER = 256  # SND_DETECT_STAGE_HEADER
DETECT_CELL_BYTES = 24    # bytes per staged cell
DETECT_NOALLOC_MAX_BYTES = 32 << 20  # SND_DETECT_NOALLOC_MAX_BYTES


class SndError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class PlanDesc(C.Structure):
    _fields_ = [
        ("nchan", C.c_int32), ("freq_mhz", C.POINTER(C.c_double)), ("tsamp_s", C.c_double),
        ("fref_mhz", C.c_double), ("ndm", C.c_int32), ("dm", C.POINTER(C.c_double)),
        ("branching", C.c_int32), ("cluster", C.c_int32), ("mode", C.c_int32), ("k_leaf", C.c_int32),
        ("k_int", C.c_int32), ("cap", C.c_int32), ("in_dtype", C.c_int32), ("node_dtype", C.c_int32),
        ("root_norm", C.c_int32), ("nsamp", C.c_int64), ("stage_levels", C.c_uint32),
        ("generic_kernels", C.c_int32), ("chunk", C.c_int32), ("tune", C.c_uint32), ("reserved", C.c_int32 * 5),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n_out", C.c_int64), ("max_delay", C.c_int64), ("n_levels", C.c_int32), ("n_stages", C.c_int32),
        ("out_dtype", C.c_int32), ("pad0", C.c_int32), ("n_neurons", C.c_int64), ("n_synapses", C.c_int64),
        ("neurons_per_level", C.c_int64 * MAX_LEVELS), ("synapses_per_level", C.c_int64 * MAX_LEVELS),
        ("nodes_per_level", C.c_int64 * MAX_LEVELS), ("table_bytes", C.c_int64), ("workspace_bytes", C.c_int64),
        ("alg_bytes", C.c_int64), ("stage_alg_bytes", C.c_int64 * MAX_LEVELS),
        ("stage_rows", C.c_int64 * MAX_LEVELS), ("stage_entries", C.c_int64 * MAX_LEVELS),
        ("build_seconds", C.c_double), ("stage_kernel", C.c_int32 * MAX_LEVELS),
        ("stage_staged", C.c_int64 * MAX_LEVELS), ("stage_batches", C.c_int64 * MAX_LEVELS),
        ("stage_windows", C.c_int64 * MAX_LEVELS),
    ]


class DetectDesc(C.Structure):
    _fields_ = [("widths", C.POINTER(C.c_int32)), ("nwidths", C.c_int32), ("closing_radius", C.c_int32),
                ("threshold", C.c_double), ("sigma_min", C.c_double), ("n_min", C.c_int32),
                ("n_base_widths", C.c_int32), ("max_pixels", C.c_int64), ("width_alpha", C.c_double),
                ("sigma_estimator", C.c_int32), ("label_on_device", C.c_int32)]


class BandCandidate(C.Structure):
    _fields_ = [("dm", C.c_double), ("t_ms", C.c_double), ("snr", C.c_double), ("band", C.c_int32),
                ("dm_index", C.c_int32), ("width", C.c_int32), ("reserved", C.c_int32), ("t", C.c_int64),
                ("npix", C.c_int64)]


class Candidate(C.Structure):
    _fields_ = [("dm_index", C.c_int32), ("width", C.c_int32), ("t", C.c_int64), ("snr", C.c_double),
                ("dm", C.c_double), ("npix", C.c_int64)]


class StreamItem(C.Structure):
    _fields_ = [("beam_id", C.c_int32), ("status", C.c_int32), ("chunk_idx", C.c_int64), ("chunk_len", C.c_int64),
                ("d_chunk", C.c_void_p), ("chunk_pitch", C.c_int64), ("d_out", C.c_void_p), ("out_pitch", C.c_int64),
                ("out_t0", C.c_int64), ("out_n", C.c_int64)]


class TuneCandidate(C.Structure):
    _fields_ = [("stage_levels", C.c_uint32), ("chunk", C.c_int32), ("tune", C.c_uint32), ("pad", C.c_int32),
                ("ms", C.c_double),
                ("workspace_bytes", C.c_int64), ("table_bytes", C.c_int64)]


_lib = None


def declared_symbols(header: str) -> list:
    import re
    text = open(header).read()
    return sorted(set(re.findall(r"\b(snd_[a-z_0-9]+)\s*\(", text)))


def lib() -> C.CDLL:
    """Load libsnd.so.  torch is imported first so that this library binds to the same HIP
    runtime (libamdhip64.so.7) as torch; there is no fallback when the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (shares its HIP runtime with libsnd)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2606_15361_amd.build` "
                           "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    I64, I32 = C.c_int64, C.c_int32
    sig = {
        "snd_plan_create": ([C.POINTER(PlanDesc), C.POINTER(P)], I32),
        "snd_plan_query": ([P, C.POINTER(PlanInfo)], I32),
        "snd_plan_delays": ([P, P, I64], I32),
        "snd_plan_upload": ([P, P, I64, P], I32),
        "snd_plan_destroy": ([P], I32),
        "snd_execute": ([P, P, I64, P, I64, P, I64, P], I32),
        "snd_execute_stage": ([P, I32, P, I64, P, I64, P, I64, P], I32),
        "snd_encode": ([P, I64, I32, I32, I64, P, I32, P, I64, P], I32),
        "snd_encode_bits": ([P, I64, I32, I32, I64, C.c_float, P, I64, P], I32),
        "snd_cast": ([P, I64, I64, I64, P, I64, I32, P], I32),
        "snd_channel_stats": ([P, I64, I32, I64, C.c_double, P, P], I32),
        "snd_normalize": ([P, I64, I32, I64, P, P, I64, P], I32),
        "snd_zero_dm": ([P, I64, I32, I64, C.c_double, P, P], I32),
        "snd_flag_channels": ([P, I64, I32, I64, I64, C.c_double, P, P, I64, P], I32),
        "snd_scrunch_factors": ([I32, P, C.c_double, I32, P, I32, P], I32),
        "snd_scrunch": ([P, I64, I32, I64, I32, P, I64, P], I32),
        "snd_merge_candidates": ([I64, P, C.c_double, C.c_double, P, C.POINTER(I64)], I32),
        "snd_effective_width": ([I32, P, C.c_double, I64, P, P, P], I32),
        "snd_fdmt_create": ([I32, P, C.c_double, C.c_double, C.c_double, I64, C.POINTER(P)], I32),
        "snd_fdmt_query": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64),
                            C.POINTER(C.c_double)], I32),
        "snd_fdmt_upload": ([P, P, I64, P], I32),
        "snd_fdmt_execute": ([P, P, I64, P, I64, P, I64, P], I32),
        "snd_fdmt_destroy": ([P], I32),
        "snd_subband_workspace_bytes": ([I32, I32, C.POINTER(I64)], I32),
        "snd_subband_combine": ([I32, I32, P, P, P, I32, P, P, P, I64, I64, P, I64, P], I32),
        "snd_match_injections": ([I64, P, P, P, I64, P, P, P, C.c_double, C.c_double, P, C.POINTER(I64)], I32),
        "snd_last_error": ([], C.c_char_p),
        "snd_version": ([], C.c_char_p),
    }
    D = C.POINTER(DetectDesc)
    sig.update({
        "snd_detect_workspace": ([P, D, C.POINTER(I64)], I32),
        "snd_snr_plane": ([P, P, I64, D, P, I64, P, I64, P, I64, P], I32),
        "snd_detect": ([P, P, I64, D, P, I64, C.POINTER(Candidate), I64, C.POINTER(I64), C.POINTER(I64), P], I32),
        "snd_detect_launch": ([P, P, I64, D, P, I64, P, I64, P], I32),
        "snd_detect_collect": ([P, D, P, I64, C.POINTER(Candidate), I64, C.POINTER(I64), C.POINTER(I64)], I32),
        "snd_detect_batch_workspace": ([I32, P, D, C.POINTER(I64)], I32),
        "snd_detect_batch_launch": ([I32, P, P, P, D, P, I64, P, I64, P], I32),
        "snd_detect_batch_collect": ([I32, P, D, P, I64, C.POINTER(Candidate), I64, P, P], I32),
        "snd_detect_launch_noalloc": ([P, P, I64, D, P, I64, P], I32),
    })
    PI64 = C.POINTER(I64)
    PP = C.POINTER(P)
    sig.update({
        "snd_autotune": ([C.POINTER(PlanDesc), C.POINTER(TuneCandidate), I32, P, I64, P, I64, P, I64, P, I64, I32,
                          C.POINTER(I32), P], I32),
        "snd_batch_records_bytes": ([I32, PP, PI64, C.POINTER(I32)], I32),
        "snd_batch_execute": ([I32, PP, PP, PI64, PP, PI64, PP, PI64, PI64, P, I64, P, C.POINTER(I32)], I32),
        "snd_stream_history_bytes": ([P, PI64], I32),
        "snd_stream_admission_bytes": ([P, PI64], I32),
        "snd_stream_create": ([I64, C.POINTER(P)], I32),
        "snd_stream_destroy": ([P], I32),
        "snd_stream_admit": ([P, I32, P, P, I64], I32),
        "snd_stream_evict": ([P, I32], I32),
        "snd_stream_push": ([P, I32, C.POINTER(StreamItem), P, I64, P], I32),
        "snd_stream_push_batched": ([P, I32, C.POINTER(StreamItem), P, I64, P, I64, P], I32),
        "snd_stream_batch_bytes": ([P, I32, C.POINTER(I32), PI64, PI64], I32),
        "snd_stream_beam_state": ([P, I32, PI64, PI64, PI64], I32),
        "snd_stream_usage": ([P, PI64, PI64, C.POINTER(I32)], I32),
        "snd_stream_export_bytes": ([P, I32, PI64], I32),
        "snd_stream_export": ([P, I32, P, I64, P], I32),
        "snd_stream_import": ([P, I32, P, I64, P], I32),
    })
    optional = {}
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    for name, (args, res) in optional.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != OK:
        raise SndError(rc, lib().snd_last_error().decode())
