"""MI355X-native Spiking Neural Dedispersion (SND).

The compute path is libsnd.so: a C-ABI library (include/snd.h) whose plan builder runs on
the host and whose tree, encoder and detection stages are hand-written HIP kernels for
gfx950.  This package is the thin Python binding used by the tests and the benchmark;
PyTorch only provides device memory and HIP streams.
"""

from ._capi import SndError, LIB_PATH  # noqa: F401
from .plan import Plan, autotune, autotune_cached, tune_word, tune_fields, encode, encode_bits, cast, channel_stats, normalize, zero_dm, flag_channels  # noqa: F401,E501
from .detect import Detector, BatchDetector  # noqa: F401
from .stream import Stream, admission_bytes, history_bytes  # noqa: F401
from .batch import Batch, records_bytes  # noqa: F401
from .multirate import MultiRate, scrunch, scrunch_factors, merge_candidates  # noqa: F401
from .validate import effective_width, match_injections  # noqa: F401
from .fdmt import Fdmt  # noqa: F401
from .subband import SubbandApprox  # noqa: F401

__all__ = ["Plan", "autotune", "autotune_cached", "tune_word", "tune_fields", "Detector", "BatchDetector", "Stream", "Batch", "history_bytes", "admission_bytes", "records_bytes", "encode", "encode_bits",
           "cast", "channel_stats", "normalize", "zero_dm", "flag_channels", "MultiRate", "scrunch", "scrunch_factors", "merge_candidates",
           "effective_width", "match_injections", "Fdmt", "SubbandApprox", "SndError", "LIB_PATH"]
