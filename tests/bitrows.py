"""Bit-row packing for the tests: the layout of the library's BITS storage, written with numpy."""

import numpy as np


def pack_bits(x):
    """Spike rows [nchan][nsamp] (non-zero = spike) as bit rows: int32 [nchan][words], bit i
    of word w = sample 32 w + i, words a multiple of 4."""
    nchan, nsamp = x.shape
    nw = (nsamp + 127) // 128 * 4
    b = np.packbits(np.asarray(x) != 0, axis=1, bitorder="little")
    out = np.zeros((nchan, nw * 4), dtype=np.uint8)
    out[:, : b.shape[1]] = b
    return out.view("<u4").view(np.int32)
