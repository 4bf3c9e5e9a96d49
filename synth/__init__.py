"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws inputs: channel frequencies, trial-DM grids, Gaussian noise
filterbanks with injected dispersed pulses, random spike rasters and random level
rasters.  It performs none of the dedispersion method's arithmetic (no delay
rounding, no tree, no encoding, no matched filter); both sides of every parity
check compute those from the arrays drawn here.
"""

from .filterbank import (  # noqa: F401
    KDM_MS,
    Pulse,
    channel_freqs,
    dm_linear,
    dm_geometric,
    make_rng,
    noise_filterbank,
    inject_pulses,
    random_pulses,
    random_spikes,
    random_levels,
    random_pulse_slots,
)
from .configs import (  # noqa: F401
    TSAMP_S,
    WorkloadSpec,
    workload,
    WORKLOADS,
    batch_beam,
    stream_beam,
    arrival_times,
    chunk_period_s,
    seed_for,
)
