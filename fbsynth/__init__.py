"""Seeded synthetic filterbank workloads shared by the tests, the smoke check and the benchmark.

This package only draws inputs (noise, dispersed pulses from a sky model,
quantisation to storage types, arrival schedules). It holds none of the
dedispersion method's arithmetic: no integer delay table and no channel sums.
"""
from .filterbank import (  # noqa: F401
    Beam, Pulse, channel_freqs, dm_trials, sky_delay_s, noise, inject_boxcar,
    to_u8, to_f16, config1, config2, config3, config4_specs, make_beam,
    config5_specs, arrival_times, U8_OFFSET, U8_SCALE,
)
