"""MI355X brute-force incoherent dedispersion (Magro 2013, Ch. 2-3) behind a C ABI.

The compute path is libdedisp.so (HIP kernels for gfx950, include/dedisp.h);
this package is its ctypes binding plus torch plumbing for device memory and
streams.
"""
from ._lib import LibraryMissing, DedispError, load as load_library  # noqa: F401
from .api import (Plan, Stream, Result, CandidateOverflow, CAND_DTYPE, PULSE_DTYPE,  # noqa: F401
                  batch_dedisperse, detrend, boxcar, boxcar_search, downfactor, time_binning,
                  BinnedPlan, BinnedResult, BinnedStream, BinnedStreamResult, bandpass, bandpass_fit,
                  rfi_mitigate, SubbandPlan)

__version__ = "1.5"
