"""MI355X (gfx950) implementation of the radio ray tracer of arXiv 2303.11103.

The computation runs in the HIP library ``librt_mi355x.so`` (C ABI in
``include/rt.h``); this package only marshals arguments.  Importing it without
the built library raises ImportError.
"""
from . import _lib  # noqa: F401  (raises if the library is missing)
from .rt import (Context, Scene, TraceParams, combine_paths, compute_paths, coverage_map, coverage_maps,  # noqa: F401
                 compute_diffraction, compute_scattering, coverage_diffraction, fibonacci_directions,
                 coverage_grad, last_candidate_count, paths_cfr, paths_cfr_adjoint, paths_coef_grad, paths_power,
                 paths_power_grad, trace_record)
