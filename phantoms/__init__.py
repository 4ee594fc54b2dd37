"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds only input generation: optical-property pixel maps,
source descriptions and detector / adjoint-source maps.  It contains none of
the Monte Carlo arithmetic, so both the GPU path and the CPU oracle can
consume its outputs without sharing any of the method's code.
"""
from .phantoms import (  # noqa: F401
    Phantom, SourceSpec, homogeneous, disc_phantom, pencil_top_centre, four_side_lines,
    point_source, map_source, config1, config2, residual_like_map, interior_pixels,
    lambertian_boundary, two_inclusion_phantom, smooth_hmeas, Config,
)
