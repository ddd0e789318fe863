"""Seeded synthetic catalogues for the positional cross-match.

This package only draws input positions and area parameters. It holds none of
the cross-match arithmetic (no distances, no region tests), so both the CPU
oracle's tests and the GPU path's tests and benchmark can share it.
"""
from .catalogues import (  # noqa: F401
    Catalogues,
    area_uniform,
    cap_uniform,
    destination,
    jitter,
    sphere_uniform,
    cfg1_patch,
    cfg2_fullsky,
    cfg3_galactic_ellipses,
    cfg4_jobs,
    cfg5_scale,
    adversarial_circle,
    SEED_BASE,
)
