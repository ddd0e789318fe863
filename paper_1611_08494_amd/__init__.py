"""MI355X positional cross-match (the C^3 tool, arXiv:1611.08494).

Python face of libc3x.so: ``build_index`` over catalogue B and ``match`` of
catalogue A against it (the "Sky" case: circle, per-source ellipse or
rectangle areas, "all" and "best" selections, equatorial or galactic
frames); ``match_concentric`` for ClumpPopulator's concentric ellipses
(Section 3); ``unmatched`` and ``join`` for the join types of Section 2.2
(rows without a stored match); ``mutual`` for the symmetric best pairs (each
other's nearest match); ``Batch`` for many independent circular jobs in one
graph launch; ``exact_match`` for the Exact Value case (equal values of one
column each); ``frame_convert`` for the conversion rule applied to a
catalogue given in the other frame. All computation happens in the HIP
library; torch tensors only carry device memory and streams.
"""
from ._binding import (  # noqa: F401
    ALL,
    BEST,
    Batch,
    CIRCLE,
    ELLIPSE,
    EQUATORIAL,
    FP64,
    GALACTIC,
    LIB_PATH,
    MIXED,
    RECT,
    C3XError,
    Index,
    MatchResult,
    JOIN_PARTS,
    build_index,
    cross_match,
    exact_match,
    frame_convert,
    frame_matrix,
    join,
    lib,
    match,
    match_concentric,
    mutual,
    result_copy,
    unmatched,
    version,
)
