"""MI355X (gfx950) Hermite-4 block-time-step N-body path after GraviDy (arXiv:1702.00440).

The compute runs in libgravidy_hip.so (C ABI: include/gravidy_hip.h); the
binding in .gravidy only marshals arguments. Importing this package does not
load the library; the first call into .gravidy does, and fails loudly if it is
not built.
"""
from .build import build  # noqa: F401

__all__ = ["build"]
