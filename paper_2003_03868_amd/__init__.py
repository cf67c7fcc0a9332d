"""bsm: block-sparse matrix multiply and Newton-Schulz sign iteration for
AMD MI355X (gfx950), as a C-ABI HIP library (``libbsm.so``) with a thin
Python binding (:mod:`paper_2003_03868_amd.bsm`)."""
from . import bsm  # noqa: F401

__all__ = ["bsm"]
