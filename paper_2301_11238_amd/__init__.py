"""MI355X (gfx950) library for the regularised-Bingham shallow-water DG method
(Fernandez, Lopez-Ordonez, Gonzalez-Andrade, arXiv 2301.11238).

The hot path -- the DG spatial operator, its element-block Jacobian, the stage
update and the Newton / GMRES solve -- runs in hand-written HIP kernels behind
the C ABI of include/bsw.h (libbsw.so).  `bsw` is the thin ctypes binding.
"""
from . import bsw  # noqa: F401

__all__ = ["bsw"]
