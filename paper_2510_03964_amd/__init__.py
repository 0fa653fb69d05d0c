"""Foveated weighted reservoir sampling on AMD Instinct MI355X (gfx950).

The per-pixel weighted-reservoir-sampling pass of "Enhancing Foveated
Rendering with Weighted Reservoir Sampling" (MIG '25, arXiv 2510.03964) as a
C-ABI HIP library (include/fwrs.h, ``libfwrs.so``) with a thin ctypes binding:

* ``fwrs``      -- the binding: ``Reservoir`` (one stream), ``Engine`` (batched ticks)
* ``synth``     -- seeded synthetic workloads shaped like the paper's
* ``build``     -- compiles ``libfwrs.so`` for gfx950
"""
from . import synth  # noqa: F401

__all__ = ["synth", "fwrs", "build"]
