"""MI355X-native matrix-free Newton-Krylov state solver for density-based
topology optimisation of natural-convection heat sinks (arXiv:1508.04596).

* ``inputs``  -- seeded synthetic workloads (grids, designs, masks, traces).
* ``fe``      -- ctypes binding of the C-ABI in ``include/fe.h`` (HIP library).
* ``autograd``-- ``torch.autograd.Function`` wrappers (state solve, compliance).
* ``build``   -- in-tree build of ``libfe_hip.so`` for gfx950.

The binding is imported lazily so that the input generators can be used
without loading the HIP library.
"""
__all__ = ["inputs", "fe", "autograd", "build"]
