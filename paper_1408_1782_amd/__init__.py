"""MI355X (gfx950) solver for the spatially inhomogeneous matrix-valued
quantum Boltzmann equation of Lu & Mendl (arXiv:1408.1782).

The numerical work runs in ``libqb.so`` (hand-written HIP, C ABI in
``include/qb.h``); this package only marshals arguments.  torch supplies
device memory and streams.  Importing the package does not need a GPU;
calling into the library does, and fails loudly when ``libqb.so`` is missing.
"""
from ._lib import (  # noqa: F401
    BC,
    Batch,
    Plan,
    Problem,
    QBError,
    load,
    lib_path,
)


def evolve(plan, W0, B, dt, nsteps, checkpoint_every=20):
    """Differentiable splitting-step integration (see ``autograd.evolve``)."""
    from .autograd import evolve as _evolve

    return _evolve(plan, W0, B, dt, nsteps, checkpoint_every)


__all__ = ["BC", "Batch", "Plan", "Problem", "QBError", "evolve", "load", "lib_path"]
