"""MI355X (gfx950) solver for the spatially inhomogeneous matrix-valued
quantum Boltzmann equation of Lu & Mendl (arXiv:1408.1782).

The numerical work runs in ``libqb.so`` (hand-written HIP, C ABI in
``include/qb.h``); this package only marshals arguments.  torch supplies
device memory and streams.  Importing the package does not need a GPU;
calling into the library does, and fails loudly when ``libqb.so`` is missing.
"""
from ._lib import (  # noqa: F401
    BC,
    Plan,
    Problem,
    QBError,
    load,
    lib_path,
)

__all__ = ["BC", "Plan", "Problem", "QBError", "load", "lib_path"]
