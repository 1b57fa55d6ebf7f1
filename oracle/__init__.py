"""FP64 CPU oracle of the LBM + IBM + FE bead-spring swimmer method
(Geyer et al., arXiv 2202.12147).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library never loads it.
"""
from .orc import Oracle, phi, lattice, icosphere, membrane_eval, spread, interp  # noqa: F401
