"""Seeded synthetic inputs for the symmetry-adapted GW hot path.

Crystals and operation tables (``crystals``), the real-harmonic convention and
the orbital representation used for group averaging (``rep``), and the seeded
Fock matrices and three-index tensors (``fields``).  Shared by the tests, the
benchmark and the oracle's callers; holds no step of the GW method itself.
"""
from .crystals import (Crystal, Workload, crystal, workload, mesh_points, mesh_index,
                       kmap, minus_k, add_k, nbf, cubic_point_group, in_td)
from .rep import BasisRep, real_harmonics, wigner_real
from .fields import Inputs
