"""FP64 CPU oracle for the symmetry-adapted GW hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its Python binding.
"""
from .gw import (tau_grid, matsubara, transform_matrices, to_freq, to_tau, fermi_factor_parts,
                 polarization_unit, self_energy_unit,
                 g0_closed_form, free_count, polarization, self_energy, screened, dyson,
                 particle_number, find_mu, gw_iteration, exchange, hartree,
                 exchange_unit, hartree_unit, ir_basis, ir_eval, ir_fourier, ir_grid, ir_transform_matrices,
                 logistic_kernel)
