"""Seeded synthetic input generator for plane-wave Kohn-Sham cells.

This module only *describes* the inputs of the Hamiltonian application and
the block-Davidson solver: the lattice, the plane-wave sphere (Miller list),
the real-space local potential on the FFT grid, the projector functions
beta(k+G), the D blocks and the random starting wavefunctions.  It contains
none of the method's arithmetic (no kinetic term, no FFT of wavefunctions,
no projector contraction, no eigensolver); both the FP64 CPU oracle and the
HIP library consume what it produces.

The paper (Quantum ESPRESSO toward the exascale, section "Quantum-engine
modules", items on lattices, plane-wave generation and pseudopotential terms)
names these ingredients without giving formulas; the forms used here are the
standard plane-wave pseudopotential ones with Gaussian model potentials.
"""

from .cells import (Cell, PROJ_SETS, make_cell, make_psi0, config_names,
                    random_served_cell, served_trace, sphere_miller,
                    fft_box_min, vloc_image_sum, vloc_fourier, radial_ft_closed,
                    real_harmonics_poly, beta_matrix, projgen_tables, gamma_half)

__all__ = ["Cell", "PROJ_SETS", "make_cell", "make_psi0", "config_names",
           "random_served_cell", "served_trace", "sphere_miller", "fft_box_min",
           "vloc_image_sum", "vloc_fourier", "radial_ft_closed",
           "real_harmonics_poly", "beta_matrix", "projgen_tables", "gamma_half"]
