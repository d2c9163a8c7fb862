"""Plain FP64 CPU oracle for the plane-wave Kohn-Sham H|psi> and block Davidson.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or calls this package; only the tests, the
graft smoke check and the CPU-baseline leg of the benchmark do.  It shares no
code with the HIP path: its only common input is the seeded cell generator
(``cellgen``), which holds none of the method's arithmetic.

What it computes, and where the paper names it (Quantum ESPRESSO toward the
exascale):

* ``apply_h``: the one-particle Hamiltonian applied to Bloch states (the
  "Hamiltonian builds" of the quantum-engine layer in section "Challenges and
  opportunities of new heterogeneous architectures"), as the sum of the
  kinetic, local-potential and pseudopotential contributions listed among the
  GPU-ported kernels (section "Evolution of the GPU-enabled version").  The
  local part goes through the oracle's own dense per-axis DFT (``dft``), the
  exact definition of the operator that the pruned FFT path computes.
* ``dense_h``: the same operator written out as a matrix for tiny cells;
  ``dense_eigs`` its lowest eigenvalues by LAPACK.
* ``davidson``: the Davidson iterative diagonalisation (same section) with the
  Rayleigh-Ritz step solved as a Hermitian generalized eigenproblem, as the
  paper's dense-solver library does.
* ``density``: the charge density generation of the same list of ported
  kernels, rho(r) = (1/Omega) sum_i f_i |psi_i(r)|^2 on the FFT grid;
  ``density_direct`` sums the plane waves point by point (tiny cells).
* ``gamma.expand`` / ``gamma.restrict``: real wavefunctions at k = 0 stored
  over half the sphere, rebuilt as full-sphere vectors for the operators above.
* ``cg``: the band-by-band preconditioned conjugate-gradient eigensolver,
  the paper's other iterative solver (same section).
* ``overlap``: the overlap operator S = 1 + sum |beta> q <beta| of ultrasoft /
  PAW pseudopotentials (also among the ported kernels) and the generalized
  Davidson for H psi = eps S psi.
* ``beta_projectors``: the projectors beta_i(k+G) built from their radial
  functions (the "calculation of pseudopotential terms" of the quantum-engine
  modules), with the radial Bessel transform taken by quadrature.

The paper prints no formula for any of these; the forms are the standard
plane-wave pseudopotential ones.  Every reading taken where the paper is
silent is listed in the design notes of the repository.

Pins: every function here is checked in ``tests/test_oracle_pins.py``,
``tests/test_oracle_density.py`` and ``tests/test_oracle_beta.py`` against
closed forms, invariants, brute force and library routines (see those files).
"""

from .dft import dft_matrix, dft_axis, inv3, fwd3
from .hamiltonian import (kinetic, vloc_psi, vnl_psi, apply_h, dense_h, dense_eigs,
                          vloc_coeffs, hdiag)
from .davidson import davidson, rayleigh_ritz
from .cg import cg
from .density import cell_volume, density, density_direct, psi_real_space
from .beta import beta_projectors, radial_transform, real_harmonics, spherical_bessel
from . import gamma
from . import overlap

__all__ = ["dft_matrix", "dft_axis", "inv3", "fwd3", "kinetic", "vloc_psi", "vnl_psi",
           "apply_h", "dense_h", "dense_eigs", "vloc_coeffs", "hdiag", "davidson", "rayleigh_ritz", "cg",
           "cell_volume", "density", "density_direct", "psi_real_space", "beta_projectors",
           "radial_transform", "real_harmonics", "spherical_bessel", "gamma", "overlap"]
