"""FP64 CPU oracle for the spin-open factorized three-point function.

TEST INFRASTRUCTURE.  This package is the checker, not the product: only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import or run it.  It shares no code with the GPU library and does not import
it.  See ``oracle.c3pt_oracle`` for the factorized form and ``oracle.brute``
for the direct evaluation of the three-point trace on tiny lattices.
"""
from .c3pt_oracle import (  # noqa: F401
    GAMMA, GAMMA5_DIAG, gamma_basis16, momenta, site_coords, phase_matrix,
    spectator_meson, spectator_baryon, insertion, covariant_derivative, covariant_derivative_vector, combine,
    all_pairs, EPS, two_sink_meson, creation_matrix, charge_conjugation, parity_projectors,
    gamma_project_meson, gamma_project_nucleon, PROTON_TERMS, smear,
)
