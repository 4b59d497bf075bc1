"""FP64 CPU oracle for the semiclassical-approximation (SCA) potential.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or call anything in this package; the product
(the HIP library and its Python binding) never does, and this package never
imports the product.

What it computes, all in float64 (Sec. II of the paper, Eqs. (1), (7), (8)):

  H_s(phi) = -t K + (Delta/2) S - s diag(phi)           s = +1 (up), -1 (down)
  A_ns     = i w_n I - H_s(phi),   w_n = (2n+1) pi T,   n = 0 .. M-1
  Omega    = sum_i phi_i^2 / U - 2 T sum_s sum_n ln|det A_ns|
  dOmega/dphi_i = 2 phi_i / U - 2 T sum_s s sum_n Re (A_ns^-1)_ii
  Omega~   = Omega + 2 N T sum_n ln w_n^2     (phi-independent shift removed)
  rho_s(w) = -(1/(pi N)) Im tr ((w + i eta) I - H_s)^-1

K is the periodic nearest-neighbour adjacency of the L x L square lattice
(site i = x + L*y; a bond counted once per direction, so K_ij = 2 on L = 2),
S = diag((-1)^(x+y)).  The paper's sum over n = -M .. M-1 pairs +w_n with
-w_n; the pair contributes 2 ln|det A_ns| because H_s is real symmetric.

Two routes that share no code:
  route D (`lu`)       -- the definition: one complex LU with partial pivoting
                          per (n, s), written out here; Leibniz brute force
                          for 4x4 matrices.
  route S (`spectral`) -- eigendecomposition of H_s and the Matsubara sums.
`closed` holds the Bloch closed forms for a staggered field, the infinite-M
limits and the Hartree-Fock equation; `adam` the Kingma-Ba recurrence;
`hmc` Hybrid Monte Carlo of the static-field weight exp(-Omega/T).

Parity status per function is listed in each module's docstring; every
function here is pinned by a test under tests/ that does not re-type its
formula (brute force, closed forms, limits, library routines, invariants).
"""
from .model import (neighbours, kinetic_matrix, stagger_signs, hamiltonian,
                    matsubara, n_sites)
from .lu import (lu_pivoted, logabsdet_lu, inverse_lu, diag_inverse_lu,
                 leibniz_det, adjugate_diag)
from .spectral import (omega_spectral, grad_spectral, dos_spectral,
                       terms_spectral)
from .api import (omega_tilde, omega_full, grad, af_order, dos, adam_solve,
                  shifted_terms, shifted_terms_s, omega_tilde_d, grad_d)
from .adam import AdamState, adam_step
from .hmc import hmc_hamiltonian, leapfrog, hmc_chain

__all__ = [
    "neighbours", "kinetic_matrix", "stagger_signs", "hamiltonian",
    "matsubara", "n_sites", "lu_pivoted", "logabsdet_lu", "inverse_lu",
    "diag_inverse_lu", "leibniz_det", "adjugate_diag", "omega_spectral",
    "grad_spectral", "dos_spectral", "terms_spectral", "omega_tilde",
    "omega_full", "grad", "af_order", "dos", "adam_solve", "shifted_terms",
    "shifted_terms_s",
    "omega_tilde_d", "grad_d", "AdamState", "adam_step", "hmc_hamiltonian",
    "leapfrog", "hmc_chain",
]
