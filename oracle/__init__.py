"""Plain FP64 CPU oracle for the chi0 / epsilon^-1 path. TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package. The GPU library never calls it and never falls back to
it. It shares no code with the HIP path; both consume the same seeded inputs
from `synth`.

Every function is written from the paper's equations (Yambo 2019, arXiv
1902.03837) and cites the passage it follows:

* oscillator strengths, Eq. (rhotw) in the Linear Response section;
* the IP response sum over states, Eq. (X_IP), with the R/F split of
  Appendix A, at imaginary and at real frequencies (chi0_real_axis);
* the q -> 0 limit through velocity matrix elements, Eq. (dip) (G-space v);
* the bare Coulomb potential, Coulomb interaction subsection;
* the RPA Dyson equation as a matrix inversion, Eq. (X_rpa_inv), and the
  symmetrised screened interaction of Eq. (W_def);
* the Bruneval-Gonze X-terminator, Eq. (X_term_def) and Appendix B;
* the Godby-Needs plasmon-pole model and the GW self-energy matrix elements
  Sigma_x and Sigma_c, Eq. (sigma_c), Eq. (I_c), Eq. (W_def) (oracle/sigma.py);
* a small MLP (not in the paper) used by the learned band tail.

Parity status: rho, chi0 and epsilon^-1 are pinned by identities, closed forms
and brute force in tests/test_oracle_pins.py; the MLP by finite differences; the plasmon-pole
fit and the self-energies in tests/test_oracle_sigma.py; the real-axis response
in tests/test_oracle_real_axis.py.
Absolute values for the synthetic crystals beyond those pins are parity
unpinned: the oracle is the reference.
"""

from .rho import rho_direct, rho_fft, orbitals_real_space, rho_head_q0  # noqa: F401
from .chi0 import chi0_from_rho, pole_weights, chi0_real_axis, chi0_prefactor, crystal_prefactor  # noqa: F401
from .epsinv import epsinv_sym, epsinv_nonsym, eps_tilde, crystal_qpg  # noqa: F401
from .pipeline import rho_all_pairs, chi0_crystal, epsinv_crystal  # noqa: F401
from .metrics import rel_fro, err_table  # noqa: F401
