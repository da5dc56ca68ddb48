"""FP64 CPU oracle for the GW+C core-level path (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow reference that the HIP path is checked
against.  Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import it; the product path never calls it and has no CPU
fallback.  It shares no code with the HIP path: the only common dependency is
the seeded input generator in `workloads/`, which holds none of the method's
arithmetic.

Contents
* `sigma`    - correlation self-energy of a core state by contour deformation
               with the resolution of the identity (paper: section
               "Self-energy evaluation", Eqs. cd_terms, cd_imaginary,
               cd_residue, cd_prefactors, cd_sigma_imaginary,
               cd_sigma_imaginary_decoupled), exchange (Eq. sigma_x) and the
               GW+C quasiparticle energy (Eq. QPGWC).
* `cumulant` - the numerical Landau cumulant and the GW+C spectral function
               (section "Numerical GW+C scheme", Eqs. landau_cumulant_truncated,
               cumulant_propagator_numerical_time, cumulant_propagator_fourier,
               cumulant_propagator_convolution, eq:AGWC).
* `wac`      - CD-WAC: W^c_nm continued from reference points by a Thiele
               continued fraction (Eq. pade_approximation).
* `analytic` - the fully analytic G0W0 route: RPA excitations from the
               Casida problem (Eqs. rpa_casida, rpa_matrices), transition
               moments (Eq. density_shifts), the pole sum of Eq. sigma_spectral
               and the G0W0 / G_DH W0 spectral functions (Eqs.
               A_explicit_real_imaginary, hedin_sigma_spectral).
* `evgw`     - evGW0 (Eq. ev_sigma_spectral): every state's quasiparticle
               equation iterated with the current energies in G and W at the
               RPA level, by a bracketed Newton solve per state.

Parity status of every function is stated in its docstring; none is
"parity unpinned" (each is pinned by tests under `tests/test_oracle_*.py`).
"""
from . import analytic, cumulant, evgw, sigma, wac  # noqa: F401
from .cumulant import spectral_cumulant
from .sigma import sigma_core

__all__ = ["sigma", "cumulant", "wac", "analytic", "evgw", "sigma_core", "spectral_cumulant"]
