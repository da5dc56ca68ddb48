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

Parity status of every function is stated in its docstring; none is
"parity unpinned" (each is pinned by tests under `tests/test_oracle_*.py`).
"""
from . import cumulant, sigma  # noqa: F401
from .cumulant import spectral_cumulant
from .sigma import sigma_core

__all__ = ["sigma", "cumulant", "sigma_core", "spectral_cumulant"]
