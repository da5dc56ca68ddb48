"""Deterministic generator of synthetic systems (NumPy PCG64).

Recipe (all draws from one `Generator(PCG64(seed))`, in this order):

1. core energies: exactly the configured value when the window has zero
   width, else U[core window] eV;
2. valence energies U[valence window] eV; 3. virtual energies U[virtual
   window] eV; each block sorted ascending, occupied block first (cores are
   the lowest occupied levels, so they take indices 0..n_core-1);
4. M_ov[P][i][a] ~ N(0,1) * m_scale / sqrt(N_aux);
5. M_oo[P][i][j] ~ N(0,1) * m_scale / sqrt(N_aux), upper triangle (i <= j)
   mirrored so that M_oo is symmetric in (i, j).

All energies are converted to Hartree (1 Ha = 27.211386245988 eV); M is in
Ha^(1/2).  Optionally (`structured=True`) the core/other-orbital coefficients
M_{c,m != c} are scaled by 1e-3 to mimic core localisation.

The virtual-virtual block M_vv (needed only when the energies of virtual
states are themselves updated, as in evGW0) comes from its own stream,
`Generator(PCG64(SeedSequence([seed, 2])))`, with the same scale and the
upper triangle (a <= b) mirrored, so that adding it changes no other array.

Grids: the imaginary axis uses the modified Gauss-Legendre mapping of
`mgl_grid`; the real axis is an inclusive linspace either on an absolute eV
window shared by all cores, or on [eps_n + lo, eps_n + hi] per core n (so the
last point equals eps_n exactly when hi == 0).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .configs import EV_PER_HA, WorkloadConfig


@dataclass
class System:
    """Arrays in the layout the C ABI takes (all float64, row-major)."""
    eps: np.ndarray         # [n_basis] Hartree, occupied first
    occ: np.ndarray         # [n_basis] 2.0 or 0.0
    M_oo: np.ndarray        # [n_aux][n_occ][n_occ]
    M_ov: np.ndarray        # [n_aux][n_occ][n_virt]
    core_idx: np.ndarray    # [n_core] int32
    omega_imag: np.ndarray  # [n_imag]
    w_imag: np.ndarray      # [n_imag]
    omega_real: np.ndarray  # [n_core][n_real]
    eta: float
    vxc: Optional[np.ndarray] = None
    name: str = ""
    seed: Optional[int] = None
    m_scale: float = 0.3

    @property
    def n_aux(self) -> int:
        return self.M_ov.shape[0]

    @property
    def n_occ(self) -> int:
        return self.M_ov.shape[1]

    @property
    def n_virt(self) -> int:
        return self.M_ov.shape[2]

    @property
    def n_basis(self) -> int:
        return self.n_occ + self.n_virt

    @property
    def n_core(self) -> int:
        return int(self.core_idx.shape[0])


def mgl_grid(n: int, omega0: float = 0.5):
    """Modified Gauss-Legendre grid on (0, inf).

    Gauss-Legendre nodes x_k and weights u_k on (-1, 1) are mapped by
    omega = omega0 (1 + x) / (1 - x); the Jacobian gives
    w_k = 2 omega0 u_k / (1 - x_k)^2.  Nodes are returned ascending.
    """
    x, u = np.polynomial.legendre.leggauss(int(n))
    omega = omega0 * (1.0 + x) / (1.0 - x)
    w = 2.0 * omega0 * u / (1.0 - x) ** 2
    order = np.argsort(omega)
    return np.ascontiguousarray(omega[order]), np.ascontiguousarray(w[order])


def make_system(n_basis: int, n_occ: int, n_core: int, n_aux: int, n_imag: int, n_real: int,
                eta_ev: float, seed: int, core_ev=(-290.5, -289.5), valence_ev=(-30.0, -8.0),
                virtual_ev=(-2.0, 60.0), real_abs_ev=None, real_rel_ev=(-25.0, 0.0),
                m_scale: float = 0.3, omega0_ha: float = 0.5, structured: bool = False,
                name: str = "") -> System:
    if not (1 <= n_core < n_occ < n_basis):
        raise ValueError("need 1 <= n_core < n_occ < n_basis")
    rng = np.random.Generator(np.random.PCG64(seed))
    n_virt = n_basis - n_occ
    n_val = n_occ - n_core
    if core_ev[0] == core_ev[1]:
        e_core = np.full(n_core, float(core_ev[0]))
    else:
        e_core = np.sort(rng.uniform(core_ev[0], core_ev[1], n_core))
    e_val = np.sort(rng.uniform(valence_ev[0], valence_ev[1], n_val))
    e_virt = np.sort(rng.uniform(virtual_ev[0], virtual_ev[1], n_virt))
    eps = np.concatenate([e_core, e_val, e_virt]) / EV_PER_HA
    occ = np.concatenate([np.full(n_occ, 2.0), np.zeros(n_virt)])

    scale = m_scale / np.sqrt(n_aux)
    M_ov = rng.standard_normal((n_aux, n_occ, n_virt)) * scale
    raw = rng.standard_normal((n_aux, n_occ, n_occ)) * scale
    iu = np.triu_indices(n_occ)
    M_oo = np.zeros_like(raw)
    M_oo[:, iu[0], iu[1]] = raw[:, iu[0], iu[1]]
    M_oo[:, iu[1], iu[0]] = raw[:, iu[0], iu[1]]
    if structured:
        for c in range(n_core):
            keep = M_oo[:, c, c].copy()
            M_oo[:, c, :] *= 1e-3
            M_oo[:, :, c] *= 1e-3
            M_oo[:, c, c] = keep
            M_ov[:, c, :] *= 1e-3

    omega_imag, w_imag = mgl_grid(n_imag, omega0_ha)
    core_idx = np.arange(n_core, dtype=np.int32)
    omega_real = np.empty((n_core, n_real))
    for c in range(n_core):
        if real_abs_ev is not None:
            omega_real[c] = np.linspace(real_abs_ev[0], real_abs_ev[1], n_real) / EV_PER_HA
        else:
            lo = eps[c] + real_rel_ev[0] / EV_PER_HA
            hi = eps[c] + real_rel_ev[1] / EV_PER_HA
            omega_real[c] = np.linspace(lo, hi, n_real)
    return System(eps=eps, occ=occ, M_oo=np.ascontiguousarray(M_oo),
                  M_ov=np.ascontiguousarray(M_ov), core_idx=core_idx,
                  omega_imag=omega_imag, w_imag=w_imag, omega_real=omega_real,
                  eta=eta_ev / EV_PER_HA, vxc=None, name=name, seed=seed, m_scale=m_scale)


def make_vv(n_aux: int, n_virt: int, seed: int, m_scale: float = 0.3) -> np.ndarray:
    """M_vv[P][a][b] ~ N(0,1) * m_scale / sqrt(N_aux), symmetric in (a, b)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 2])))
    raw = rng.standard_normal((n_aux, n_virt, n_virt)) * (m_scale / np.sqrt(n_aux))
    iu = np.triu_indices(n_virt)
    M_vv = np.zeros_like(raw)
    M_vv[:, iu[0], iu[1]] = raw[:, iu[0], iu[1]]
    M_vv[:, iu[1], iu[0]] = raw[:, iu[0], iu[1]]
    return np.ascontiguousarray(M_vv)


def vv_block(system: System) -> np.ndarray:
    """The M_vv block belonging to a generated system (its seed and scale)."""
    if system.seed is None:
        raise ValueError("system has no seed")
    return make_vv(system.n_aux, system.n_virt, system.seed, system.m_scale)


def system_from_config(cfg: WorkloadConfig, structured: bool = False, **over) -> System:
    kw = dict(
        n_basis=cfg.n_basis, n_occ=cfg.n_occ, n_core=cfg.n_core, n_aux=cfg.n_aux,
        n_imag=cfg.n_imag, n_real=cfg.n_real, eta_ev=cfg.eta_ev, seed=cfg.seed,
        core_ev=cfg.core_ev, valence_ev=cfg.valence_ev, virtual_ev=cfg.virtual_ev,
        real_abs_ev=cfg.real_abs_ev, real_rel_ev=cfg.real_rel_ev, m_scale=cfg.m_scale,
        omega0_ha=cfg.omega0_ha, structured=structured, name=cfg.name,
    )
    kw.update(over)
    return make_system(**kw)
