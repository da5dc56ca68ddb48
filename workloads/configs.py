"""Molecule-shaped synthetic workloads.

The paper's systems (the CORE65 set, benzene to pentacene) are replaced by
synthetic inputs with the same shapes: numbers of occupied and virtual
orbitals, auxiliary basis size, core levels near -290 eV (carbon 1s), valence
levels in [-30, -8] eV and virtual levels in [-2, 60] eV.  Energies are stated
in eV here and converted to Hartree by the generator.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional, Tuple

EV_PER_HA = 27.211386245988


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n_basis: int
    n_occ: int
    n_core: int
    n_aux: int
    n_imag: int
    n_real: int
    eta_ev: float
    seed: int
    # core levels: exact value (single core) or a uniform window around -290 eV
    core_ev: Tuple[float, float] = (-290.5, -289.5)
    valence_ev: Tuple[float, float] = (-30.0, -8.0)
    virtual_ev: Tuple[float, float] = (-2.0, 60.0)
    # real grid: absolute window (eV) shared by every core, or a window relative
    # to each core level (eV below, eV above)
    real_abs_ev: Optional[Tuple[float, float]] = None
    real_rel_ev: Tuple[float, float] = (-25.0, 0.0)
    m_scale: float = 0.3
    omega0_ha: float = 0.5  # scale of the imaginary-axis grid mapping
    description: str = ""

    @property
    def n_virt(self) -> int:
        return self.n_basis - self.n_occ

    @property
    def n_ov(self) -> int:
        return self.n_occ * self.n_virt


CONFIGS = {
    "c1": WorkloadConfig(
        name="c1", n_basis=40, n_occ=5, n_core=1, n_aux=160, n_imag=24, n_real=120,
        eta_ev=0.1, seed=1, core_ev=(-290.0, -290.0), real_abs_ev=(-320.0, -280.0),
        description="1 core state, N_basis=40, N_aux=160, 24 imaginary / 120 real frequencies",
    ),
    "c2": WorkloadConfig(
        name="c2", n_basis=300, n_occ=21, n_core=6, n_aux=1200, n_imag=32, n_real=400,
        eta_ev=0.1, seed=2,
        description="benzene-sized: 6 C1s levels, N_basis=300, N_aux=1200, 32 imag / 400 real",
    ),
    "c3": WorkloadConfig(
        name="c3", n_basis=520, n_occ=34, n_core=10, n_aux=2100, n_imag=32, n_real=400,
        eta_ev=0.1, seed=3,
        description="naphthalene-sized: 10 C1s levels, N_basis=520, N_aux=2100",
    ),
    "c4": WorkloadConfig(
        name="c4", n_basis=1100, n_occ=73, n_core=22, n_aux=4400, n_imag=40, n_real=600,
        eta_ev=0.05, seed=4,
        description="pentacene-sized: 22 C1s levels, N_basis=1100, N_aux=4400",
    ),
}


def serving_request_config(n_basis: int, seed: int) -> WorkloadConfig:
    """Shape of one molecule in the serving stream: N_aux = 4 N_basis,
    N_occ = max(2, round(N_basis/15)), N_core = max(1, round(0.3 N_occ)),
    24 imaginary and 120 real frequencies on [eps_n - 30, eps_n + 10] eV."""
    n_occ = max(2, int(round(n_basis / 15)))
    n_core = max(1, int(round(0.3 * n_occ)))
    n_core = min(n_core, n_occ - 1)
    return WorkloadConfig(
        name=f"serve_nb{n_basis}_s{seed}", n_basis=n_basis, n_occ=n_occ, n_core=n_core,
        n_aux=4 * n_basis, n_imag=24, n_real=120, eta_ev=0.1, seed=seed,
        real_rel_ev=(-30.0, 10.0),
        description="serving request",
    )


def small_config(name: str = "tiny", n_occ: int = 3, n_virt: int = 5, n_core: int = 1,
                 n_aux: int = 12, n_imag: int = 16, n_real: int = 9, seed: int = 11,
                 eta_ev: float = 0.1, **kw) -> WorkloadConfig:
    """A tiny system for brute-force checks and ragged-tile tests."""
    return WorkloadConfig(
        name=name, n_basis=n_occ + n_virt, n_occ=n_occ, n_core=n_core, n_aux=n_aux,
        n_imag=n_imag, n_real=n_real, eta_ev=eta_ev, seed=seed, **kw,
    )


def with_overrides(cfg: WorkloadConfig, **kw) -> WorkloadConfig:
    return replace(cfg, **kw)
