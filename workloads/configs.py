"""Workload parameters for the Holstein square-lattice fermion solve.

Each configuration fixes the lattice (L x L periodic square lattice, N = L*L
sites), the imaginary-time discretisation (Ltau slices of width dtau, so
beta = Ltau*dtau), the model parameters of the Holstein Hamiltonian (hopping
t, chemical potential mu, phonon frequency omega, coupling alpha; Sec. II A,
Eqs. H_total..H_elph), the recipe of the synthetic phonon field, the number
of right-hand sides and the solver tolerance.  The paper's own benchmarks use
the square lattice with t = 1 and dtau = 0.1 (Sec. II B); its equilibrated
phonon fields are not available, so seeded synthetic fields of the same
shape stand in for them.
"""

from dataclasses import dataclass, field
from typing import Optional, Tuple


@dataclass(frozen=True)
class Params:
    name: str
    L: int                 # lattice side (even, >= 4); N = L*L
    Ltau: int              # number of imaginary-time slices (even)
    dtau: float
    t: float
    mu: float
    omega: float           # phonon frequency: only shapes the synthetic field
    alpha: float
    field: str             # recipe name, see workloads.inputs.phonon_field
    n_gauss: int = 1       # pseudofermion right-hand sides Phi = M(x)^T phi
    n_rademacher: int = 0  # measurement right-hand sides b = M(x)^T xi
    tol: float = 1e-10     # relative residual |b - M^T M u| / |b|
    cfg_id: int = 0        # seed component
    L_choices: Tuple[int, ...] = field(default_factory=tuple)  # batched only
    n_systems: int = 1
    # Chebyshev order constants (a1, a2) of the preconditioner,
    # N_P = floor(db (a1/phi + a2)) (App. C, Eq. NP_heuristic): the paper's
    # order-one values, or the pair measured fastest for the workload.
    cheb: Tuple[float, float] = (1.0, 1.0)

    @property
    def N(self) -> int:
        return self.L * self.L

    @property
    def dim(self) -> int:
        return self.N * self.Ltau

    @property
    def beta(self) -> float:
        return self.Ltau * self.dtau


# Five workloads.  Sizes: d = N*Ltau = 640, 40960, 409600, 6400..57600
# (batched), 1638400.
CONFIGS = {
    "c1": Params("holstein_L4_Ltau40", L=4, Ltau=40, dtau=0.1, t=1.0, mu=0.0,
                 omega=1.0, alpha=1.0, field="iid", tol=1e-10, cfg_id=1),
    "c2": Params("holstein_L16_Ltau160_cdw", L=16, Ltau=160, dtau=0.1, t=1.0,
                 mu=0.0, omega=0.5, alpha=1.5, field="cdw_ar1", tol=1e-10,
                 cfg_id=2),
    "c3": Params("holstein_L32_Ltau400", L=32, Ltau=400, dtau=0.05, t=1.0,
                 mu=-0.2, omega=1.0, alpha=1.2, field="ar1", tol=1e-8,
                 cfg_id=3, cheb=(0.15, 12.0)),
    "c4": Params("holstein_batched64_L8to24_Ltau100", L=0, Ltau=100, dtau=0.1,
                 t=1.0, mu=0.0, omega=1.0, alpha=1.0, field="iid",
                 n_gauss=8, n_rademacher=32, tol=1e-8, cfg_id=4,
                 L_choices=(8, 12, 16, 20, 24), n_systems=64),
    "c5": Params("holstein_L64_Ltau400", L=64, Ltau=400, dtau=0.05, t=1.0,
                 mu=0.0, omega=1.0, alpha=1.5, field="iid_shift", tol=1e-8,
                 cfg_id=5, cheb=(0.05, 12.0)),
}


def get_config(key: str) -> Params:
    return CONFIGS[key]


@dataclass(frozen=True)
class HmcParams:
    """Settings of one hybrid Monte Carlo update (Sec. III).

    The paper's benchmarks use dt = 1/(100 omega0), Nt = 100 steps, nt = 10
    bosonic sub-steps and m_reg = omega0 (Sec. III C), two pseudofermion
    fields, and solve to 1e-5 for forces and 1e-10 for the action difference
    (Sec. V B).  m_reg = None means no Fourier acceleration (M = dtau I).
    """
    omega0: float
    m_reg: Optional[float]
    dt: float
    Nt: int = 100
    nt: int = 10
    nfields: int = 2
    tol_force: float = 1e-5
    tol_action: float = 1e-10


def hmc_params(p: Params, **over) -> HmcParams:
    """The paper's HMC settings for configuration ``p`` (phonon frequency p.omega)."""
    base = dict(omega0=p.omega, m_reg=p.omega, dt=1.0 / (100.0 * p.omega))
    base.update(over)
    return HmcParams(**base)
