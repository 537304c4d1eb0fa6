"""Seeded random draws for the synthetic workloads.

Every draw comes from ``numpy.random.default_rng(SeedSequence([220301291,
cfg_id, stream, *extra]))`` and is returned in FP64 on the host.  Streams:

    0  phonon field x                       shape [Ltau, N]
    1  Gaussian draws phi (pseudofermion)   shape [R, Ltau, N]
    2  Rademacher draws xi (measurement)    shape [R, Ltau, N]
    3  lattice sides of batched systems
    4  finite-difference component picks
    5  perturbation of x away from the field that defined Phi
    6  HMC pseudofermion draws R_sigma         shape [nfields, Ltau, N]
    7  HMC momentum draws R                    shape [Ltau, N]
    8  HMC Metropolis uniform r                scalar in [0, 1)

Layout convention: site index i = x + L*y is fastest, then the time slice
tau = 0..Ltau-1, then the right-hand-side index.  The pseudofermion field
itself is Phi = M(x)^T phi (Eq. PhiSample-1 with Lambda = I); forming it
needs the operator M, so each consumer (oracle or GPU path) computes it from
``phi`` with its own code.
"""

import numpy as np

_ROOT_SEED = 220301291


def rng_for(cfg_id: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng(
        np.random.SeedSequence([_ROOT_SEED, int(cfg_id), int(stream), *map(int, extra)]))


def _ar1(rng, Ltau, N, rho, sigma):
    """Stationary AR(1) process along tau, independently per site."""
    eta = np.empty((Ltau, N))
    eta[0] = sigma * rng.standard_normal(N)
    s = sigma * np.sqrt(1.0 - rho * rho)
    for tau in range(1, Ltau):
        eta[tau] = rho * eta[tau - 1] + s * rng.standard_normal(N)
    return eta


def phonon_field(p, L=None, system=None):
    """Synthetic phonon field x[tau, i] for configuration ``p``.

    Recipes:
      iid        x ~ N(0, 1) independently.
      iid_shift  x ~ N(0, 1) + 0.5.
      ar1        stationary AR(1) in tau, coefficient 0.95, variance 1/omega.
      cdw_ar1    0.8*(-1)^(x+y) checkerboard plus AR(1) noise in tau
                 (coefficient 0.95, standard deviation 0.3).
    """
    L = p.L if L is None else L
    N = L * L
    extra = () if system is None else (system,)
    rng = rng_for(p.cfg_id, 0, *extra)
    if p.field == "iid":
        return rng.standard_normal((p.Ltau, N))
    if p.field == "iid_shift":
        return rng.standard_normal((p.Ltau, N)) + 0.5
    if p.field == "ar1":
        return _ar1(rng, p.Ltau, N, 0.95, np.sqrt(1.0 / p.omega))
    if p.field == "cdw_ar1":
        xs, ys = np.meshgrid(np.arange(L), np.arange(L), indexing="xy")
        sign = np.where((xs + ys) % 2 == 0, 1.0, -1.0).reshape(N)
        return 0.8 * sign[None, :] + _ar1(rng, p.Ltau, N, 0.95, 0.3)
    raise ValueError(f"unknown field recipe {p.field!r}")


def gaussian_rhs(p, nrhs, L=None, system=None):
    """Gaussian draws phi[r, tau, i] ~ N(0, 1) (the paper's R_sigma)."""
    L = p.L if L is None else L
    extra = () if system is None else (system,)
    return rng_for(p.cfg_id, 1, *extra).standard_normal((nrhs, p.Ltau, L * L))


def rademacher_rhs(p, nrhs, L=None, system=None):
    """Rademacher draws xi[r, tau, i] in {-1, +1}."""
    L = p.L if L is None else L
    extra = () if system is None else (system,)
    bits = rng_for(p.cfg_id, 2, *extra).integers(0, 2, size=(nrhs, p.Ltau, L * L))
    return (2 * bits - 1).astype(np.float64)


def perturbed_field(p, x, scale=0.1):
    """x + scale * N(0,1): a field away from the one that defined Phi."""
    return x + scale * rng_for(p.cfg_id, 5).standard_normal(x.shape)


def batched_systems(p):
    """Lattice sides of the batched workload, drawn uniformly from L_choices."""
    rng = rng_for(p.cfg_id, 3)
    return [int(v) for v in rng.choice(np.array(p.L_choices), size=p.n_systems)]


def fd_sample_indices(p, count, L=None):
    """Distinct (tau, i) components for finite-difference checks."""
    L = p.L if L is None else L
    d = p.Ltau * L * L
    flat = rng_for(p.cfg_id, 4).choice(d, size=min(count, d), replace=False)
    return [(int(k) // (L * L), int(k) % (L * L)) for k in flat]


def hmc_draws(p, nfields=2, traj=0, L=None):
    """Random inputs of one HMC update: (R_fields, R_mom, r_uniform).

    R_fields[sigma] ~ N(0, 1) defines Phi_sigma = M(x)^T R_sigma
    (Eq. PhiSample-1), R_mom ~ N(0, 1) defines p = sqrt(M) R (Eq. sample_p)
    and r ~ U[0, 1) is the Metropolis draw (Algorithm 1).  ``traj`` numbers
    successive updates.
    """
    L = p.L if L is None else L
    N = L * L
    R_fields = rng_for(p.cfg_id, 6, traj).standard_normal((nfields, p.Ltau, N))
    R_mom = rng_for(p.cfg_id, 7, traj).standard_normal((p.Ltau, N))
    r = float(rng_for(p.cfg_id, 8, traj).random())
    return R_fields, R_mom, r
