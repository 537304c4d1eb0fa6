"""Hybrid Monte Carlo update of the phonon field (Sec. III, Algorithm 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

The sampled action is the one with A = M (Lambda = I), Eq. (S_prime):

    S'(x) = S_B(x) - dtau*alpha*sum_{i,tau} x_{i,tau}
            + 1/2 sum_sigma Phi_sigma^T (M^T M)^{-1} Phi_sigma,

where the linear term is the exponent of Eq. (Z_path_orig) (beta*alpha*xbar
summed over sites), and each Phi_sigma = M(x_i)^T R_sigma is drawn at the
start of the update (Eq. PhiSample-1).  The x-only part
S_B - dtau*alpha*sum x is what the bosonic sub-steps of the time-step
splitting integrate (Sec. III B 2).

Readings of the paper used here (stated once, used by every function):

* Periodic imaginary time for the phonon field: x_{i,Ltau} = x_{i,0} in
  Eq. (S_B) and x_{i,-1} = x_{i,Ltau-1} in Eq. (dSB_dx).
* Eq. (Qww_def) and the mass matrix print sin^2(2 pi w / Ltau).  The
  stencil of Eq. (dSB_dx) and the paper's own statement that the extreme
  values sit at w = Ltau/2 (omega_0^2 + 4/dtau^2) and w = 0 (omega_0^2) fix
  the argument to pi w / Ltau, which is used in both.
* m_reg = infinity (``m_reg=None``) is the limit M = dtau * I.
* The fermion force of each step is evaluated once per phonon configuration
  (the paper notes that the two half kicks at the same x share it); the two
  half kicks are still applied one after the other.

Functions are pinned in ``tests/test_oracle_hmc.py``: closed forms of S_B
for constant and single-Fourier-mode fields, finite differences of every
action against its force, the Fourier form of Q against the stencil, the
limits of the mass matrix, exact harmonic motion under M = Q/omega_0^2,
reversibility, O(dt^2) energy error, and a unit Jacobian of the trajectory
map (volume conservation).
"""

import numpy as np

from . import lattice as lat_mod
from . import solve as solve_mod
from . import force as force_mod


# ---------------------------------------------------------------- bosonic part

def bosonic_action(lat, x, omega0):
    """S_B of Eq. (S_B), periodic in tau.  x: [Ltau, N]."""
    x = np.asarray(x, dtype=np.float64)
    xn = np.roll(x, -1, axis=0)                     # x_{i,tau+1}, x_{i,Ltau} = x_{i,0}
    return 0.5 * lat.dtau * np.sum(omega0 ** 2 * x * x + ((xn - x) / lat.dtau) ** 2)


def linear_action(lat, x):
    """-dtau*alpha*sum_{i,tau} x_{i,tau}: the linear term of Eqs. (Z_path_orig, S_prime)."""
    return -lat.dtau * lat.alpha * np.sum(np.asarray(x, dtype=np.float64))


def bosonic_force(lat, x, omega0):
    """dS_B/dx of Eq. (dSB_dx), periodic in tau."""
    x = np.asarray(x, dtype=np.float64)
    lap = np.roll(x, -1, axis=0) - 2.0 * x + np.roll(x, 1, axis=0)
    return lat.dtau * (omega0 ** 2 * x - lap / lat.dtau ** 2)


def x_action(lat, x, omega0):
    """The x-only part of S': S_B - dtau*alpha*sum x."""
    return bosonic_action(lat, x, omega0) + linear_action(lat, x)


def x_force(lat, x, omega0):
    """Gradient of ``x_action``: dS_B/dx - dtau*alpha."""
    return bosonic_force(lat, x, omega0) - lat.dtau * lat.alpha


# ------------------------------------------------ Fourier basis in imaginary time

def q_tilde(Ltau, dtau, omega0):
    """Diagonal of Q in the Fourier basis, Eq. (Qww_def), w = 0..Ltau-1."""
    w = np.arange(Ltau)
    return dtau * (omega0 ** 2 + 4.0 / dtau ** 2 * np.sin(np.pi * w / Ltau) ** 2)


def mass_tilde(Ltau, dtau, omega0, m_reg):
    """Diagonal of the dynamical mass in the Fourier basis (Sec. III B 1).

    m_reg=None is the m_reg -> infinity limit, M = dtau * I.
    """
    if m_reg is None:
        return np.full(Ltau, float(dtau))
    w = np.arange(Ltau)
    s = 4.0 / dtau ** 2 * np.sin(np.pi * w / Ltau) ** 2
    r = m_reg ** 2 + omega0 ** 2
    return dtau * (r + s) / r


def tau_fourier_apply(v, diag):
    """F^{-1} diag(diag) F v along imaginary time (Eqs. F_forward, F_def).

    v: [..., Ltau, N].  F is the unitary DFT of Eq. (F_def).  For a diag that
    is even in w (diag[w] = diag[Ltau-w]) the result is real; it is returned
    as such.
    """
    vh = np.fft.fft(np.asarray(v, dtype=np.float64), axis=-2, norm="ortho")
    out = np.fft.ifft(np.asarray(diag)[:, None] * vh, axis=-2, norm="ortho")
    return out.real


def sample_momentum(R, mt):
    """p = sqrt(M) R (Eq. sample_p), with sqrt taken mode by mode."""
    return tau_fourier_apply(R, np.sqrt(mt))


def kinetic_energy(p, mt):
    """p^T M^{-1} p / 2."""
    return 0.5 * float(np.sum(p * tau_fourier_apply(p, 1.0 / mt)))


# ---------------------------------------------------------------- fermion part

def pseudofermions(lat, x, R_fields, C=None):
    """Phi_sigma = M(x)^T R_sigma (Eq. PhiSample-1 with A = M)."""
    C = lat_mod.checkerboard_C(lat) if C is None else C
    return np.stack([lat_mod.apply_MT(lat, x, R, C) for R in R_fields])


def solve_lu(lat, x, Phis, C=None):
    """u_sigma = (M^T M)^{-1} Phi_sigma by a sparse LU of M."""
    return solve_mod.solve_sparse(lat, x, Phis, C)


def fermion_action(lat, x, Phis, C=None, solve=solve_lu):
    """1/2 sum_sigma Phi_sigma . (M^T M)^{-1} Phi_sigma (Eq. S_F with A = M)."""
    u = solve(lat, x, Phis, C)
    return 0.5 * float(np.sum(Phis * u))


def fermion_force(lat, x, Phis, C=None, solve=solve_lu):
    """d/dx of ``fermion_action``: 1/2 sum_sigma of the one-field force (Eq. dSF_dx)."""
    u = solve(lat, x, Phis, C)
    return 0.5 * np.sum(force_mod.force_from_solution(lat, x, u, C), axis=0)


# ----------------------------------------------------------- Hamiltonian dynamics

def hamiltonian(lat, omega0, mt, x, p, Phis, C=None, solve=solve_lu, lam=False):
    """H(x, p) = S(x) + p^T M^{-1} p / 2 and its parts; S is S' (A = M) or,
    with ``lam``, the action with A = M Lambda (Eq. S_again)."""
    if lam:
        from . import lam as lam_mod
        sb = bosonic_action(lat, x, omega0)
        sf = lam_mod.fermion_action(lat, x, Phis, C, solve)
    else:
        sb = x_action(lat, x, omega0)
        sf = fermion_action(lat, x, Phis, C, solve)
    k = kinetic_energy(p, mt)
    return {"H": sb + sf + k, "S_B": sb, "S_F": sf, "K": k}


def leapfrog_split(lat, omega0, mt, x, p, dt, Nt, nt, f_force, b_force=None):
    """Time-step splitting leapfrog of Algorithm 1 (Eqs. leapfrog1-3).

    f_force(x) returns the fermion force dS_F/dx at x; the bosonic sub-steps
    use b_force (default ``x_force``: S_B and the linear term of S').
    Returns (x, p) after Nt steps of length dt, each holding nt bosonic
    sub-steps of length dt/nt.  Inputs are not modified.
    """
    if b_force is None:
        b_force = lambda v: x_force(lat, v, omega0)
    x = np.array(x, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    h = dt / nt
    minv = 1.0 / mt
    fF = f_force(x)
    for _ in range(Nt):
        p = p - 0.5 * dt * fF
        for _ in range(nt):
            p = p - 0.5 * h * b_force(x)
            x = x + h * tau_fourier_apply(p, minv)
            p = p - 0.5 * h * b_force(x)
        fF = f_force(x)
        p = p - 0.5 * dt * fF
    return x, p


def hmc_update(lat, omega0, m_reg, dt, Nt, nt, x_i, R_fields, R_mom, r_uniform,
               C=None, solve=solve_lu, lam=False):
    """One HMC trial update (Algorithm 1) with the action S' (A = M) or, with
    ``lam``, the action S of Eq. (S_again) (A = M Lambda, bosonic part S_B).

    x_i: [Ltau, N]; R_fields: [nfields, Ltau, N] Gaussian draws for the
    pseudofermions; R_mom: [Ltau, N] Gaussian draws for the momentum;
    r_uniform in (0, 1).  Returns a dict with the final (x_f, p_f), the
    energies before and after, the acceptance probability, the decision and
    the field kept (x_f if accepted, else x_i).
    """
    C = lat_mod.checkerboard_C(lat) if C is None else C
    x_i = np.asarray(x_i, dtype=np.float64)
    mt = mass_tilde(lat.Ltau, lat.dtau, omega0, m_reg)
    p_i = sample_momentum(R_mom, mt)
    if lam:
        from . import lam as lam_mod
        Phis = lam_mod.pseudofermions(lat, x_i, R_fields, C)
        f_force = lambda x: lam_mod.fermion_force(lat, x, Phis, C, solve)
        b_force = lambda x: bosonic_force(lat, x, omega0)
    else:
        Phis = pseudofermions(lat, x_i, R_fields, C)
        f_force = lambda x: fermion_force(lat, x, Phis, C, solve)
        b_force = None
    Hi = hamiltonian(lat, omega0, mt, x_i, p_i, Phis, C, solve, lam)
    x_f, p_f = leapfrog_split(lat, omega0, mt, x_i, p_i, dt, Nt, nt, f_force, b_force)
    Hf = hamiltonian(lat, omega0, mt, x_f, p_f, Phis, C, solve, lam)
    dH = Hf["H"] - Hi["H"]
    prob = min(1.0, float(np.exp(-dH)))
    accepted = bool(r_uniform < prob)
    return {"x_f": x_f, "p_f": p_f, "p_i": p_i, "Phi": Phis, "H_i": Hi, "H_f": Hf, "dH": dH,
            "accept_prob": prob, "accepted": accepted, "x_out": x_f if accepted else x_i}
