"""Phonon force dS_F/dx and brute-force derivatives of S_F.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

With one field, Lambda = I and S_F = Phi^T (M^T M)^{-1} Phi, the identity
d(C^{-1}) = -C^{-1} dC C^{-1} gives (Sec. III A, Eq. dSF_dx)

    dS_F/dx_{i,tau} = -u^T (dM^T M + M^T dM) u = -2 (M u) . (dM/dx_{i,tau} u),

with u = (M^T M)^{-1} Phi.  Only block row tau of M depends on x_{i,tau}
(Eq. dB/dx: the derivative acts on the diagonal factor exp(-dtau V_tau)),
and only its row i: d E_{tau,i} / d x_{i,tau} = -dtau*alpha*E_{tau,i}.
"""

import numpy as np

from . import lattice as lat_mod
from . import solve as solve_mod


def force_from_solution(lat, x, u, C=None):
    """dS_F/dx[tau, i] from the solution u (Eq. dSF_dx with Lambda = I).

    u may be [Ltau, N] or [R, Ltau, N]; the result has the same shape
    (one force per right-hand side).  C may be dense or scipy sparse.
    """
    C = lat_mod.checkerboard_C(lat) if C is None else C
    E = lat_mod.E_field(lat, x)
    u = np.asarray(u)
    Mu = lat_mod.apply_M(lat, x, u, C)
    # (dM/dx_{i,tau} u) at row (i, tau):  -(dE_{tau,i}) (C u~_{tau-1})_i
    #   = dtau*alpha*E_{tau,i} (C u~_{tau-1})_i, with u~_{-1} = -u_{Ltau-1}.
    dMu = np.empty_like(Mu)
    for tau in range(lat.Ltau):
        prev = u[..., tau - 1, :] if tau >= 1 else -u[..., lat.Ltau - 1, :]
        dMu[..., tau, :] = lat.dtau * lat.alpha * E[tau] * (prev @ C.T)
    return -2.0 * Mu * dMu


def action_at(lat, x, Phi, C=None):
    """S_F(x) = Phi . (M^T M)^{-1} Phi with a dense LU (complex x allowed)."""
    u = solve_mod.solve_dense(lat, x, Phi, C)
    return np.sum(Phi * u, axis=(-2, -1))


def force_complex_step(lat, x, Phi, h=1e-20, C=None):
    """dS_F/dx by complex-step differentiation (Squire & Trapp, 1998).

    dS/dx_k = Im S_F(x + i h e_k) / h.  M(x) is analytic in x and only plain
    transposes appear, so the derivative is exact to rounding with no
    subtractive cancellation.  One dense complex solve per component: use
    on small lattices only.
    """
    C = lat_mod.checkerboard_C(lat) if C is None else C
    x = np.asarray(x, dtype=np.float64)
    g = np.empty(x.shape)
    for tau in range(lat.Ltau):
        for i in range(lat.N):
            xc = x.astype(np.complex128)
            xc[tau, i] += 1j * h
            g[tau, i] = np.imag(action_at(lat, xc, Phi, C)) / h
    return g


def force_central_fd(lat, x, Phi, comps, h=1e-4, C=None):
    """Central differences of S_F with one Richardson step, for listed (tau, i).

    D(h) = (S(x+h e_k) - S(x-h e_k)) / 2h;  result = (4 D(h/2) - D(h)) / 3.
    Loses digits to cancellation when S_F is large: use on small lattices.
    """
    C = lat_mod.checkerboard_C(lat) if C is None else C
    x = np.asarray(x, dtype=np.float64)

    def D(hh, tau, i):
        xp = x.copy()
        xm = x.copy()
        xp[tau, i] += hh
        xm[tau, i] -= hh
        return (action_at(lat, xp, Phi, C) - action_at(lat, xm, Phi, C)) / (2 * hh)

    return np.array([(4 * D(h / 2, tau, i) - D(h, tau, i)) / 3 for tau, i in comps])
