"""The Lambda reformulation of the fermion action and the global updates (Secs. II C, IV; App. B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

Z = int Dx e^{-S_B} [det(M Lambda)]^2 (Eq. Z_path) with any Lambda whose
det Lambda^2 = exp(dtau alpha sum x) (Eq. Lambda_constraint); the paper's
choice (Eq. Lambda_def) couples slice tau to slice tau + 1 of the same site:

    Lambda[(i,tau), (i,tau+1)] = s(tau+1) exp(+dtau alpha x_{i,tau+1} / 2),
    s(t) = +1 if t = 0 else -1,         (tau + 1 taken mod Ltau)

and its inverse (Eq. Lambda_inv)

    Lambda^{-1}[(i,tau), (i,tau-1)] = s(tau) exp(-dtau alpha x_{i,tau} / 2).

With A = M Lambda the action is S = S_B + 1/2 sum_sigma |A^{-T} Phi_sigma|^2
(Eqs. S_again, S_F) and Phi_sigma = A(x)^T R_sigma (Eq. PhiSample-1).
Writing b = Lambda^{-T} Phi gives |A^{-T} Phi|^2 = b^T (M^T M)^{-1} b, so the
solve is the same normal-equation solve as with A = M, on the right-hand
side b, which now depends on x.

Force (Eq. dSF_dx with A = M Lambda): for one field f = b^T u, u = (M^T M)^{-1} b,
    df/dx_{i,tau} = -2 (M u) . (dM/dx_{i,tau} u) + 2 u . (db/dx_{i,tau}),
and b_{i,t} = s(t+1) exp(-dtau alpha x_{i,t+1}/2) Phi_{i,t+1} depends only on
x_{i,t+1}, with derivative -(dtau alpha / 2) b_{i,t}; so the second term is
-dtau alpha (b * u)_{i,tau-1} (slice tau - 1 taken mod Ltau).

Pinned in ``tests/test_oracle_lam.py``: Lambda Lambda^{-1} = I from the two
printed formulas, det Lambda^2 against Eq. (Lambda_constraint), the matrix
A^T printed in App. B (Eq. A_x) and the exact symmetry D_x = D_{-x} there,
the b-form of the action against the definition |A^{-T} Phi|^2, the force
against complex-step derivatives of the definition, and the reflection
symmetry of Delta S (Eq. Delta_S_sym) in the single-site adiabatic limit.
"""

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import lattice as lat_mod
from . import force as force_mod
from . import solve as solve_mod


def _sign(t):
    return 1.0 if t == 0 else -1.0


def lambda_sparse(lat, x):
    """Lambda of Eq. (Lambda_def) as a CSR matrix over (tau, i) rows (index tau*N + i)."""
    x = np.asarray(x)
    N, T = lat.N, lat.Ltau
    rows, cols, vals = [], [], []
    for tau in range(T):
        tp = (tau + 1) % T
        for i in range(N):
            rows.append(tau * N + i)
            cols.append(tp * N + i)
            vals.append(_sign(tp) * np.exp(0.5 * lat.dtau * lat.alpha * x[tp, i]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(lat.dim, lat.dim),
                         dtype=np.result_type(x, np.float64))


def lambda_inv_sparse(lat, x):
    """Lambda^{-1} of Eq. (Lambda_inv) as a CSR matrix."""
    x = np.asarray(x)
    N, T = lat.N, lat.Ltau
    rows, cols, vals = [], [], []
    for tau in range(T):
        tm = (tau - 1) % T
        for i in range(N):
            rows.append(tau * N + i)
            cols.append(tm * N + i)
            vals.append(_sign(tau) * np.exp(-0.5 * lat.dtau * lat.alpha * x[tau, i]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(lat.dim, lat.dim),
                         dtype=np.result_type(x, np.float64))


def _flat(v, lat):
    v = np.asarray(v)
    return v.reshape(-1, lat.dim)


def apply_lambda_T(lat, x, w):
    """Lambda(x)^T w for w [..., Ltau, N]."""
    Lm = lambda_sparse(lat, x).T.tocsr()
    f = _flat(w, lat)
    return np.stack([Lm @ r for r in f]).reshape(np.shape(w))


def apply_lambda_invT(lat, x, w):
    """Lambda(x)^{-T} w for w [..., Ltau, N]."""
    Li = lambda_inv_sparse(lat, x).T.tocsr()
    f = _flat(w, lat)
    return np.stack([Li @ r for r in f]).reshape(np.shape(w))


def dense_A(lat, x, C=None):
    """A = M Lambda as a dense matrix."""
    return lat_mod.dense_M(lat, x, C) @ lambda_sparse(lat, x).toarray()


def pseudofermions(lat, x, R_fields, C=None):
    """Phi_sigma = A(x)^T R_sigma = Lambda^T M^T R_sigma (Eq. PhiSample-1)."""
    C = lat_mod.checkerboard_C(lat) if C is None else C
    return np.stack([apply_lambda_T(lat, x, lat_mod.apply_MT(lat, x, R, C)) for R in R_fields])


def action_definition(lat, x, Phis, C=None):
    """1/2 sum_sigma |A^{-T} Phi_sigma|^2 by an LU of the dense A (Eq. S_F); complex x allowed."""
    A = dense_A(lat, x, C)
    lu = scipy.linalg.lu_factor(A)
    z = scipy.linalg.lu_solve(lu, np.asarray(Phis).reshape(-1, lat.dim).T, trans=1)
    return 0.5 * np.sum(z * z)


def rhs_b(lat, x, Phis):
    """b_sigma = Lambda(x)^{-T} Phi_sigma."""
    return apply_lambda_invT(lat, x, Phis)


def fermion_action(lat, x, Phis, C=None, solve=solve_mod.solve_sparse):
    """1/2 sum_sigma b_sigma . (M^T M)^{-1} b_sigma, b = Lambda^{-T} Phi."""
    b = rhs_b(lat, x, Phis)
    u = solve(lat, x, b, C)
    return 0.5 * float(np.sum(b * u))


def fermion_force(lat, x, Phis, C=None, solve=solve_mod.solve_sparse):
    """d/dx of ``fermion_action`` (module docstring): 1/2 sum_sigma of
    -2 (M u) . (dM u) - dtau alpha shift_tau(b * u)."""
    b = rhs_b(lat, x, Phis)
    u = solve(lat, x, b, C)
    g = np.sum(force_mod.force_from_solution(lat, x, u, C), axis=0)
    bu = np.sum(b * u, axis=0)
    g = g - lat.dtau * lat.alpha * np.roll(bu, 1, axis=0)
    return 0.5 * g


def force_complex_step(lat, x, Phis, comps, h=1e-20, C=None):
    """d/dx of ``action_definition`` at listed (tau, i) by complex-step differentiation."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    for tau, i in comps:
        xc = x.astype(np.complex128)
        xc[tau, i] += 1j * h
        out.append(np.imag(action_definition(lat, xc, Phis, C)) / h)
    return np.array(out)


# ------------------------------------------------------------- global updates

def reflect(x, i):
    """x_i -> -x_i at every tau (Sec. IV)."""
    y = np.array(x, dtype=np.float64)
    y[:, i] = -y[:, i]
    return y


def swap(x, i, j):
    """(x_i, x_j) -> (x_j, x_i) at every tau (Sec. IV)."""
    y = np.array(x, dtype=np.float64)
    y[:, [i, j]] = y[:, [j, i]]
    return y


def global_update(lat, omega0, x, kind, sites, R_fields, r_uniform, lam=True, C=None,
                  solve=solve_mod.solve_sparse):
    """One reflection or swap Metropolis update (Eqs. metropolis, Delta_S_F).

    Phi_sigma is drawn at x (Eq. PhiSample-1 with A = M Lambda if ``lam``,
    else A = M and the action S' of Eq. S_prime); the proposal x' is the
    reflection of site sites[0] or the swap of sites (i, j); accept with
    probability min(1, exp(-Delta S)).
    """
    from . import hmc as hmc_mod
    C = lat_mod.checkerboard_C(lat) if C is None else C
    x = np.asarray(x, dtype=np.float64)
    xp = reflect(x, sites[0]) if kind == "reflect" else swap(x, sites[0], sites[1])
    if lam:
        Phis = pseudofermions(lat, x, R_fields, C)
        Sx = lambda v: hmc_mod.bosonic_action(lat, v, omega0)
        SF = lambda v: fermion_action(lat, v, Phis, C, solve)
    else:
        Phis = hmc_mod.pseudofermions(lat, x, R_fields, C)
        Sx = lambda v: hmc_mod.x_action(lat, v, omega0)
        SF = lambda v: hmc_mod.fermion_action(lat, v, Phis, C, solve)
    dSB = Sx(xp) - Sx(x)
    SF0 = SF(x)
    SF1 = SF(xp)
    dS = dSB + SF1 - SF0
    prob = min(1.0, float(np.exp(-dS)))
    acc = bool(r_uniform < prob)
    return {"x_prop": xp, "dS_B": dSB, "S_F_old": SF0, "S_F_new": SF1, "dS": dS,
            "accept_prob": prob, "accepted": acc, "x_out": xp if acc else x}
