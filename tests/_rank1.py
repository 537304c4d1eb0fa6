"""Exact change of the fermion action under a one-component field change.

Changing one component x_k, k = (tau, i), changes only row k of M
(Eq. M_def: row k holds E_{tau,i} times row i of C acting on slice tau-1,
or on slice Ltau-1 with a minus sign when tau = 0).  So
M' = M + e_k r^T with r^T v = -dE s (C v_{tp})_i, dE = E'_{tau,i} - E_{tau,i},
(tp, s) = (tau-1, +1) for tau >= 1 and (Ltau-1, -1) for tau = 0.  With
u = (M^T M)^{-1} Phi and u' = (M'^T M')^{-1} Phi,

  S' - S = Phi.u' - Phi.u = -u^T (M'^T M' - M^T M) u'
         = -[(M u)_k (r.u') + (r.u)(M u')_k + (r.u)(r.u')],

exact for any size of the change, and free of the cancellation of
subtracting two actions of size ~d.  Used for finite-difference checks of
the force on lattices too large for a direct solve.
"""

import numpy as np


def action_change(lat, E, C_row, k, x_new, u, u_new):
    """S(x with x_k = x_new) - S(x) from the two solutions.

    E: [Ltau][N] at the unperturbed field; C_row: (indices, values) of row i
    of C; u, u_new: [Ltau][N] solutions (only slices tau and tp are read).
    """
    tau, i = k
    tp, s = (tau - 1, 1.0) if tau >= 1 else (lat.Ltau - 1, -1.0)
    idx, val = C_row
    e_old = E[tau, i]
    e_new = np.exp(-lat.dtau * (lat.alpha * x_new - lat.mu))
    dE = e_new - e_old

    def c_dot(v):
        return float(np.dot(val, v[tp][idx]))

    def M_k(v):          # (M v)_k with the unperturbed M
        return float(v[tau][i] - e_old * s * c_dot(v))

    def r_dot(v):        # r . v
        return float(-dE * s * c_dot(v))

    ru, run = r_dot(u), r_dot(u_new)
    return -(M_k(u) * run + ru * M_k(u_new) + ru * run)


def c_row(C, i):
    """(indices, values) of row i of a scipy sparse C."""
    row = C.getrow(i)
    return row.indices.copy(), row.data.copy()
