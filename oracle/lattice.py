"""Lattice, hopping, checkerboard factors and the space-time matrix M.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

Conventions
-----------
* Square L x L lattice, periodic, L even and >= 4.  Site index i = x + L*y.
* Hopping matrix K_ij = -t for nearest neighbours (Sec. II C, Eq. V_K_def).
* The phonon field is stored as x[tau, i], tau = 0..Ltau-1 (Sec. II C).
* V_tau = diag(alpha*x_tau - mu), so exp(-dtau V_tau) = diag(E_tau) with
  E_tau = exp(-dtau*(alpha*x_tau - mu))  (Eqs. B_def, V_K_def).
* B_tau = exp(-dtau V_tau) C, where C approximates exp(-dtau K) by the
  checkerboard factorisation (Sec. II D).  The paper cites the "minimal
  split" checkerboard without spelling it out.  Reading used here: the four
  bond families of the square lattice (x-bonds starting at even x, at odd
  x, y-bonds starting at even y, at odd y) fall into two groups,
      A = {x-even, y-even}  (disjoint 4-site plaquettes with even corner),
      B = {x-odd,  y-odd}   (disjoint 4-site plaquettes with odd corner,
                             wrapping around the periodic boundary),
  the hopping inside each group commutes, each group is exponentiated
  exactly, and C = exp(-dtau K_A) exp(-dtau K_B): group B acts first on a
  vector.  C is not symmetric for L >= 6 and differs from exp(-dtau K)
  at O(dtau^2) (Sec. II D; App. C notes the slight non-Hermiticity).
* M (Eq. M_def): identity diagonal blocks, -B_tau at block (tau, tau-1) for
  tau >= 1 and +B_0 at block (0, Ltau-1).
"""

from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse as sp


@dataclass(frozen=True)
class Lattice:
    L: int
    Ltau: int
    dtau: float
    t: float
    mu: float
    alpha: float

    @property
    def N(self):
        return self.L * self.L

    @property
    def dim(self):
        return self.N * self.Ltau

    @classmethod
    def from_params(cls, p, L=None):
        return cls(L=p.L if L is None else L, Ltau=p.Ltau, dtau=p.dtau,
                   t=p.t, mu=p.mu, alpha=p.alpha)


def site(x, y, L):
    return (x % L) + L * (y % L)


def bond_families(L):
    """The four nearest-neighbour bond families as lists of (i, j) pairs."""
    fam = {"x_even": [], "x_odd": [], "y_even": [], "y_odd": []}
    for y in range(L):
        for x in range(L):
            fam["x_even" if x % 2 == 0 else "x_odd"].append((site(x, y, L), site(x + 1, y, L)))
            fam["y_even" if y % 2 == 0 else "y_odd"].append((site(x, y, L), site(x, y + 1, L)))
    return fam


def _hopping_from_bonds(N, bonds, t):
    K = np.zeros((N, N))
    for i, j in bonds:
        K[i, j] -= t
        K[j, i] -= t
    return K


def hopping_matrix(L, t):
    """Dense K with K_ij = -t on nearest-neighbour bonds (Eq. V_K_def)."""
    fam = bond_families(L)
    bonds = fam["x_even"] + fam["x_odd"] + fam["y_even"] + fam["y_odd"]
    return _hopping_from_bonds(L * L, bonds, t)


def group_hopping(L, t, group):
    """Hopping restricted to checkerboard group 'A' or 'B' (see module doc)."""
    fam = bond_families(L)
    if group == "A":
        bonds = fam["x_even"] + fam["y_even"]
    elif group == "B":
        bonds = fam["x_odd"] + fam["y_odd"]
    else:
        raise ValueError(group)
    return _hopping_from_bonds(L * L, bonds, t)


def checkerboard_factors(lat):
    """Dense exp(-dtau K_A) and exp(-dtau K_B) by matrix exponential."""
    if lat.L % 2 or lat.L < 4:
        raise ValueError("checkerboard needs even L >= 4")
    PA = scipy.linalg.expm(-lat.dtau * group_hopping(lat.L, lat.t, "A"))
    PB = scipy.linalg.expm(-lat.dtau * group_hopping(lat.L, lat.t, "B"))
    return PA, PB


def checkerboard_C(lat):
    """Dense checkerboard approximation C = exp(-dtau K_A) exp(-dtau K_B)."""
    PA, PB = checkerboard_factors(lat)
    return PA @ PB


def exact_expK(lat):
    """Dense exp(-dtau K) without the checkerboard split."""
    return scipy.linalg.expm(-lat.dtau * hopping_matrix(lat.L, lat.t))


def plaquettes(L, group):
    """Site lists (corner, +x, +y, +x+y) of the disjoint plaquettes of a group."""
    off = 0 if group == "A" else 1
    out = []
    for y0 in range(off, L + off, 2):
        for x0 in range(off, L + off, 2):
            out.append((site(x0, y0, L), site(x0 + 1, y0, L),
                        site(x0, y0 + 1, L), site(x0 + 1, y0 + 1, L)))
    return out


def sparse_factor(lat, group):
    """Sparse exp(-dtau K_group): one 4x4 matrix exponential per plaquette.

    Each plaquette's hopping matrix (4 bonds of the group) is exponentiated
    with scipy.linalg.expm; the factor is the direct sum of these blocks.
    """
    rows, cols, vals = [], [], []
    for sites in plaquettes(lat.L, group):
        h = np.zeros((4, 4))
        for a, b in ((0, 1), (2, 3), (0, 2), (1, 3)):
            h[a, b] = h[b, a] = -lat.t
        blk = scipy.linalg.expm(-lat.dtau * h)
        for a in range(4):
            for b in range(4):
                rows.append(sites[a])
                cols.append(sites[b])
                vals.append(blk[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(lat.N, lat.N))


def sparse_C(lat):
    """Sparse C = exp(-dtau K_A) exp(-dtau K_B) from per-plaquette exponentials."""
    return (sparse_factor(lat, "A") @ sparse_factor(lat, "B")).tocsr()


def E_field(lat, x):
    """E[tau, i] = exp(-dtau*(alpha*x[tau, i] - mu)): diagonal of exp(-dtau V_tau)."""
    return np.exp(-lat.dtau * (lat.alpha * np.asarray(x) - lat.mu))


def B_blocks(lat, x, C=None):
    """Dense B_tau = diag(E_tau) C for every tau (Eq. B_def)."""
    C = checkerboard_C(lat) if C is None else C
    E = E_field(lat, x)
    return [E[tau][:, None] * C for tau in range(lat.Ltau)]


def dense_M(lat, x, C=None):
    """Dense NLtau x NLtau matrix M of Eq. M_def (complex x gives complex M)."""
    C = checkerboard_C(lat) if C is None else C
    E = E_field(lat, x)
    N, T = lat.N, lat.Ltau
    M = np.eye(N * T, dtype=np.result_type(E, C))
    for tau in range(T):
        B = E[tau][:, None] * C
        if tau >= 1:
            M[tau * N:(tau + 1) * N, (tau - 1) * N:tau * N] = -B
        else:
            M[0:N, (T - 1) * N:T * N] = B
    return M


def sparse_M(lat, x, C=None):
    """CSR form of the same M, assembled block by block from a sparse C."""
    C = sparse_C(lat) if C is None else sp.csr_matrix(C)
    E = E_field(lat, x)
    T = lat.Ltau
    blocks = [[None] * T for _ in range(T)]
    for tau in range(T):
        blocks[tau][tau] = sp.identity(lat.N, format="csr")
        B = sp.diags(E[tau]) @ C
        if tau >= 1:
            blocks[tau][tau - 1] = -B
        else:
            blocks[0][T - 1] = B
    return sp.bmat(blocks, format="csr")


def apply_M(lat, x, v, C=None):
    """M v for v[..., tau, i] by block rows of Eq. M_def (dense C per slice)."""
    C = checkerboard_C(lat) if C is None else C
    E = E_field(lat, x)
    v = np.asarray(v)
    out = np.empty(np.broadcast_shapes(v.shape, E.shape), dtype=np.result_type(v, E, C))
    for tau in range(lat.Ltau):
        prev = v[..., tau - 1, :] if tau >= 1 else -v[..., lat.Ltau - 1, :]
        out[..., tau, :] = v[..., tau, :] - E[tau] * (prev @ C.T)
    return out


def apply_MT(lat, x, w, C=None):
    """M^T w by block columns of Eq. M_def: block (tau-1, tau) of M^T is -B_tau^T."""
    C = checkerboard_C(lat) if C is None else C
    E = E_field(lat, x)
    w = np.asarray(w)
    out = np.empty(np.broadcast_shapes(w.shape, E.shape), dtype=np.result_type(w, E, C))
    T = lat.Ltau
    for tau in range(T):
        if tau + 1 < T:
            nxt = E[tau + 1] * w[..., tau + 1, :]
        else:
            nxt = -E[0] * w[..., 0, :]
        out[..., tau, :] = w[..., tau, :] - nxt @ C
    return out


def det_M_via_product(lat, x, C=None):
    """log|det(I + B_{Ltau-1} ... B_0)| and its sign (Eq. detM_alt)."""
    Bs = B_blocks(lat, x, C)
    prod = np.eye(lat.N)
    for B in Bs:
        prod = B @ prod
    return np.linalg.slogdet(np.eye(lat.N) + prod)
