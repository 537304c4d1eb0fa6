"""Space-time matrix, fermion action and force of an SSH-type coupling.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

The paper (Sec. II C, closing remark; Sec. III A, force of the SSH model)
says only that in the SSH model the phonon coordinates of the sites enter
the hopping matrix K_tau, and that the force then follows by the product
rule through the sparse checkerboard factors of exp(-dtau K_tau).  It does
not write the coupling down.  Reading used here (stated once, used by both
sides):

* the phonon field x[tau, i] lives on sites, as in the Holstein model;
* a nearest-neighbour bond b = (i, j), j = i + x^ or i + y^, hops with
  t_b(x_tau) = t - g * (x_{j,tau} - x_{i,tau})  (site-displacement SSH form);
* the checkerboard keeps the four bond families of the Holstein matrix
  (x-bonds from even x, y-bonds from even y, x-bonds from odd x, y-bonds
  from odd y); within a family the bonds are disjoint, so each family is
  exponentiated exactly, and
      C(x_tau) = F_xe F_ye F_xo F_yo,   F_f = exp(-dtau K_f(x_tau)),
  (F_yo acts first on a vector).  With g = 0 the x- and y-families inside a
  plaquette commute and C equals the Holstein C = exp(-dtau K_A) exp(-dtau K_B);
* the on-site factor stays diag(E_tau) = exp(-dtau (alpha x_tau - mu)), so
  alpha = 0 gives the pure SSH coupling and g = 0 the Holstein matrix;
* B_tau = diag(E_tau) C(x_tau), and M has the block structure of Eq. M_def
  (identity diagonal, -B_tau below it, +B_0 in the corner).

S_F = Phi . (M^T M)^{-1} Phi per field (Eq. Sf_Psi with Lambda = I), and
dS_F/dx = -2 (M u) . (dM/dx u) with u = (M^T M)^{-1} Phi (Eq. dSF_dx).  The
derivative of each factor is taken with the Frechet derivative of the
matrix exponential (scipy.linalg.expm_frechet): no closed form of the bond
factors is used here.  Dense matrices for small lattices; ``sparse_M`` builds
the same matrix from the exponentials of the two-site hopping blocks
(scipy.linalg.expm per bond) for lattices up to L = 64.
"""

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lattice as lat_mod

FAMILIES = ("x_even", "y_even", "x_odd", "y_odd")  # left to right in C


def hoppings(lat, g, x_tau):
    """{family: [(i, j, t_b)]} for one time slice (the coupling read above)."""
    fam = lat_mod.bond_families(lat.L)
    x_tau = np.asarray(x_tau)
    return {f: [(i, j, lat.t - g * (x_tau[j] - x_tau[i])) for i, j in fam[f]] for f in FAMILIES}


def family_hopping(lat, bonds):
    """Dense K_f with K_ij = K_ji = -t_b on the family's bonds (complex t_b allowed)."""
    dt = np.result_type(*[b[2] for b in bonds], np.float64)
    K = np.zeros((lat.N, lat.N), dtype=dt)
    for i, j, tb in bonds:
        K[i, j] -= tb
        K[j, i] -= tb
    return K


def factors(lat, g, x_tau):
    """[F_xe, F_ye, F_xo, F_yo], each exp(-dtau K_f(x_tau)) by scipy expm."""
    hp = hoppings(lat, g, x_tau)
    return [scipy.linalg.expm(-lat.dtau * family_hopping(lat, hp[f])) for f in FAMILIES]


def C_slice(lat, g, x_tau):
    """C(x_tau) = F_xe F_ye F_xo F_yo."""
    F = factors(lat, g, x_tau)
    return F[0] @ F[1] @ F[2] @ F[3]


def full_hopping(lat, g, x_tau):
    """Dense K(x_tau) of all bonds (no checkerboard split)."""
    hp = hoppings(lat, g, x_tau)
    return sum(family_hopping(lat, hp[f]) for f in FAMILIES)


def B_slice(lat, g, x, tau):
    """B_tau = diag(E_tau) C(x_tau)."""
    E = lat_mod.E_field(lat, x)
    return E[tau][:, None] * C_slice(lat, g, x[tau])


def dense_M(lat, g, x):
    """Dense N Ltau x N Ltau matrix M (block structure of Eq. M_def)."""
    x = np.asarray(x)
    N, T = lat.N, lat.Ltau
    Bs = [B_slice(lat, g, x, tau) for tau in range(T)]
    M = np.eye(N * T, dtype=np.result_type(*Bs))
    for tau in range(T):
        if tau >= 1:
            M[tau * N:(tau + 1) * N, (tau - 1) * N:tau * N] = -Bs[tau]
        else:
            M[0:N, (T - 1) * N:T * N] = Bs[0]
    return M


def apply(lat, g, x, v, op="M"):
    """M v, M^T v or M^T M v for v[..., Ltau, N] through the dense matrix."""
    M = dense_M(lat, g, x)
    v = np.asarray(v)
    sh = v.shape
    w = v.reshape(-1, lat.dim).T
    if op == "M":
        out = M @ w
    elif op == "MT":
        out = M.T @ w
    elif op == "MTM":
        out = M.T @ (M @ w)
    else:
        raise ValueError(op)
    return out.T.reshape(sh)


def solve(lat, g, x, Phi):
    """u = (M^T M)^{-1} Phi by LU of the dense M: w = M^{-T} Phi, then
    u = M^{-1} w (Phi [..., Ltau, N]; complex x allowed).  M^T M is never
    formed: that would square the condition number."""
    M = dense_M(lat, g, x)
    lu = scipy.linalg.lu_factor(M)
    Phi = np.asarray(Phi)
    sh = Phi.shape
    w = scipy.linalg.lu_solve(lu, Phi.reshape(-1, lat.dim).T.astype(M.dtype), trans=1)
    u = scipy.linalg.lu_solve(lu, w, trans=0)
    return u.T.reshape(sh)


def action(lat, g, x, Phi):
    """S_F = sum over fields of Phi . (M^T M)^{-1} Phi (complex x allowed)."""
    u = solve(lat, g, x, Phi)
    return np.sum(np.asarray(Phi) * u)


def dM_dx(lat, g, x, tau, i):
    """Dense dM/dx_{i,tau}: only block (tau, tau-1) (or the corner for tau = 0).

    d B_tau = d diag(E_tau) C + diag(E_tau) sum_f F_1 .. dF_f .. F_4, with
    dF_f the Frechet derivative of expm at -dtau K_f in the direction
    -dtau dK_f/dx_i (product rule through the factors).
    """
    x = np.asarray(x, dtype=np.float64)
    N, T = lat.N, lat.Ltau
    E = lat_mod.E_field(lat, x)[tau]
    hp = hoppings(lat, g, x[tau])
    Ks = [family_hopping(lat, hp[f]) for f in FAMILIES]
    Fs = [scipy.linalg.expm(-lat.dtau * K) for K in Ks]
    C = Fs[0] @ Fs[1] @ Fs[2] @ Fs[3]
    dC = np.zeros((N, N))
    fam = lat_mod.bond_families(lat.L)
    for k, f in enumerate(FAMILIES):
        dK = np.zeros((N, N))
        for a, b in fam[f]:
            # t_b = t - g (x_b - x_a): dt_b/dx_i = g [i == a] - g [i == b]; K_ab = -t_b
            dt = g * ((i == a) - (i == b))
            dK[a, b] -= dt
            dK[b, a] -= dt
        if not dK.any():
            continue
        dF = scipy.linalg.expm_frechet(-lat.dtau * Ks[k], -lat.dtau * dK, compute_expm=False)
        left = np.eye(N)
        for m in range(k):
            left = left @ Fs[m]
        right = np.eye(N)
        for m in range(k + 1, 4):
            right = right @ Fs[m]
        dC += left @ dF @ right
    dE = np.zeros(N)
    dE[i] = -lat.dtau * lat.alpha * E[i]
    dB = dE[:, None] * C + E[:, None] * dC
    dM = np.zeros((N * T, N * T))
    r0 = tau * N
    if tau >= 1:
        dM[r0:r0 + N, (tau - 1) * N:tau * N] = -dB
    else:
        dM[0:N, (T - 1) * N:T * N] = dB
    return dM


def force(lat, g, x, Phi):
    """dS_F/dx[tau, i] = -2 sum_fields (M u) . (dM/dx_{i,tau} u) (Eq. dSF_dx)."""
    x = np.asarray(x, dtype=np.float64)
    u = solve(lat, g, x, Phi).reshape(-1, lat.dim)
    M = dense_M(lat, g, x)
    y = u @ M.T
    out = np.zeros((lat.Ltau, lat.N))
    for tau in range(lat.Ltau):
        for i in range(lat.N):
            dM = dM_dx(lat, g, x, tau, i)
            out[tau, i] = -2.0 * np.sum(y * (u @ dM.T))
    return out


def force_complex_step(lat, g, x, Phi, h=1e-20):
    """dS_F/dx by complex-step differentiation of action() (Squire & Trapp, 1998)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape)
    for tau in range(lat.Ltau):
        for i in range(lat.N):
            xc = x.astype(np.complex128)
            xc[tau, i] += 1j * h
            out[tau, i] = np.imag(action(lat, g, xc, Phi)) / h
    return out


def sparse_M(lat, g, x):
    """CSR form of the same M.  The bonds of a family are disjoint, so each
    family factor is the direct sum of the exponentials of its two-site
    hopping blocks, each taken with scipy.linalg.expm; complex x allowed."""
    x = np.asarray(x)
    N, T = lat.N, lat.Ltau
    E = lat_mod.E_field(lat, x)
    blocks = [[None] * T for _ in range(T)]
    fam = lat_mod.bond_families(lat.L)
    for tau in range(T):
        C = None
        for f in FAMILIES:
            rows, cols, vals = [], [], []
            for i, j in fam[f]:
                tb = lat.t - g * (x[tau][j] - x[tau][i])
                blk = scipy.linalg.expm(-lat.dtau * np.array([[0.0, -tb], [-tb, 0.0]]))
                for a, ia in enumerate((i, j)):
                    for b, jb in enumerate((i, j)):
                        rows.append(ia)
                        cols.append(jb)
                        vals.append(blk[a, b])
            F = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
            C = F if C is None else C @ F
        B = sp.diags(E[tau]) @ C
        blocks[tau][tau] = sp.identity(N, format="csr", dtype=B.dtype)
        if tau >= 1:
            blocks[tau][tau - 1] = -B
        else:
            blocks[0][T - 1] = B
    return sp.bmat(blocks, format="csr")


def _sparse_normal_solve(M, Phi):
    """(M^T M)^{-1} Phi for the columns of Phi with one sparse LU of M:
    M^T w = Phi (plain transpose, so complex M stays analytic), then M u = w."""
    lu = spla.splu(M.tocsc())
    w = lu.solve(Phi.astype(M.dtype), trans="T")
    return lu.solve(w, trans="N")


def sparse_action(lat, g, x, Phi):
    """S_F = sum over fields of Phi . (M^T M)^{-1} Phi with a sparse LU of M (complex x allowed)."""
    M = sparse_M(lat, g, x)
    Phi = np.asarray(Phi).reshape(-1, lat.dim)
    u = _sparse_normal_solve(M, Phi.T)
    return np.sum(Phi.T * u)


def sparse_solve(lat, g, x, Phi):
    """u = (M^T M)^{-1} Phi by a sparse LU of M (Phi [..., Ltau, N], real x)."""
    M = sparse_M(lat, g, x)
    Phi = np.asarray(Phi)
    sh = Phi.shape
    u = _sparse_normal_solve(M, Phi.reshape(-1, lat.dim).T)
    return u.T.reshape(sh)


def directional_derivative(lat, g, x, Phi, direction, h=1e-20):
    """d S_F(x + s direction)/ds at s = 0 by one complex step of sparse_action."""
    xc = np.asarray(x, dtype=np.complex128) + 1j * h * np.asarray(direction)
    return float(np.imag(sparse_action(lat, g, xc, Phi)) / h)


# ------------------------------------------------------------- HMC with the SSH operator

def pseudofermions(lat, g, x, R_fields):
    """Phi_sigma = M(x)^T R_sigma (Eq. PhiSample-1 with A = M, the SSH-type M)."""
    M = sparse_M(lat, g, x)
    R = np.asarray(R_fields).reshape(-1, lat.dim)
    return (M.T @ R.T).T.reshape(np.shape(R_fields))


def hmc_action(lat, g, omega0, x, Phis):
    """S' = S_B - dtau alpha sum x + 1/2 sum_sigma Phi_sigma . (M^T M)^{-1} Phi_sigma."""
    from . import hmc as hmc_mod
    return hmc_mod.x_action(lat, x, omega0) + 0.5 * float(np.real(sparse_action(lat, g, x, Phis)))


def hmc_update(lat, g, omega0, m_reg, dt, Nt, nt, x_i, R_fields, R_mom, r_uniform):
    """One HMC trial update (Algorithm 1) of the action S' with the SSH-type M:
    the Holstein update's mass, momenta, time-step splitting and Metropolis
    test (oracle.hmc) with this operator's pseudofermions, action and force."""
    from . import hmc as hmc_mod
    x_i = np.asarray(x_i, dtype=np.float64)
    mt = hmc_mod.mass_tilde(lat.Ltau, lat.dtau, omega0, m_reg)
    p_i = hmc_mod.sample_momentum(R_mom, mt)
    Phis = pseudofermions(lat, g, x_i, R_fields)
    f_force = lambda x: 0.5 * force(lat, g, x, Phis)

    def ham(x, p):
        sb = hmc_mod.x_action(lat, x, omega0)
        sf = 0.5 * float(np.real(sparse_action(lat, g, x, Phis)))
        k = hmc_mod.kinetic_energy(p, mt)
        return {"H": sb + sf + k, "S_B": sb, "S_F": sf, "K": k}

    Hi = ham(x_i, p_i)
    x_f, p_f = hmc_mod.leapfrog_split(lat, omega0, mt, x_i, p_i, dt, Nt, nt, f_force)
    Hf = ham(x_f, p_f)
    dH = Hf["H"] - Hi["H"]
    prob = min(1.0, float(np.exp(-dH)))
    accepted = bool(r_uniform < prob)
    return {"x_f": x_f, "p_f": p_f, "p_i": p_i, "Phi": Phis, "H_i": Hi, "H_f": Hf, "dH": dH,
            "accept_prob": prob, "accepted": accepted, "x_out": x_f if accepted else x_i}
