"""Solves of the normal equations (M^T M) u = Phi and the action S_F.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

The action with one pseudofermion field and Lambda = I is
S_F = Phi^T (M^T M)^{-1} Phi = Phi . u  (Sec. II D, Eqs. S_F, Sf_Psi,
psi_def, CG; this is the paper's per-spin term times two, i.e. the
traditional action S' of Sec. IV).  The right-hand side used throughout is
Phi = M(x0)^T phi with Gaussian phi (Eq. PhiSample-1 with A = M), so at
x = x0 the solution is u = M^{-1} phi and S_F = |phi|^2.
"""

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

from . import lattice as lat_mod


def solve_dense(lat, x, Phi, C=None):
    """u = (M^T M)^{-1} Phi by LU of the dense M: w = M^{-T} Phi, u = M^{-1} w.

    M^T M is never formed (that would square the condition number).
    Phi may be [Ltau, N] or [R, Ltau, N].
    """
    M = lat_mod.dense_M(lat, x, C)
    lu = scipy.linalg.lu_factor(M)
    Phi = np.asarray(Phi)
    flat = Phi.reshape(-1, lat.dim).T
    w = scipy.linalg.lu_solve(lu, flat, trans=1)
    u = scipy.linalg.lu_solve(lu, w, trans=0)
    return u.T.reshape(Phi.shape)


def solve_sparse(lat, x, Phi, C=None):
    """Same solve with a sparse LU (SuperLU) of the CSR M."""
    M = lat_mod.sparse_M(lat, x, C).tocsc()
    lu = spla.splu(M)
    Phi = np.asarray(Phi)
    flat = Phi.reshape(-1, lat.dim)
    out = np.empty_like(flat)
    for r in range(flat.shape[0]):
        w = lu.solve(flat[r], trans="T")
        out[r] = lu.solve(w, trans="N")
    return out.reshape(Phi.shape)


def action(Phi, u):
    """S_F = Phi . u per right-hand side (Eqs. Sf_Psi and the identity Phi^T Psi = b^T v)."""
    Phi = np.asarray(Phi)
    u = np.asarray(u)
    return np.sum(Phi * u, axis=(-2, -1))


def rhs_from_phi(lat, x0, phi, C=None):
    """Phi = M(x0)^T phi (Eq. PhiSample-1 with A = M)."""
    return lat_mod.apply_MT(lat, x0, phi, C)


def relative_residual(matvec, b, u):
    """|b - A u| / |b| (the stopping quantity epsilon of Sec. V B)."""
    r = b - matvec(u)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def cg(matvec, b, tol=1e-12, maxiter=100000, precond=None, x0=None):
    """Textbook (preconditioned) conjugate gradient for an SPD operator.

    Used on A = M^T M (Sec. II D, Eq. CG) and, with ``precond`` = F F^T, in
    the preconditioned form of Sec. V A (Eq. CG_precon): each iteration
    applies A once and the preconditioner once.  Stops when the recursively
    updated residual satisfies |r| / |b| < tol.  Returns (u, iterations,
    history of |r|/|b|).
    """
    b = np.asarray(b, dtype=np.float64)
    u = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - matvec(u) if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0, [0.0]
    z = precond(r) if precond is not None else r
    p = z.copy()
    rz = float(np.vdot(r, z))
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while hist[-1] >= tol and it < maxiter:
        Ap = matvec(p)
        alpha = rz / float(np.vdot(p, Ap))
        u += alpha * p
        r -= alpha * Ap
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] < tol:
            break
        z = precond(r) if precond is not None else r
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return u, it, hist


def normal_matvec_sparse(lat, x, C=None):
    """v -> M^T M v with an explicitly assembled CSR M (shape [Ltau, N] in/out)."""
    M = lat_mod.sparse_M(lat, x, C)
    MT = M.T.tocsr()
    shape = (lat.Ltau, lat.N)

    def mv(v):
        return (MT @ (M @ np.asarray(v).reshape(-1))).reshape(shape)
    return mv


def solve_cg_sparse(lat, x, Phi, tol=1e-13, maxiter=200000, C=None):
    """Iterative oracle for sizes where no direct solve fits: textbook CG on
    the CSR M^T M to a tight tolerance.  Returns (u, iterations, final |r|/|b|).
    """
    mv = normal_matvec_sparse(lat, x, C)
    u, it, hist = cg(mv, Phi, tol=tol, maxiter=maxiter)
    return u, it, hist[-1]


def lanczos_condition_estimate(matvec, b, iters=200):
    """Estimate kappa(M^T M) from the Lanczos tridiagonal that CG builds.

    Runs plain CG for ``iters`` steps from b and forms the tridiagonal
    matrix T from the CG coefficients (the standard CG-Lanczos relation);
    the ratio of its extreme eigenvalues lower-bounds kappa.
    """
    b = np.asarray(b, dtype=np.float64)
    r = b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    alphas, betas = [], []
    for _ in range(iters):
        Ap = matvec(p)
        a = rr / float(np.vdot(p, Ap))
        r = r - a * Ap
        rr_new = float(np.vdot(r, r))
        bt = rr_new / rr
        alphas.append(a)
        betas.append(bt)
        p = r + bt * p
        rr = rr_new
        if rr_new == 0.0:
            break
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])
