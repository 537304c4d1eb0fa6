"""The adiabatic preconditioner P and its Chebyshev (KPM) apply.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 / complex128.

Definitions followed (Sec. V A and App. C):

* e^{-dtau Vbar} = (1/Ltau) sum_tau e^{-dtau V_tau}     (Eq. expnVbar)
  i.e. dbar_i = mean_tau E_{tau,i}, and Bbar = diag(dbar) C (Eq. Bbar).
* P has the block structure of M with every B_tau replaced by Bbar
  (Eq. P_def).
* U = F Theta, U_{w,tau} = exp(-2 pi i tau (w + 1/2) / Ltau) / sqrt(Ltau)
  (Eqs. udef, U_omega); in this basis P is block diagonal with blocks
  I - e^{-i phi_w} Bbar, phi_w = 2 pi (w + 1/2) / Ltau (Eqs. Mww, P_block),
  and P^{-1} v = U^dagger Ptilde^{-1} U v (Eq. P_change_basis).
* Each block inverse is f_w(A) with A = 2 (Bbar - bmin)/db - 1,
  f_w(y) = 1 / (1 - e^{-i phi_w} b(y)), b(y) = bmin + (y + 1) db / 2
  (Eqs. A_def, f_y), approximated by a truncated Chebyshev series with
  g_m = 1 whose coefficients come from Chebyshev-Gauss quadrature with
  N_Q = 2 N_P points (Eq. Cheby-Gauss) and whose order follows
  N_P = floor(db (a1/phi_w + a2)) (Eq. NP_heuristic), phi_w taken in
  (0, pi) through the symmetry f_{Ltau-1-w} = f_w^* (App. C).  The series
  is applied with the recurrence alpha_{m+1} = 2 A alpha_m - alpha_{m-1}
  (Eqs. Minv_KPM, alpha_recur).

Readings (the paper is silent or leaves a choice):
* N_P is clamped to at least 1 (the heuristic gives 0 for large phi when
  db is small).
* Spectral bounds: the paper estimates them with ~20 Arnoldi steps plus a
  5% margin.  The default here is a guaranteed enclosure instead:
  ||C|| and ||C^{-1}|| are at most e^{4 dtau |t|} (four bond families,
  each factor kron(C2, C2) with eigenvalues e^{+-2 dtau t} and 1), so every
  real eigenvalue of Bbar lies in [min(dbar) e^{-4 dtau|t|},
  max(dbar) e^{+4 dtau|t|}].  ``spectral_bounds_arnoldi`` gives the
  paper's estimate for comparison.
* F denotes the truncated-series approximation of P^{-1}; the
  preconditioner used inside CG is F F^T, where F^T is the exact transpose
  of F: the same series with conjugated coefficients in A^T.

Parity: the preconditioner only changes the speed of CG, never its
answer.  The pieces are pinned in tests by: the block-diagonal form of
U M U^dagger for tau-constant fields, the convergence of f_w(A) to the
exact block inverse as N_P grows, the closed-form Chebyshev coefficients of
1/(z - y), the matrix-vector count N_mat-vec/Ltau = 1.6 printed for
Ltau = 200 (App. C), and the exact transpose relation of F and F^T.
"""

import math

import numpy as np
import scipy.sparse as sp

from . import lattice as lat_mod


def dbar(lat, x):
    """dbar_i = (1/Ltau) sum_tau E_{tau,i}  (Eq. expnVbar)."""
    return np.mean(lat_mod.E_field(lat, x), axis=0)


def Bbar_dense(lat, x, C=None):
    """Dense Bbar = diag(dbar) C (Eq. Bbar)."""
    C = lat_mod.checkerboard_C(lat) if C is None else C
    return dbar(lat, x)[:, None] * C


def P_dense(lat, x, C=None):
    """Dense P of Eq. P_def: the structure of M with Bbar in every block."""
    Bb = Bbar_dense(lat, x, C)
    N, T = lat.N, lat.Ltau
    P = np.eye(N * T)
    for tau in range(1, T):
        P[tau * N:(tau + 1) * N, (tau - 1) * N:tau * N] = -Bb
    P[0:N, (T - 1) * N:T * N] = Bb
    return P


def spectral_bounds(lat, db):
    """Guaranteed enclosure [bmin, bmax] of the real spectrum of Bbar (see module doc)."""
    g = math.exp(4.0 * lat.dtau * abs(lat.t))
    return float(np.min(db)) / g, float(np.max(db)) * g


def spectral_bounds_arnoldi(lat, x, rng, iters=20, margin=0.05, C=None):
    """The paper's estimate (App. C): Arnoldi on Bbar and on Bbar^{-1}.

    bmax = (1 + margin) * max Re eig(H(Bbar)),
    bmin = 1 / ((1 + margin) * max Re eig(H(Bbar^{-1}))).
    """
    Bb = Bbar_dense(lat, x, C)
    Binv = np.linalg.inv(Bb)

    def top(A):
        n = A.shape[0]
        k = min(iters, n)
        Q = np.zeros((n, k + 1))
        H = np.zeros((k + 1, k))
        q = rng.standard_normal(n)
        Q[:, 0] = q / np.linalg.norm(q)
        for j in range(k):
            w = A @ Q[:, j]
            for i in range(j + 1):
                H[i, j] = Q[:, i] @ w
                w = w - H[i, j] * Q[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] < 1e-14:
                k = j + 1
                break
            Q[:, j + 1] = w / H[j + 1, j]
        return float(np.max(np.linalg.eigvals(H[:k, :k]).real))

    return 1.0 / ((1.0 + margin) * top(Binv)), (1.0 + margin) * top(Bb)


def phi_omega(w, Ltau):
    """phi_w = 2 pi (w + 1/2) / Ltau (Eq. Mww)."""
    return 2.0 * math.pi * (w + 0.5) / Ltau


def poly_order(w, Ltau, db, a1=1.0, a2=1.0):
    """N_P(w) = floor(db (a1/phi + a2)) with phi in (0, pi), clamped to >= 1."""
    wp = min(w, Ltau - 1 - w)
    n = math.floor(db * (a1 / phi_omega(wp, Ltau) + a2))
    return max(1, int(n))


def matvec_count(Ltau, db, a1=1.0, a2=1.0):
    """N_mat-vec = 2 sum_{w < Ltau/2} (N_P(w) - 1) without the clamp (App. C)."""
    total = 0
    for w in range(Ltau // 2):
        total += math.floor(db * (a1 / phi_omega(w, Ltau) + a2)) - 1
    return 2 * total


def matvec_bound(Ltau, db, a1=1.0, a2=1.0):
    """Upper bound of Eq. N_mv_bound: Ltau db [a1/pi (gamma + ln 2 Ltau) + a2] - Ltau."""
    gamma = 0.5772156649015329
    return Ltau * db * (a1 / math.pi * (gamma + math.log(2 * Ltau)) + a2) - Ltau


def cheb_coeffs(phi, bmin, bmax, NP):
    """Chebyshev-Gauss coefficients c_m, m < NP, of f(y) = 1/(1 - e^{-i phi} b(y))
    with N_Q = 2 NP abscissas theta_n = pi (n + 1/2)/N_Q (Eq. Cheby-Gauss)."""
    NQ = 2 * NP
    db = bmax - bmin
    theta = np.pi * (np.arange(NQ) + 0.5) / NQ
    b = bmin + (np.cos(theta) + 1.0) * db / 2.0
    f = 1.0 / (1.0 - np.exp(-1j * phi) * b)
    c = np.empty(NP, dtype=np.complex128)
    for m in range(NP):
        qm = (math.pi / 2.0) * (2.0 if m == 0 else 1.0)
        c[m] = math.pi / (qm * NQ) * np.sum(np.cos(m * theta) * f)
    return c


def U_matrix(Ltau):
    """U_{w,tau} = exp(-2 pi i tau (w + 1/2)/Ltau)/sqrt(Ltau) (Eq. U_omega)."""
    w = np.arange(Ltau)[:, None]
    tau = np.arange(Ltau)[None, :]
    return np.exp(-2j * np.pi * tau * (w + 0.5) / Ltau) / np.sqrt(Ltau)


class Preconditioner:
    """Tables of one field x: dbar, bounds, N_P(w) and c_m(w) for all w."""

    def __init__(self, lat, x, a1=1.0, a2=1.0, bounds=None, C=None):
        self.lat = lat
        self.C = lat_mod.checkerboard_C(lat) if C is None else C  # dense or CSR
        self.dbar = dbar(lat, x)
        self.bmin, self.bmax = spectral_bounds(lat, self.dbar) if bounds is None else bounds
        self.db = self.bmax - self.bmin
        self.NP = [poly_order(w, lat.Ltau, self.db, a1, a2) for w in range(lat.Ltau)]
        self.coef = [cheb_coeffs(phi_omega(w, lat.Ltau), self.bmin, self.bmax, self.NP[w])
                     for w in range(lat.Ltau)]
        if sp.issparse(self.C):
            self.Bbar = (sp.diags(self.dbar) @ self.C).tocsr()
            eye = sp.identity(lat.N, format="csr")
        else:
            self.Bbar = self.dbar[:, None] * self.C
            eye = np.eye(lat.N)
        self.U = U_matrix(lat.Ltau)
        self._A = None
        if self.db > 0.0:
            self._A = 2.0 * (self.Bbar - self.bmin * eye) / self.db - eye
            self._AT = self._A.T.tocsr() if sp.issparse(self._A) else self._A.T

    def A_matrix(self):
        """A = 2 (Bbar - bmin)/db - 1 (Eq. A_def)."""
        return self._A

    def block_apply(self, w, v, transpose=False):
        """sum_m c_m T_m(A) v by the three-term recurrence (Eqs. Minv_KPM, alpha_recur).

        With transpose=True: sum_m conj(c_m) T_m(A^T) v, the conjugate
        transpose of the same block.
        """
        c = self.coef[w]
        if transpose:
            c = np.conj(c)
        NP = len(c)
        out = c[0] * v
        if NP == 1:
            return out
        A = self._AT if transpose else self._A
        a_prev = v
        a_cur = A @ v
        out = out + c[1] * a_cur
        for m in range(2, NP):
            a_next = 2.0 * (A @ a_cur) - a_prev
            out = out + c[m] * a_next
            a_prev, a_cur = a_cur, a_next
        return out

    def apply_F(self, v, transpose=False):
        """F v (or F^T v) = U^dagger [blockdiag series] U v (Eq. P_change_basis).

        v is real [Ltau, N] (or [R, Ltau, N]); returns the real part (the
        imaginary part vanishes to rounding by the conjugate symmetry of
        the coefficients)."""
        v = np.asarray(v, dtype=np.float64)
        if v.ndim == 3:
            return np.stack([self.apply_F(vr, transpose) for vr in v])
        vh = self.U @ v
        wh = np.stack([self.block_apply(w, vh[w], transpose) for w in range(self.lat.Ltau)])
        out = self.U.conj().T @ wh
        return out.real

    def apply_FFt(self, v):
        """The CG preconditioner z = F (F^T v)."""
        return self.apply_F(self.apply_F(v, transpose=True))

    def F_dense(self, transpose=False):
        """Dense F (or F^T) built column by column; small lattices only."""
        d = self.lat.dim
        cols = []
        for k in range(d):
            e = np.zeros(d)
            e[k] = 1.0
            cols.append(self.apply_F(e.reshape(self.lat.Ltau, self.lat.N), transpose).reshape(d))
        return np.stack(cols, axis=1)
