"""Pins of the CPU oracle's operator, solve, action and force.

Each test checks the oracle against something other than itself: an
identity printed in the paper, a closed form, a special case that reduces
to a library routine, or brute force.  No GPU.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import force as F
from oracle import lattice as Lm
from oracle import solve as S
from workloads import gaussian_rhs, get_config, perturbed_field, phonon_field

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def lat_small(L=4, Ltau=8, dtau=0.1, t=1.0, mu=0.0, alpha=1.0):
    return Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)


def rand_field(lat, seed, scale=1.0, shift=0.0):
    return shift + scale * np.random.default_rng(seed).standard_normal((lat.Ltau, lat.N))


# ---------------------------------------------------------------- lattice --

def test_K_spectrum_extremes():
    """App. C: on the square lattice with t = 1 the extreme eigenvalues of K are +-4."""
    g = json.load(open(GOLD))["K_extremes"]
    for L in (4, 6, 8):
        ev = np.linalg.eigvalsh(Lm.hopping_matrix(L, g["t"]))
        assert ev[0] == pytest.approx(g["min"], abs=1e-12)
        assert ev[-1] == pytest.approx(g["max"], abs=1e-12)


def test_K_matches_plane_waves():
    """K is diagonal in lattice Fourier modes with eps_k = -2t (cos kx + cos ky)."""
    L, t = 6, 0.7
    K = Lm.hopping_matrix(L, t)
    ks = 2 * np.pi * np.arange(L) / L
    eps = sorted(-2 * t * (np.cos(kx) + np.cos(ky)) for kx in ks for ky in ks)
    assert np.allclose(np.linalg.eigvalsh(K), eps, atol=1e-12)


@pytest.mark.parametrize("dtau,t", [(0.1, 1.0), (0.05, 1.0), (0.3, 0.7)])
def test_checkerboard_exact_at_L4(dtau, t):
    """At L = 4 the two bond groups commute, so C = exp(-dtau K) exactly."""
    lat = lat_small(L=4, dtau=dtau, t=t)
    assert np.abs(Lm.checkerboard_C(lat) - Lm.exact_expK(lat)).max() < 1e-14


def test_checkerboard_factor_closed_form():
    """Each plaquette block of a factor equals kron(C2, C2) with
    C2 = [[cosh(dtau t), sinh(dtau t)], [sinh, cosh]] (hopping -t, so
    -dtau K has +dtau t off the diagonal)."""
    lat = lat_small(L=8, dtau=0.13, t=1.1)
    ch, sh = math.cosh(lat.dtau * lat.t), math.sinh(lat.dtau * lat.t)
    C2 = np.array([[ch, sh], [sh, ch]])
    blk = np.kron(C2, C2)
    PA, PB = Lm.checkerboard_factors(lat)
    for P, group in ((PA, "A"), (PB, "B")):
        ref = np.zeros((lat.N, lat.N))
        for sites in Lm.plaquettes(lat.L, group):
            # local order (corner, +x, +y, +x+y) = index dx + 2 dy; kron(C2_y, C2_x)
            for a in range(4):
                for b in range(4):
                    ref[sites[a], sites[b]] = blk[a, b]
        assert np.abs(P - ref).max() < 1e-14
        assert np.abs(Lm.sparse_factor(lat, group).toarray() - ref).max() < 1e-14


def test_checkerboard_groups_cover_each_bond_once():
    """The plaquettes of groups A and B hold every nearest-neighbour bond once."""
    L = 8
    K = Lm.hopping_matrix(L, 1.0)
    KA = Lm.group_hopping(L, 1.0, "A")
    KB = Lm.group_hopping(L, 1.0, "B")
    assert np.array_equal(KA + KB, K)
    assert np.array_equal(KA, KA.T) and np.array_equal(KB, KB.T)
    assert np.abs(KA @ KB - KB @ KA).max() > 0 or L == 4
    assert np.count_nonzero(KA * KB) == 0


@pytest.mark.parametrize("L", [6, 8])
def test_checkerboard_error_is_order_dtau2(L):
    """|C - exp(-dtau K)| = O(dtau^2) (Sec. II D): local slope ~ 2."""
    errs = []
    dts = [0.1, 0.05, 0.025]
    for dt in dts:
        lat = lat_small(L=L, dtau=dt)
        errs.append(np.linalg.norm(Lm.checkerboard_C(lat) - Lm.exact_expK(lat), 2))
    slopes = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert all(1.9 < s < 2.1 for s in slopes), slopes


def test_checkerboard_not_symmetric_beyond_L4():
    """App. C: the checkerboard approximation slightly breaks Hermiticity."""
    lat = lat_small(L=6)
    C = Lm.checkerboard_C(lat)
    assert np.abs(C - C.T).max() > 1e-4
    assert np.abs(np.linalg.eigvals(C).imag).max() < 1e-10


# --------------------------------------------------------------- matrix M --

@pytest.mark.parametrize("L,Ltau", [(4, 8), (6, 6), (4, 40)])
def test_det_identity(L, Ltau):
    """det M = det(I + B_{Ltau-1} ... B_0) (Eq. detM_alt); pins the block layout
    and the sign of the corner block."""
    lat = lat_small(L=L, Ltau=Ltau)
    x = rand_field(lat, 1)
    s1, ld1 = np.linalg.slogdet(Lm.dense_M(lat, x))
    s2, ld2 = Lm.det_M_via_product(lat, x)
    assert s1 == s2
    assert ld1 == pytest.approx(ld2, rel=1e-10)


def test_det_identity_catches_wrong_corner_sign():
    """A corner block -B_0 (periodic instead of antiperiodic) violates Eq. detM_alt."""
    lat = lat_small(L=4, Ltau=6)
    x = rand_field(lat, 2)
    M = Lm.dense_M(lat, x)
    N = lat.N
    M[0:N, (lat.Ltau - 1) * N:] *= -1.0
    _, ld_bad = np.linalg.slogdet(M)
    _, ld = Lm.det_M_via_product(lat, x)
    assert abs(ld_bad - ld) > 1e-3


def free_electron_eps(L, t):
    k = 2 * np.pi * np.arange(L) / L
    # site i = x + L y  ->  fft2 over axes (y, x) of a [L, L] array
    return -2 * t * (np.cos(k)[None, :] + np.cos(k)[:, None])


@pytest.mark.parametrize("L,Ltau,mu,use_cb", [(4, 10, 0.0, True), (4, 12, -0.3, True),
                                             (6, 8, 0.2, False)])
def test_free_electron_logdet(L, Ltau, mu, use_cb):
    """x = 0: log det M = sum_k log(1 + exp(-beta (eps_k - mu))) (Eq. detM_alt
    with B = e^{dtau mu} e^{-dtau K}).  At L = 4 the checkerboard is exact."""
    lat = lat_small(L=L, Ltau=Ltau, mu=mu)
    C = Lm.checkerboard_C(lat) if use_cb else Lm.exact_expK(lat)
    x = np.zeros((Ltau, lat.N))
    _, ld = np.linalg.slogdet(Lm.dense_M(lat, x, C))
    beta = Ltau * lat.dtau
    eps = free_electron_eps(L, lat.t)
    ref = np.sum(np.log1p(np.exp(-beta * (eps - mu))))
    assert ld == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("L,Ltau,mu,use_cb", [(4, 10, 0.0, True), (6, 8, 0.25, False)])
def test_free_electron_solve_closed_form(L, Ltau, mu, use_cb):
    """x = 0: M is diagonal in (k, w) with m = 1 - e^{-i phi_w} e^{-dtau (eps_k - mu)}
    (Eqs. U_omega, Mww with Bbar = B), so u = W^dag |m|^{-2} W Phi, computed
    here with numpy FFTs (twisted DFT in tau, 2-D DFT in space)."""
    lat = lat_small(L=L, Ltau=Ltau, mu=mu)
    C = Lm.checkerboard_C(lat) if use_cb else Lm.exact_expK(lat)
    x = np.zeros((Ltau, lat.N))
    Phi = np.random.default_rng(3).standard_normal((Ltau, lat.N))
    u = S.solve_dense(lat, x, Phi, C)

    tau = np.arange(Ltau)
    twist = np.exp(-1j * np.pi * tau / Ltau)[:, None, None]
    P = Phi.reshape(Ltau, L, L)
    Pk = np.fft.fft2(P, axes=(1, 2), norm="ortho")
    Pkw = np.fft.fft(twist * Pk, axis=0, norm="ortho")
    phi_w = 2 * np.pi * (np.arange(Ltau) + 0.5) / Ltau
    eps = free_electron_eps(L, lat.t)
    m = 1 - np.exp(-1j * phi_w)[:, None, None] * np.exp(-lat.dtau * (eps - mu))[None]
    Ukw = Pkw / np.abs(m) ** 2
    Uk = np.conj(twist) * np.fft.ifft(Ukw, axis=0, norm="ortho")
    ref = np.fft.ifft2(Uk, axes=(1, 2), norm="ortho").real.reshape(Ltau, lat.N)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-12


def test_single_site_limit_t0():
    """t = 0: M splits into N scalar cyclic systems, det M = prod_i (1 +
    exp(-dtau sum_tau (alpha x - mu))) (Sec. IV, Eq. SDQMC_def with the sum
    over tau = 0..Ltau-1), and M^{-1} is a scalar recurrence."""
    lat = lat_small(L=4, Ltau=12, t=0.0, mu=0.3, alpha=1.3)
    x = rand_field(lat, 4, scale=0.7)
    _, ld = np.linalg.slogdet(Lm.dense_M(lat, x))
    ref = np.sum(np.log1p(np.exp(-lat.dtau * np.sum(lat.alpha * x - lat.mu, axis=0))))
    assert ld == pytest.approx(ref, rel=1e-12)

    E = np.exp(-lat.dtau * (lat.alpha * x - lat.mu))
    Phi = np.random.default_rng(5).standard_normal((lat.Ltau, lat.N))

    def solve_M(w):   # v_tau = w_tau + E_tau v~_{tau-1}, v~_{-1} = -v_{L-1}
        T = lat.Ltau
        a = np.empty_like(w)
        c = np.empty_like(w)
        a[0], c[0] = w[0], -E[0]
        for tau in range(1, T):
            a[tau] = w[tau] + E[tau] * a[tau - 1]
            c[tau] = E[tau] * c[tau - 1]
        vlast = a[T - 1] / (1 - c[T - 1])
        return a + c * vlast

    def solve_MT(w):  # v_tau = w_tau + E_{tau+1} v~_{tau+1}, v~_{T} = -v_0
        T = lat.Ltau
        a = np.empty_like(w)
        c = np.empty_like(w)
        a[T - 1], c[T - 1] = w[T - 1], -E[0]
        for tau in range(T - 2, -1, -1):
            a[tau] = w[tau] + E[tau + 1] * a[tau + 1]
            c[tau] = E[tau + 1] * c[tau + 1]
        v0 = a[0] / (1 - c[0])
        return a + c * v0

    ref_u = solve_M(solve_MT(Phi))
    u = S.solve_dense(lat, x, Phi)
    assert np.abs(u - ref_u).max() / np.abs(ref_u).max() < 1e-13


def test_dense_sparse_and_block_applies_agree():
    lat = lat_small(L=6, Ltau=6, mu=0.1, alpha=1.2)
    x = rand_field(lat, 6)
    M = Lm.dense_M(lat, x)
    Ms = Lm.sparse_M(lat, x).toarray()
    assert np.abs(M - Ms).max() < 1e-14
    v = np.random.default_rng(7).standard_normal((2, lat.Ltau, lat.N))
    for r in range(2):
        assert np.allclose(Lm.apply_M(lat, x, v)[r].reshape(-1), M @ v[r].reshape(-1), atol=1e-13)
        assert np.allclose(Lm.apply_MT(lat, x, v)[r].reshape(-1), M.T @ v[r].reshape(-1), atol=1e-13)


def test_normal_matrix_spd():
    """M^T M is symmetric positive definite (Sec. II D): Cholesky succeeds."""
    p = get_config("c1")
    lat = Lm.Lattice.from_params(p)
    M = Lm.dense_M(lat, phonon_field(p))
    A = M.T @ M
    scipy.linalg.cholesky(A)
    assert np.linalg.eigvalsh(A)[0] > 0


# ------------------------------------------------------- solve and action --

def test_action_equals_phi_norm_at_x0():
    """Phi = M(x0)^T phi  =>  S_F(x0) = |phi|^2 (Sec. II D, after Eq. Delta_S_F)."""
    p = get_config("c1")
    lat = Lm.Lattice.from_params(p)
    x0 = phonon_field(p)
    phi = gaussian_rhs(p, 3)
    Phi = S.rhs_from_phi(lat, x0, phi)
    u = S.solve_dense(lat, x0, Phi)
    assert np.allclose(S.action(Phi, u), np.sum(phi ** 2, axis=(1, 2)), rtol=1e-12)


def test_dense_sparse_cg_solves_agree():
    p = get_config("c1")
    lat = Lm.Lattice.from_params(p)
    x = perturbed_field(p, phonon_field(p))
    Phi = np.random.default_rng(8).standard_normal((lat.Ltau, lat.N))
    u1 = S.solve_dense(lat, x, Phi)
    u2 = S.solve_sparse(lat, x, Phi)
    u3, it, res = S.solve_cg_sparse(lat, x, Phi, tol=1e-14)
    assert np.linalg.norm(u1 - u2) / np.linalg.norm(u1) < 1e-12
    assert np.linalg.norm(u1 - u3) / np.linalg.norm(u1) < 1e-9
    M = Lm.dense_M(lat, x)
    r = Phi.reshape(-1) - M.T @ (M @ u1.reshape(-1))
    assert np.linalg.norm(r) / np.linalg.norm(Phi) < 1e-12


def test_lanczos_condition_estimate():
    p = get_config("c1")
    lat = Lm.Lattice.from_params(p)
    x = phonon_field(p)
    M = Lm.dense_M(lat, x)
    A = M.T @ M
    kappa = np.linalg.cond(A)
    b = np.random.default_rng(9).standard_normal(lat.dim)
    est = S.lanczos_condition_estimate(lambda v: A @ v, b, iters=400)
    assert 0.5 * kappa < est <= kappa * (1 + 1e-6)


# ------------------------------------------------------------------ force --

def test_force_adjoint_matches_complex_step():
    """Eq. dSF_dx (adjoint form) vs complex-step derivatives of S_F."""
    lat = lat_small(L=4, Ltau=6, mu=0.2, alpha=1.3)
    x0 = rand_field(lat, 10)
    x = x0 + 0.1 * rand_field(lat, 11)
    phi = np.random.default_rng(12).standard_normal((lat.Ltau, lat.N))
    Phi = S.rhs_from_phi(lat, x0, phi)
    u = S.solve_dense(lat, x, Phi)
    g = F.force_from_solution(lat, x, u)
    gcs = F.force_complex_step(lat, x, Phi)
    assert np.linalg.norm(g - gcs) / np.linalg.norm(gcs) < 1e-12


def test_force_complex_step_matches_central_fd():
    lat = lat_small(L=4, Ltau=4, mu=-0.1, alpha=0.9)
    x = rand_field(lat, 13)
    Phi = np.random.default_rng(14).standard_normal((lat.Ltau, lat.N))
    comps = [(0, 0), (1, 5), (3, 15), (2, 7)]
    gcs = F.force_complex_step(lat, x, Phi)
    gfd = F.force_central_fd(lat, x, Phi, comps, h=1e-3)
    ref = np.array([gcs[c] for c in comps])
    assert np.abs(gfd - ref).max() / np.abs(ref).max() < 1e-7


def test_force_t0_against_scalar_closed_form():
    """t = 0: S_F is a sum of independent single-site terms; central FD of
    the scalar recurrence solution pins the force formula."""
    lat = lat_small(L=4, Ltau=10, t=0.0, mu=0.1, alpha=1.4)
    x = rand_field(lat, 15)
    Phi = np.random.default_rng(16).standard_normal((lat.Ltau, lat.N))

    def S_site(xs, b):
        E = np.exp(-lat.dtau * (lat.alpha * xs - lat.mu))
        T = lat.Ltau
        # w = M^{-T} b
        a = np.empty(T)
        c = np.empty(T)
        a[T - 1], c[T - 1] = b[T - 1], -E[0]
        for tau in range(T - 2, -1, -1):
            a[tau] = b[tau] + E[tau + 1] * a[tau + 1]
            c[tau] = E[tau + 1] * c[tau + 1]
        w = a + c * (a[0] / (1 - c[0]))
        return float(w @ w)   # Phi^T (M^T M)^{-1} Phi = |M^{-T} Phi|^2

    u = S.solve_dense(lat, x, Phi)
    g = F.force_from_solution(lat, x, u)
    h = 1e-5
    for i in (0, 3, 9):
        for tau in (0, 4, 9):
            xp, xm = x[:, i].copy(), x[:, i].copy()
            xp[tau] += h
            xm[tau] -= h
            fd = (S_site(xp, Phi[:, i]) - S_site(xm, Phi[:, i])) / (2 * h)
            assert g[tau, i] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_force_multi_rhs_shape():
    lat = lat_small(L=4, Ltau=4)
    x = rand_field(lat, 17)
    u = np.random.default_rng(18).standard_normal((3, lat.Ltau, lat.N))
    g = F.force_from_solution(lat, x, u)
    assert g.shape == u.shape
    for r in range(3):
        assert np.allclose(g[r], F.force_from_solution(lat, x, u[r]))


def test_stored_full_size_values_match_sparse_direct_solve():
    """The stored L=16, Ltau=160 values (written by the oracle's CG) against
    a sparse LU solve of M and M^T at full size: two independent solvers."""
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c2.json")))
    p = get_config("c2")
    lat = Lm.Lattice.from_params(p)
    x0 = phonon_field(p)
    x = perturbed_field(p, x0)
    Cs = Lm.sparse_C(lat)
    phi = gaussian_rhs(p, 1)[0]
    Phi = (Lm.sparse_M(lat, x0, Cs).T @ phi.reshape(-1)).reshape(lat.Ltau, lat.N)
    u = S.solve_sparse(lat, x, Phi[None], Cs)[0]
    idx = np.array(ref["samples"])
    us = u[idx[:, 0], idx[:, 1]]
    assert np.linalg.norm(us - ref["u_samples"]) <= 1e-10 * np.linalg.norm(ref["u_samples"])
    assert abs(float(np.sum(Phi * u)) - ref["S_F"]) <= 1e-12 * abs(ref["S_F"])
    assert float(np.linalg.norm(u)) == pytest.approx(ref["u_norm"], rel=1e-11)
