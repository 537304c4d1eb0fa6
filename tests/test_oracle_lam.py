"""Pins of the CPU oracle's Lambda reformulation and global updates (Secs. II C, IV; App. B).

Each test checks the oracle against something other than itself: the
printed Lambda against its printed inverse and against the determinant
constraint, the matrix A^T printed in App. B and the symmetry D_x = D_{-x}
proved there, the action's b-form against its definition, the force
against complex-step derivatives of the definition, the reflection symmetry
of Delta S (Eq. Delta_S_sym) that the paper contrasts with S', closed forms
of the bosonic action change under the global moves, and the integrator's
properties with the Lambda action.  No GPU.
"""

import numpy as np
import pytest

from oracle import hmc as H
from oracle import lam as LA
from oracle import lattice as Lm


def lat_small(L=4, Ltau=8, dtau=0.1, t=1.0, mu=0.0, alpha=1.0):
    return Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)


def rand(shape, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("Ltau", [2, 6, 7, 12])
def test_lambda_times_inverse(Ltau):
    """Eq. (Lambda_def) times Eq. (Lambda_inv) is the identity."""
    lat = lat_small(Ltau=Ltau, alpha=1.3)
    x = rand((Ltau, lat.N), Ltau)
    P = (LA.lambda_sparse(lat, x) @ LA.lambda_inv_sparse(lat, x)).toarray()
    np.testing.assert_allclose(P, np.eye(lat.dim), atol=1e-13)


@pytest.mark.parametrize("Ltau", [4, 7, 10])
def test_lambda_determinant(Ltau):
    """Eq. (Lambda_constraint): det Lambda^2 = exp(dtau alpha sum x), and det Lambda > 0."""
    lat = lat_small(Ltau=Ltau, alpha=0.8, dtau=0.2)
    x = rand((Ltau, lat.N), 3)
    sign, logdet = np.linalg.slogdet(LA.lambda_sparse(lat, x).toarray())
    assert sign == 1.0
    assert 2 * logdet == pytest.approx(lat.dtau * lat.alpha * x.sum(), rel=1e-12, abs=1e-12)


def test_app_b_printed_matrices():
    """App. B: for t = 0, mu = 0 and a tau-constant field xbar, A^T = Lambda^T M^T is the
    matrix of Eq. (A_x) (diagonal Bbar^{1/2}, sub-diagonal -Bbar^{-1/2}, corner +Bbar^{-1/2},
    Bbar = exp(-dtau alpha xbar)) on every site, and D = A^T A is unchanged by xbar -> -xbar."""
    lat = lat_small(Ltau=6, t=0.0, mu=0.0, alpha=1.4)
    xbar = 0.63
    x = np.full((lat.Ltau, lat.N), xbar)
    Bb = np.exp(-lat.dtau * lat.alpha * xbar)
    T = lat.Ltau
    A1 = np.zeros((T, T))
    for tau in range(T):
        A1[tau, tau] = Bb ** 0.5
        if tau >= 1:
            A1[tau, tau - 1] = -Bb ** -0.5
    A1[0, T - 1] = Bb ** -0.5
    AT = LA.dense_A(lat, x).T
    np.testing.assert_allclose(AT, np.kron(A1, np.eye(lat.N)), atol=1e-14)
    D = lambda v: LA.dense_A(lat, v).T @ LA.dense_A(lat, v)
    np.testing.assert_allclose(D(x), D(-x), atol=1e-13)


def test_action_b_form_equals_definition():
    """1/2 b.(M^T M)^{-1} b with b = Lambda^{-T} Phi equals 1/2 |A^{-T} Phi|^2 (Eq. S_F)."""
    lat = lat_small(L=4, Ltau=10, mu=0.2, alpha=1.2)
    x = rand((lat.Ltau, lat.N), 5, 0.7)
    Phis = rand((2, lat.Ltau, lat.N), 6)
    assert LA.fermion_action(lat, x, Phis) == pytest.approx(LA.action_definition(lat, x, Phis), rel=1e-12)


def test_pseudofermion_action_at_draw():
    """Phi = A(x)^T R gives S_F(x) = |R|^2/2 (Sec. II D)."""
    lat = lat_small(L=4, Ltau=8, mu=-0.1)
    x = rand((lat.Ltau, lat.N), 8, 0.6)
    R = rand((2, lat.Ltau, lat.N), 9)
    Phis = LA.pseudofermions(lat, x, R)
    assert LA.fermion_action(lat, x, Phis) == pytest.approx(0.5 * np.sum(R * R), rel=1e-12)


def test_force_complex_step():
    """The force (adjoint M part plus the Lambda term) against complex-step derivatives of
    the definition, at components in the first slice (wrap of the Lambda shift), the last
    slice and the middle."""
    lat = lat_small(L=4, Ltau=8, mu=0.1, alpha=1.1)
    x = rand((lat.Ltau, lat.N), 11, 0.5)
    Phis = rand((2, lat.Ltau, lat.N), 12)
    comps = [(0, 0), (0, 5), (lat.Ltau - 1, 3), (4, 9), (1, 15)]
    g = LA.fermion_force(lat, x, Phis)
    cs = LA.force_complex_step(lat, x, Phis, comps)
    np.testing.assert_allclose([g[c] for c in comps], cs, rtol=1e-10, atol=1e-12)


def test_reflection_symmetry_single_site_adiabatic():
    """Eq. (Delta_S_sym): in the single-site (t = 0), half-filled, tau-constant limit,
    Delta S(xbar) = Delta S(-xbar) for every Phi drawn at x0 with the action S, while the
    action S' breaks the symmetry (Sec. IV)."""
    lat = lat_small(L=4, Ltau=20, t=0.0, mu=0.0, alpha=1.4142135623730951, dtau=0.1)
    w0 = 1.0
    x0 = np.full((lat.Ltau, lat.N), lat.alpha / w0 ** 2)
    R = rand((2, lat.Ltau, lat.N), 21)
    xb = np.full_like(x0, 0.9)
    # action S (A = M Lambda)
    Phis = LA.pseudofermions(lat, x0, R)
    S = lambda v: H.bosonic_action(lat, v, w0) + LA.fermion_action(lat, v, Phis)
    assert S(xb) - S(x0) == pytest.approx(S(-xb) - S(x0), abs=1e-9)
    # action S' (A = M): no such symmetry
    Phis2 = H.pseudofermions(lat, x0, R)
    S2 = lambda v: H.x_action(lat, v, w0) + H.fermion_action(lat, v, Phis2)
    assert abs((S2(xb) - S2(x0)) - (S2(-xb) - S2(x0))) > 1.0


def test_global_moves_closed_forms():
    """Reflection and swap are involutions; the swap leaves S_B and sum x unchanged; a
    reflection of site i changes the linear term of S' by 2 dtau alpha sum_tau x_{i,tau}."""
    lat = lat_small(L=4, Ltau=8, alpha=1.2)
    x = rand((lat.Ltau, lat.N), 30)
    w0 = 0.8
    assert np.array_equal(LA.reflect(LA.reflect(x, 3), 3), x)
    assert np.array_equal(LA.swap(LA.swap(x, 2, 6), 2, 6), x)
    assert H.bosonic_action(lat, LA.swap(x, 2, 6), w0) == pytest.approx(H.bosonic_action(lat, x, w0), rel=1e-14)
    assert H.bosonic_action(lat, LA.reflect(x, 3), w0) == pytest.approx(H.bosonic_action(lat, x, w0), rel=1e-14)
    d = H.linear_action(lat, LA.reflect(x, 3)) - H.linear_action(lat, x)
    assert d == pytest.approx(2 * lat.dtau * lat.alpha * x[:, 3].sum(), rel=1e-12)


def test_global_update_decision():
    """The update's Delta S equals the difference of the two actions evaluated by their
    definitions, S_F(x) = |R|^2/2, and the decision follows r < exp(-Delta S)."""
    lat = lat_small(L=4, Ltau=8, alpha=1.0, mu=0.0)
    x = rand((lat.Ltau, lat.N), 40, 0.8)
    R = rand((2, lat.Ltau, lat.N), 41)
    w0 = 1.0
    for kind, sites in (("reflect", (5,)), ("swap", (1, 2))):
        out = LA.global_update(lat, w0, x, kind, sites, R, 0.3)
        Phis = LA.pseudofermions(lat, x, R)
        ref = (H.bosonic_action(lat, out["x_prop"], w0) + LA.action_definition(lat, out["x_prop"], Phis)
               - H.bosonic_action(lat, x, w0) - LA.action_definition(lat, x, Phis))
        assert out["dS"] == pytest.approx(ref, rel=1e-10, abs=1e-10)
        assert out["S_F_old"] == pytest.approx(0.5 * np.sum(R * R), rel=1e-12)
        assert out["accepted"] == (0.3 < np.exp(-out["dS"]))


def test_hmc_with_lambda_reversible_and_second_order():
    """The split leapfrog with the Lambda action: reversible, energy error O(dt^2)."""
    lat = lat_small(L=4, Ltau=8, mu=0.1, alpha=1.0)
    x = rand((lat.Ltau, lat.N), 50, 0.5)
    R = rand((2, lat.Ltau, lat.N), 51)
    Phis = LA.pseudofermions(lat, x, R)
    w0 = 1.0
    mt = H.mass_tilde(lat.Ltau, lat.dtau, w0, w0)
    f = lambda v: LA.fermion_force(lat, v, Phis)
    b = lambda v: H.bosonic_force(lat, v, w0)
    p = H.sample_momentum(rand(x.shape, 52), mt)
    x1, p1 = H.leapfrog_split(lat, w0, mt, x, p, 0.05, 6, 3, f, b)
    x2, p2 = H.leapfrog_split(lat, w0, mt, x1, -p1, 0.05, 6, 3, f, b)
    np.testing.assert_allclose(x2, x, atol=1e-11)
    H0 = H.hamiltonian(lat, w0, mt, x, p, Phis, lam=True)["H"]
    dH = []
    for Nt in (10, 20):
        xa, pa = H.leapfrog_split(lat, w0, mt, x, p, 0.5 / Nt, Nt, 4, f, b)
        dH.append(abs(H.hamiltonian(lat, w0, mt, xa, pa, Phis, lam=True)["H"] - H0))
    assert 3.0 < dH[0] / dH[1] < 5.0
