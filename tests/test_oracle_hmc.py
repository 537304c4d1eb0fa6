"""Pins of the CPU oracle's hybrid Monte Carlo update (Sec. III, Algorithm 1).

Each test checks the oracle against something other than itself: closed
forms of the bosonic action, finite differences of every action against its
force, the Fourier-basis form of Q against the tau-stencil, values the paper
states for the extreme Fourier modes and the mass-matrix limits, the exact
harmonic motion of a purely bosonic system, and the three properties the
paper requires of the integrator (time reversibility, volume conservation,
energy error of order dt^2).  No GPU.
"""

import json
import os

import numpy as np
import pytest

from oracle import hmc as H
from oracle import lattice as Lm
from workloads import get_config, hmc_draws, hmc_params, phonon_field

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def lat_small(L=4, Ltau=8, dtau=0.1, t=1.0, mu=0.0, alpha=1.0):
    return Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)


def rand(shape, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal(shape)


def central_fd(f, x, comps, h=1e-3):
    out = []
    for tau, i in comps:
        xp = x.copy()
        xm = x.copy()
        xp[tau, i] += h
        xm[tau, i] -= h
        out.append((f(xp) - f(xm)) / (2 * h))
    return np.array(out)


# ------------------------------------------------------------ bosonic action --

def test_sb_constant_field():
    """A tau- and site-constant field has no kinetic term: S_B = dtau N Ltau omega0^2 c^2 / 2."""
    lat = lat_small(Ltau=10, dtau=0.05)
    c, w0 = 0.7, 1.3
    x = np.full((lat.Ltau, lat.N), c)
    assert H.bosonic_action(lat, x, w0) == pytest.approx(0.5 * lat.dtau * lat.N * lat.Ltau * w0 ** 2 * c * c,
                                                         rel=1e-14)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_sb_single_mode(k):
    """x_tau = A cos(theta tau + phi_i), theta = 2 pi k / Ltau: sum of cos^2 is Ltau/2 and
    x_{tau+1} - x_tau = -2 A sin(theta/2) sin(theta tau + theta/2 + phi), so
    S_B = N A^2 Ltau/4 * dtau (omega0^2 + 4 sin^2(pi k/Ltau)/dtau^2); this is N A^2 Ltau/4 * Qtilde_k."""
    lat = lat_small(Ltau=20, dtau=0.1)
    A, w0 = 0.9, 0.6
    phase = np.random.default_rng(k).uniform(0, 2 * np.pi, lat.N)
    tau = np.arange(lat.Ltau)[:, None]
    x = A * np.cos(2 * np.pi * k * tau / lat.Ltau + phase[None, :])
    closed = lat.N * A * A * lat.Ltau / 4 * lat.dtau * (w0 ** 2 + 4 * np.sin(np.pi * k / lat.Ltau) ** 2 / lat.dtau ** 2)
    assert H.bosonic_action(lat, x, w0) == pytest.approx(closed, rel=1e-13)
    qt = H.q_tilde(lat.Ltau, lat.dtau, w0)
    assert closed == pytest.approx(lat.N * A * A * lat.Ltau / 4 * qt[k], rel=1e-13)


def test_linear_action_closed_form():
    lat = lat_small(Ltau=6, alpha=1.7, dtau=0.2)
    x = np.full((lat.Ltau, lat.N), -0.4)
    assert H.linear_action(lat, x) == pytest.approx(-0.2 * 1.7 * (-0.4) * lat.N * lat.Ltau, rel=1e-14)


def test_bosonic_force_fd():
    """dS_B/dx (Eq. dSB_dx) against central differences of S_B (Eq. S_B); S_B is quadratic,
    so the difference quotient is exact up to rounding.  Components include both tau wraps."""
    lat = lat_small(Ltau=12, dtau=0.1)
    x = rand((lat.Ltau, lat.N), 1)
    w0 = 0.8
    comps = [(0, 0), (lat.Ltau - 1, 3), (5, 7), (1, lat.N - 1)]
    fd = central_fd(lambda v: H.bosonic_action(lat, v, w0), x, comps)
    g = H.bosonic_force(lat, x, w0)
    np.testing.assert_allclose([g[c] for c in comps], fd, rtol=1e-8, atol=1e-9)
    fd2 = central_fd(lambda v: H.x_action(lat, v, w0), x, comps)
    g2 = H.x_force(lat, x, w0)
    np.testing.assert_allclose([g2[c] for c in comps], fd2, rtol=1e-8, atol=1e-9)


# -------------------------------------------------------------- Fourier basis --

def test_q_fourier_equals_stencil():
    """Eq. (bosonic_force): F^{-1} Qtilde F x equals the tau-stencil of Eq. (dSB_dx)."""
    for Ltau, dtau, w0 in ((12, 0.1, 1.0), (40, 0.05, 0.3), (7 * 2, 0.2, 2.0)):
        lat = lat_small(Ltau=Ltau, dtau=dtau)
        x = rand((Ltau, lat.N), Ltau)
        np.testing.assert_allclose(H.tau_fourier_apply(x, H.q_tilde(Ltau, dtau, w0)),
                                   H.bosonic_force(lat, x, w0), rtol=1e-12, atol=1e-12)


def test_q_extremes_paper_values():
    """The values the paper states for the slowest and fastest modes and their ratio."""
    g = json.load(open(GOLD))["Q_extremes"]
    for c in g["cases"]:
        qt = H.q_tilde(40, c["dtau"], c["omega0"]) / c["dtau"]
        assert qt[20] == pytest.approx(c["w_half"], rel=1e-13)
        assert qt[0] == pytest.approx(c["w_zero"], rel=1e-13)
        assert qt.max() == pytest.approx(qt[20], rel=1e-15)
        assert qt[20] / qt[0] == pytest.approx(c["ratio"], rel=1e-12)


def test_mass_limits():
    """Sec. III B 1: M -> dtau I as m_reg -> infinity; M = Q/omega0^2 at m_reg = 0."""
    Ltau, dtau, w0 = 40, 0.1, 0.7
    assert np.all(H.mass_tilde(Ltau, dtau, w0, None) == dtau)
    np.testing.assert_allclose(H.mass_tilde(Ltau, dtau, w0, 1e7), dtau, rtol=1e-9)
    np.testing.assert_allclose(H.mass_tilde(Ltau, dtau, w0, 0.0), H.q_tilde(Ltau, dtau, w0) / w0 ** 2,
                               rtol=1e-14)
    mt = H.mass_tilde(Ltau, dtau, w0, w0)
    assert mt[0] == pytest.approx(dtau, rel=1e-14)       # constant at w = 0
    assert np.all(mt > 0)
    np.testing.assert_allclose(mt[1:], mt[1:][::-1], rtol=1e-14)   # even in w


def test_mass_matrix_spectrum_and_sqrt():
    """The dense tau-matrix of the mass is symmetric with eigenvalues equal to Mtilde (checked
    with a symmetric eigensolver, not a Fourier transform); sqrt(M) sqrt(M) = M;
    p = sqrt(M) R gives p^T M^{-1} p = |R|^2."""
    Ltau, dtau, w0 = 10, 0.1, 1.0
    mt = H.mass_tilde(Ltau, dtau, w0, w0)
    Mdense = np.stack([H.tau_fourier_apply(np.eye(Ltau)[:, j:j + 1], mt)[:, 0] for j in range(Ltau)], axis=1)
    np.testing.assert_allclose(Mdense, Mdense.T, atol=1e-14)
    np.testing.assert_allclose(np.linalg.eigvalsh(Mdense), np.sort(mt), rtol=1e-12)
    R = rand((Ltau, 5), 3)
    p = H.sample_momentum(R, mt)
    np.testing.assert_allclose(H.sample_momentum(p, mt), Mdense @ R, rtol=1e-12, atol=1e-13)
    assert H.kinetic_energy(p, mt) == pytest.approx(0.5 * np.sum(R * R), rel=1e-12)


# ------------------------------------------------------------------ dynamics --

def test_harmonic_motion_with_q_mass():
    """S = S_B only (alpha = 0) and M = Q/omega0^2 (m_reg = 0): every mode obeys
    x'' = -omega0^2 x, so x(T) = x0 cos(omega0 T) + M^{-1} p0 sin(omega0 T)/omega0.
    The leapfrog error is O(dt^2): halving dt divides it by 4."""
    lat = lat_small(Ltau=16, dtau=0.1, alpha=0.0)
    w0 = 0.9
    mt = H.mass_tilde(lat.Ltau, lat.dtau, w0, 0.0)
    x0 = rand((lat.Ltau, lat.N), 5)
    p0 = rand((lat.Ltau, lat.N), 6)
    T = 1.3
    exact = x0 * np.cos(w0 * T) + H.tau_fourier_apply(p0, 1.0 / mt) * np.sin(w0 * T) / w0
    zero = lambda v: np.zeros_like(v)
    errs = []
    for Nt in (26, 52):
        xT, _ = H.leapfrog_split(lat, w0, mt, x0, p0, T / Nt, Nt, 1, zero)
        errs.append(np.abs(xT - exact).max())
    assert errs[0] < 5e-3
    assert 3.6 < errs[0] / errs[1] < 4.4
    # the sub-step count is immaterial when there is no fermion force
    xs, _ = H.leapfrog_split(lat, w0, mt, x0, p0, T / 13, 13, 2, zero)
    x26, _ = H.leapfrog_split(lat, w0, mt, x0, p0, T / 26, 26, 1, zero)
    np.testing.assert_allclose(xs, x26, rtol=1e-12, atol=1e-12)


def _tiny_system(L=4, Ltau=8, seed=11):
    lat = lat_small(L=L, Ltau=Ltau, dtau=0.1, alpha=1.0, mu=0.1)
    x = rand((Ltau, lat.N), seed, 0.5)
    R = rand((2, Ltau, lat.N), seed + 1)
    Phis = H.pseudofermions(lat, x, R)
    return lat, x, Phis


def test_total_force_fd():
    """The force the integrator uses, x_force + fermion_force, against central differences of
    the full action S' = x_action + fermion_action (pins the 1/2 and the sum over fields)."""
    lat, x, Phis = _tiny_system()
    xe = x + rand(x.shape, 99, 0.1)
    w0 = 1.0
    S = lambda v: H.x_action(lat, v, w0) + H.fermion_action(lat, v, Phis)
    comps = [(0, 0), (3, 5), (7, 15)]
    fd = central_fd(S, xe, comps, h=1e-4)
    g = H.x_force(lat, xe, w0) + H.fermion_force(lat, xe, Phis)
    np.testing.assert_allclose([g[c] for c in comps], fd, rtol=1e-7)


def test_initial_fermion_action_is_half_R_squared():
    """With Phi = M(x)^T R, S_F(x) = |R|^2 / 2 summed over fields (Sec. II D)."""
    lat, x, Phis = _tiny_system()
    R = rand((2, lat.Ltau, lat.N), 12)
    assert H.fermion_action(lat, x, Phis) == pytest.approx(0.5 * np.sum(R * R), rel=1e-12)


def test_reversible():
    """Leapfrog with splitting is exactly time reversible: integrate, flip p, integrate."""
    lat, x, Phis = _tiny_system()
    w0 = 1.0
    mt = H.mass_tilde(lat.Ltau, lat.dtau, w0, w0)
    p = rand(x.shape, 21)
    f = lambda v: H.fermion_force(lat, v, Phis)
    x1, p1 = H.leapfrog_split(lat, w0, mt, x, p, 0.05, 6, 3, f)
    assert np.abs(x1 - x).max() > 1e-2
    x2, p2 = H.leapfrog_split(lat, w0, mt, x1, -p1, 0.05, 6, 3, f)
    np.testing.assert_allclose(x2, x, atol=1e-11)
    np.testing.assert_allclose(-p2, p, atol=1e-11)


def test_energy_error_second_order():
    """|Delta H| falls by about 4 when dt is halved at fixed trajectory length."""
    lat, x, Phis = _tiny_system()
    w0 = 1.0
    mt = H.mass_tilde(lat.Ltau, lat.dtau, w0, w0)
    p = H.sample_momentum(rand(x.shape, 31), mt)
    f = lambda v: H.fermion_force(lat, v, Phis)
    H0 = H.hamiltonian(lat, w0, mt, x, p, Phis)["H"]
    dH = []
    for Nt in (10, 20, 40):
        x1, p1 = H.leapfrog_split(lat, w0, mt, x, p, 0.5 / Nt, Nt, 4, f)
        dH.append(abs(H.hamiltonian(lat, w0, mt, x1, p1, Phis)["H"] - H0))
    assert dH[0] < 0.05
    assert 3.0 < dH[0] / dH[1] < 5.0 and 3.0 < dH[1] / dH[2] < 5.0


def test_volume_conserving():
    """The trajectory map (x, p) -> (x', p') has unit Jacobian determinant (symplectic)."""
    lat, x, Phis = _tiny_system(L=4, Ltau=2, seed=41)
    w0 = 1.0
    mt = H.mass_tilde(lat.Ltau, lat.dtau, w0, w0)
    p = rand(x.shape, 42)
    f = lambda v: H.fermion_force(lat, v, Phis)
    n = x.size
    z0 = np.concatenate([x.ravel(), p.ravel()])

    def flow(z):
        a, b = H.leapfrog_split(lat, w0, mt, z[:n].reshape(x.shape), z[n:].reshape(x.shape), 0.1, 3, 2, f)
        return np.concatenate([a.ravel(), b.ravel()])

    h = 1e-6
    J = np.empty((2 * n, 2 * n))
    for k in range(2 * n):
        e = np.zeros(2 * n)
        e[k] = h
        J[:, k] = (flow(z0 + e) - flow(z0 - e)) / (2 * h)
    sign, logdet = np.linalg.slogdet(J)
    assert sign == 1 and abs(logdet) < 1e-6


def test_hmc_update_decision():
    """Algorithm 1 end to end on c1's lattice: H_i has S_F = |R|^2/2 and K = |R_p|^2/2, the
    decision is r < exp(-dH), the kept field follows it, and dH is small at the paper's dt."""
    p = get_config("c1")
    lat = Lm.Lattice.from_params(p)
    hp = hmc_params(p, Nt=20)
    x = phonon_field(p)
    R_fields, R_mom, r = hmc_draws(p, hp.nfields)
    out = H.hmc_update(lat, hp.omega0, hp.m_reg, hp.dt, hp.Nt, hp.nt, x, R_fields, R_mom, r)
    assert out["H_i"]["S_F"] == pytest.approx(0.5 * np.sum(R_fields ** 2), rel=1e-11)
    assert out["H_i"]["K"] == pytest.approx(0.5 * np.sum(R_mom ** 2), rel=1e-12)
    assert abs(out["dH"]) < 0.5
    assert out["accepted"] == (r < np.exp(-out["dH"]))
    ref = out["x_f"] if out["accepted"] else x
    assert np.array_equal(out["x_out"], ref)
