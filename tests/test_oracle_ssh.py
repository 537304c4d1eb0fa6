"""Pins of the oracle's SSH-type coupling (x in the hopping; oracle.ssh).

Checked against things other than the oracle itself: the Holstein matrix
built from plaquette exponentials (g = 0), the closed form of a two-site
exponential, hand values of the bond hoppings at one displaced site, the
checkerboard's O(dtau^2) distance from exp(-dtau K(x)), the determinant
identity of the block-cyclic matrix, and complex-step and central-difference
derivatives of the action.  No GPU.
"""

import numpy as np
import pytest
import scipy.linalg

from oracle import force as Fh
from oracle import lattice as Lm
from oracle import ssh as S


def lat4(L=4, Ltau=4, dtau=0.1, t=1.0, mu=-0.2, alpha=0.7):
    return Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)


def field(lat, seed, scale=0.5):
    return scale * np.random.default_rng(seed).standard_normal((lat.Ltau, lat.N))


def test_g0_is_holstein_matrix():
    """g = 0: the four bond families recombine into the plaquette factors of the Holstein C."""
    for L in (4, 6):
        lat = lat4(L=L)
        x = field(lat, 1)
        assert np.abs(S.dense_M(lat, 0.0, x) - Lm.dense_M(lat, x)).max() < 1e-13


def test_uniform_shift_leaves_hopping_unchanged():
    """The hopping depends on differences of x only: C(x + c) = C(x); a constant x gives the Holstein C."""
    lat = lat4()
    x = field(lat, 2)[0]
    assert np.abs(S.C_slice(lat, 0.3, x + 1.7) - S.C_slice(lat, 0.3, x)).max() < 1e-13
    assert np.abs(S.C_slice(lat, 0.3, np.full(lat.N, 0.9)) - Lm.checkerboard_C(lat)).max() < 1e-13


def test_bond_factor_closed_form_and_hand_values():
    """A two-site block of exp(-dtau K_f) is [[cosh, sinh], [sinh, cosh]](dtau t_b); one site
    displaced by delta raises the hopping of its outgoing bonds to t + g delta and lowers its
    incoming ones to t - g delta."""
    lat = lat4(L=6)
    g, delta, s = 0.4, 0.25, Lm.site(2, 3, 6)
    x = np.zeros(lat.N)
    x[s] = delta
    F = dict(zip(S.FAMILIES, S.factors(lat, g, x)))
    want = {  # (family, i, j): t_b
        ("x_even", s, Lm.site(3, 3, 6)): 1.0 + g * delta,
        ("y_odd", s, Lm.site(2, 4, 6)): 1.0 + g * delta,
        ("x_odd", Lm.site(1, 3, 6), s): 1.0 - g * delta,
        ("y_even", Lm.site(2, 2, 6), s): 1.0 - g * delta,
        ("x_even", Lm.site(4, 0, 6), Lm.site(5, 0, 6)): 1.0,
    }
    for (f, i, j), tb in want.items():
        a = lat.dtau * tb
        assert F[f][i, j] == pytest.approx(np.sinh(a), rel=1e-13)
        assert F[f][j, i] == pytest.approx(np.sinh(a), rel=1e-13)
        assert F[f][i, i] == pytest.approx(np.cosh(a), rel=1e-13)
        assert F[f][j, j] == pytest.approx(np.cosh(a), rel=1e-13)
        assert np.count_nonzero(np.abs(F[f][i]) > 1e-15) == 2


def test_checkerboard_error_is_second_order():
    """|C(x) - exp(-dtau K(x))| falls 4x when dtau halves (Sec. II D: O(dtau^2) per slice)."""
    errs = []
    for dtau in (0.1, 0.05, 0.025):
        lat = lat4(L=6, dtau=dtau)
        x = field(lat, 3)[0]
        ex = scipy.linalg.expm(-dtau * S.full_hopping(lat, 0.5, x))
        errs.append(np.abs(S.C_slice(lat, 0.5, x) - ex).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs
    assert errs[0] > 1e-4  # the split is not exact once the hoppings differ


def test_determinant_identity():
    """det M = det(I + B_{Ltau-1} ... B_0) for the block-cyclic M of Eq. M_def."""
    lat = lat4(Ltau=5)
    x = field(lat, 4)
    g = 0.35
    P = np.eye(lat.N)
    for tau in range(lat.Ltau):
        P = S.B_slice(lat, g, x, tau) @ P
    s1, l1 = np.linalg.slogdet(S.dense_M(lat, g, x))
    s2, l2 = np.linalg.slogdet(np.eye(lat.N) + P)
    assert s1 == s2 and l1 == pytest.approx(l2, abs=1e-11)


@pytest.mark.parametrize("alpha", [0.0, 0.7])
def test_force_matches_complex_step(alpha):
    """The product-rule adjoint force equals the complex-step derivative of S_F."""
    lat = lat4(alpha=alpha)
    x = field(lat, 5)
    phi = np.random.default_rng(6).standard_normal((2, lat.Ltau, lat.N))
    g = 0.45
    f = S.force(lat, g, x, phi)
    fc = S.force_complex_step(lat, g, x, phi)
    assert np.abs(f - fc).max() < 1e-9 * np.abs(fc).max()


def test_force_central_difference_and_g0():
    """A few components against central differences; g = 0 against the Holstein force."""
    lat = lat4()
    x = field(lat, 7)
    phi = np.random.default_rng(8).standard_normal((lat.Ltau, lat.N))
    g = 0.3
    f = S.force(lat, g, x, phi)
    for tau, i in ((0, 0), (2, 5), (3, 15)):
        h = 1e-5
        xp, xm = x.copy(), x.copy()
        xp[tau, i] += h
        xm[tau, i] -= h
        fd = (S.action(lat, g, xp, phi) - S.action(lat, g, xm, phi)) / (2 * h)
        assert f[tau, i] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    u = S.solve(lat, 0.0, x, phi)
    assert np.abs(S.force(lat, 0.0, x, phi) - Fh.force_from_solution(lat, x, u)).max() < 1e-10


def test_sparse_matrix_and_directional_derivative():
    """The sparse construction (sparse exponentials) equals the dense one; the complex-step
    directional derivative of the sparse action equals the adjoint force projected on it."""
    lat = lat4(L=6, Ltau=4)
    x = field(lat, 9)
    g = 0.4
    assert np.abs(S.sparse_M(lat, g, x).toarray() - S.dense_M(lat, g, x)).max() < 1e-13
    lat = lat4()
    x = field(lat, 10)
    phi = np.random.default_rng(11).standard_normal((2, lat.Ltau, lat.N))
    v = np.random.default_rng(12).standard_normal(x.shape)
    f = S.force(lat, g, x, phi)
    dd = S.directional_derivative(lat, g, x, phi, v)
    assert dd == pytest.approx(float(np.sum(f * v)), rel=1e-10)
    assert np.abs(S.sparse_solve(lat, g, x, phi) - S.solve(lat, g, x, phi)).max() < 1e-10


def test_hmc_reversible_and_second_order():
    """The leapfrog with the SSH force runs back to its start under p -> -p, and its energy
    error falls 4x when dt halves (it only does so if the force is the action's gradient)."""
    from oracle import hmc as H
    lat = lat4(Ltau=4, dtau=0.1, alpha=0.5)
    g, om = 0.4, 1.0
    x = field(lat, 13, scale=0.3)
    rng = np.random.default_rng(14)
    R = rng.standard_normal((1, lat.Ltau, lat.N))
    Rm = rng.standard_normal((lat.Ltau, lat.N))
    out = S.hmc_update(lat, g, om, 1.0, 0.1, 4, 2, x, R, Rm, 0.5)
    mt = H.mass_tilde(lat.Ltau, lat.dtau, om, 1.0)
    fF = lambda v: 0.5 * S.force(lat, g, v, out["Phi"])
    xb, pb = H.leapfrog_split(lat, om, mt, out["x_f"], -out["p_f"], 0.1, 4, 2, fF)
    assert np.abs(xb - x).max() < 1e-10 and np.abs(pb + out["p_i"]).max() < 1e-10
    dh = [abs(S.hmc_update(lat, g, om, 1.0, 0.4 / n, n, 2, x, R, Rm, 0.5)["dH"]) for n in (4, 8)]
    assert 3.3 < dh[0] / dh[1] < 4.7, dh


def test_planted_mistakes_fail_the_pins(monkeypatch):
    """Plausible mistakes planted in the oracle each fail one of the pins above: the sign of the
    coupling in t_b, a dropped on-site term of the force, and the direction of dt_b/dx."""
    import oracle.ssh as mod

    # 1. t_b = t + g (x_j - x_i): the hand values around a displaced site catch it
    good = mod.hoppings
    flipped = lambda lat, g, x_tau: good(lat, -g, x_tau)
    monkeypatch.setattr(mod, "hoppings", flipped)
    with pytest.raises(AssertionError):
        test_bond_factor_closed_form_and_hand_values()
    monkeypatch.setattr(mod, "hoppings", good)

    lat = lat4(alpha=0.7)
    x = field(lat, 5)
    phi = np.random.default_rng(6).standard_normal((1, lat.Ltau, lat.N))
    fc = S.force_complex_step(lat, 0.45, x, phi)

    # 2. the on-site term of dB/dx dropped: complex step catches it
    good_E = mod.lat_mod.E_field
    monkeypatch.setattr(mod, "dM_dx", _dM_dx_without_onsite)
    f = mod.force(lat, 0.45, x, phi)
    assert np.abs(f - fc).max() > 1e-3 * np.abs(fc).max()
    monkeypatch.undo()

    # 3. dt_b/dx with the bond's ends swapped: complex step catches it
    monkeypatch.setattr(mod, "dM_dx", _dM_dx_swapped_ends)
    f = mod.force(lat, 0.45, x, phi)
    assert np.abs(f - fc).max() > 1e-3 * np.abs(fc).max()
    monkeypatch.undo()
    assert mod.lat_mod.E_field is good_E


def _dM_dx_variant(lat, g, x, tau, i, onsite=True, swap=False):
    # a copy of oracle.ssh.dM_dx with one term changed (planted mistakes)
    N, T = lat.N, lat.Ltau
    E = Lm.E_field(lat, x)[tau]
    hp = S.hoppings(lat, g, x[tau])
    Ks = [S.family_hopping(lat, hp[f]) for f in S.FAMILIES]
    Fs = [scipy.linalg.expm(-lat.dtau * K) for K in Ks]
    C = Fs[0] @ Fs[1] @ Fs[2] @ Fs[3]
    dC = np.zeros((N, N))
    fam = Lm.bond_families(lat.L)
    for k, f in enumerate(S.FAMILIES):
        dK = np.zeros((N, N))
        for a, b in fam[f]:
            dt = g * ((i == b) - (i == a)) if swap else g * ((i == a) - (i == b))
            dK[a, b] -= dt
            dK[b, a] -= dt
        if not dK.any():
            continue
        dF = scipy.linalg.expm_frechet(-lat.dtau * Ks[k], -lat.dtau * dK, compute_expm=False)
        left, right = np.eye(N), np.eye(N)
        for m in range(k):
            left = left @ Fs[m]
        for m in range(k + 1, 4):
            right = right @ Fs[m]
        dC += left @ dF @ right
    dE = np.zeros(N)
    if onsite:
        dE[i] = -lat.dtau * lat.alpha * E[i]
    dB = dE[:, None] * C + E[:, None] * dC
    dM = np.zeros((N * T, N * T))
    if tau >= 1:
        dM[tau * N:(tau + 1) * N, (tau - 1) * N:tau * N] = -dB
    else:
        dM[0:N, (T - 1) * N:T * N] = dB
    return dM


def _dM_dx_without_onsite(lat, g, x, tau, i):
    return _dM_dx_variant(lat, g, x, tau, i, onsite=False)


def _dM_dx_swapped_ends(lat, g, x, tau, i):
    return _dM_dx_variant(lat, g, x, tau, i, swap=True)
