"""Pins of the CPU oracle's stochastic Green's-function measurements (Sec. VI).

Each test checks the oracle against something other than itself: FFT
cross-correlations against direct sums, the estimator with a complete set of
vectors against the exact average from a dense inverse, the free-electron
Green's function in closed form, and the statistical convergence of
random-vector estimates to the exact values.  No GPU.
"""

import numpy as np
import pytest

from oracle import lattice as Lm
from oracle import measure as MS


def lat_small(L=4, Ltau=4, dtau=0.1, t=1.0, mu=0.0, alpha=1.0):
    return Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)


def rademacher(n, lat, seed):
    return 2.0 * np.random.default_rng(seed).integers(0, 2, size=(n, lat.Ltau, lat.N)) - 1.0


def test_two_point_fft_equals_direct_sum():
    lat = lat_small(Ltau=6)
    rng = np.random.default_rng(1)
    xis = rng.standard_normal((2, lat.Ltau, lat.N))
    gxs = rng.standard_normal((2, lat.Ltau, lat.N))
    np.testing.assert_allclose(MS.green_average_estimate(lat, xis, gxs),
                               MS.green_average_direct(lat, xis, gxs), atol=1e-13)


def test_pair_products_fft_equal_direct_sums():
    lat = lat_small(Ltau=4)
    rng = np.random.default_rng(2)
    xis = rng.standard_normal((3, lat.Ltau, lat.N))
    gxs = rng.standard_normal((3, lat.Ltau, lat.N))
    np.testing.assert_allclose(MS.pair_products_estimate(lat, xis, gxs),
                               MS.pair_products_direct(lat, xis, gxs), atol=1e-13)


def test_complete_set_reproduces_exact_average():
    """With xi_n = sqrt(Ncal) e_n over all n, (1/N_rv) sum_n (G xi_n) xi_n^T = G exactly, so the
    FFT estimator returns the exact space-time average of G^ext."""
    lat = lat_small(Ltau=4, mu=0.2)
    x = np.random.default_rng(3).standard_normal((lat.Ltau, lat.N))
    G = MS.green_dense(lat, x)
    n = lat.dim
    xis = np.sqrt(n) * np.eye(n).reshape(n, lat.Ltau, lat.N)
    gxs = np.sqrt(n) * G.T.reshape(n, lat.Ltau, lat.N)      # row k of G^T is G e_k
    np.testing.assert_allclose(MS.green_average_estimate(lat, xis, gxs), MS.gext_average_exact(lat, G),
                               atol=1e-13)


def test_free_electron_closed_form():
    """Constant field, L = 4 (where the checkerboard product equals exp(-dtau K)): per momentum k
    the blocks are b_k = exp(-dtau (alpha x - mu)) exp(2 dtau t (cos kx + cos ky)) and
    G_{l,l'} = b^{l-l'}/(1 + b^Ltau) (l >= l'), -b^{Ltau+l-l'}/(1 + b^Ltau) (l < l'), so the
    average of G^ext at (dtau, dr) is (1/N) sum_k e^{i k.dr} b_k^dtau / (1 + b_k^Ltau)."""
    lat = lat_small(L=4, Ltau=8, dtau=0.1, t=1.0, mu=0.3, alpha=0.7)
    xc = 0.4
    G = MS.green_dense(lat, np.full((lat.Ltau, lat.N), xc))
    GA = MS.gext_average_exact(lat, G)
    L = lat.L
    ks = 2 * np.pi * np.arange(L) / L
    ref = np.zeros_like(GA)
    for kx in ks:
        for ky in ks:
            b = np.exp(-lat.dtau * (lat.alpha * xc - lat.mu)) * np.exp(2 * lat.dtau * lat.t * (np.cos(kx) + np.cos(ky)))
            for dt in range(lat.Ltau):
                for dy in range(L):
                    for dx in range(L):
                        ref[dt, dy, dx] += np.real(np.exp(1j * (kx * dx + ky * dy))) * b ** dt / (1 + b ** lat.Ltau)
    np.testing.assert_allclose(GA, ref / lat.N, atol=1e-13)


def test_random_vector_estimate_converges():
    """Rademacher estimates of the average of G^ext approach the exact one like N_rv^{-1/2}."""
    lat = lat_small(Ltau=4, mu=-0.1)
    x = 0.5 * np.random.default_rng(4).standard_normal((lat.Ltau, lat.N))
    G = MS.green_dense(lat, x)
    exact = MS.gext_average_exact(lat, G)
    errs = []
    for n, seed in ((64, 5), (1024, 6)):
        xis = rademacher(n, lat, seed)
        gxs = np.einsum("ij,nj->ni", G, xis.reshape(n, -1)).reshape(xis.shape)
        errs.append(np.abs(MS.green_average_estimate(lat, xis, gxs) - exact).max())
    assert errs[1] < 0.5 * errs[0]
    assert errs[1] < 0.02 * np.abs(exact).max()


def test_pair_products_converge_to_exact():
    """The pair-averaged products approach the exact averages of G G (Eq. GG_approx_better);
    for T1 and T3 the error falls faster than N_rv^{-1/2} (the paper expects about N_rv^{-1})."""
    lat = lat_small(Ltau=4, mu=0.1)
    x = 0.5 * np.random.default_rng(7).standard_normal((lat.Ltau, lat.N))
    G = MS.green_dense(lat, x)
    exact = MS.pair_products_exact(lat, G)
    rms = []
    for n in (30, 240):
        xis = rademacher(n, lat, 8)
        gxs = np.einsum("ij,nj->ni", G, xis.reshape(n, -1)).reshape(xis.shape)
        est = MS.pair_products_estimate(lat, xis, gxs)
        rms.append([float(np.sqrt(np.mean((est[k] - exact[k]) ** 2))) for k in range(3)])
    for k in range(3):
        assert np.abs(est[k] - exact[k]).max() < 0.05 * np.abs(exact[k]).max(), k
    assert rms[0][0] / rms[1][0] > 3.0 and rms[0][2] / rms[1][2] > 3.0
