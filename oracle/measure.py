"""Stochastic Green's-function measurements with FFT acceleration (Sec. VI).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout.

G = M^{-1} estimates the Green's function (Eq. Green_approx).  For random
vectors xi with <xi xi^T> = I, G ~ (G xi) xi^T (Eqs. Hutch_approx, G_approx);
G xi solves M^T M v = M^T xi.  Averages over all space-time displacements
Delta = (dx, dy, dtau) use the extension G^ext = Q G Q^T, Q = [I; -I]
(Eq. G_def-1), whose doubled imaginary time 0 <= tau < 2 Ltau is periodic:

    GA_Delta = (1/Ncal) sum_{i} G^ext_{(i+Delta), i},   Ncal = N Ltau,

with i over the N Ltau distinct space-time points (reading: the paper's sum
runs over the doubled range, which counts each element twice; as an average
of the Ncal distinct elements it carries 1/(2 Ncal) there).  With
a = Q xi, b = Q G xi the stochastic estimate is (1/(2 Ncal)) (a * b)_Delta,
the circular cross-correlation (a * b)_Delta = sum_i a_i b_{i+Delta} on the
doubled grid, computed as F^{-1}{ conj(F[a]) F[b] } (Eq. cross_corr).
GA is antiperiodic in dtau (GA_{dtau + Ltau} = -GA_{dtau}); arrays hold
dtau in [0, Ltau).

Four-point products (Wick's theorem) use two independent vectors and, for
N_rv vectors, the average over all pairs n < m (Eq. GG_approx_better):

    T1_Delta = (1/Ncal) sum_i G_{i+D,i} G_{i+D,i}      ~ (xi_n . xi_m) * (Gxi_n . Gxi_m)
    T2_Delta = (1/Ncal) sum_i G_{i+D,i+D} G_{i,i}      ~ (xi_n . Gxi_n) * (xi_m . Gxi_m)
    T3_Delta = (1/Ncal) sum_i G_{i+D,i} G_{i,i+D}      ~ (xi_n . Gxi_m) * (xi_m . Gxi_n)

('.' elementwise, '*' cross-correlation).  The two signs of G^ext cancel in
each product, so these are periodic in dtau with period Ltau and use the
original grid.

Layout: vectors are [Ltau, N] with site i = x + L*y; results are [Ltau, L, L]
indexed [dtau, dy, dx].

Pinned in ``tests/test_oracle_measure.py``: FFT cross-correlations against
direct sums, the estimator with the complete set xi_n = sqrt(Ncal) e_n
against the exact average of G^ext from a dense inverse, the free-electron
Green's function in closed form, and the convergence of random-vector
estimates of G and of products of G to the exact values.
"""

import numpy as np

from . import lattice as lat_mod


def _grid(v, lat):
    """[..., Ltau, N] -> [..., Ltau, L, L] (axes tau, y, x)."""
    v = np.asarray(v)
    return v.reshape(v.shape[:-2] + (lat.Ltau, lat.L, lat.L))


def green_dense(lat, x, C=None):
    """G = M^{-1} (Eq. Green_approx) by a dense inverse."""
    return np.linalg.inv(lat_mod.dense_M(lat, x, C))


def green_vectors(lat, x, xis, C=None):
    """G xi from (M^T M) v = M^T xi (Sec. VI B) by an LU of M."""
    from . import solve as solve_mod
    b = lat_mod.apply_MT(lat, x, np.asarray(xis), C)
    return solve_mod.solve_sparse(lat, x, b, C)


def gext_average_exact(lat, G):
    """GA_Delta from the full matrix G by its definition (direct sum over i)."""
    L, T, N = lat.L, lat.Ltau, lat.N
    out = np.zeros((T, L, L))
    for dt in range(T):
        for dy in range(L):
            for dx in range(L):
                acc = 0.0
                for tau in range(T):
                    t2 = tau + dt
                    sgn = 1.0 if t2 < T else -1.0
                    t2 %= T
                    for y in range(L):
                        for xx in range(L):
                            i = xx + L * y
                            j = (xx + dx) % L + L * ((y + dy) % L)
                            acc += sgn * G[t2 * N + j, tau * N + i]
                out[dt, dy, dx] = acc / (N * T)
    return out


def cross_correlation(a, b, axes):
    """(a * b)_Delta = sum_i a_i b_{i+Delta} (circular) by FFTs (Eq. cross_corr)."""
    A = np.fft.fftn(a, axes=axes)
    B = np.fft.fftn(b, axes=axes)
    return np.real(np.fft.ifftn(np.conj(A) * B, axes=axes))


def _doubled(v, lat):
    g = _grid(v, lat)
    return np.concatenate([g, -g], axis=-3)


def green_average_estimate(lat, xis, Gxis):
    """(1/N_rv) sum_n (1/(2 Ncal)) (Q xi_n * Q G xi_n)_Delta, dtau in [0, Ltau) (Eq. G_approx_better)."""
    xis = np.asarray(xis)
    Gxis = np.asarray(Gxis)
    acc = np.zeros((lat.Ltau, lat.L, lat.L))
    for xi, gx in zip(xis, Gxis):
        cc = cross_correlation(_doubled(xi, lat), _doubled(gx, lat), axes=(-3, -2, -1))
        acc += cc[:lat.Ltau] / (2.0 * lat.N * lat.Ltau)
    return acc / len(xis)


def green_average_direct(lat, xis, Gxis):
    """The same estimate by direct summation over i (no FFT), for small grids."""
    L, T, N = lat.L, lat.Ltau, lat.N
    out = np.zeros((T, L, L))
    for xi, gx in zip(np.asarray(xis), np.asarray(Gxis)):
        for dt in range(T):
            for dy in range(L):
                for dx in range(L):
                    acc = 0.0
                    for tau in range(T):
                        t2 = tau + dt
                        sgn = 1.0 if t2 < T else -1.0
                        t2 %= T
                        for y in range(L):
                            for xx in range(L):
                                i = xx + L * y
                                j = (xx + dx) % L + L * ((y + dy) % L)
                                acc += xi[tau, i] * sgn * gx[t2, j]
                    out[dt, dy, dx] += acc / (N * T)
    return out / len(xis)


def pair_products_estimate(lat, xis, Gxis):
    """[T1, T2, T3] averaged over all pairs n < m (Eq. GG_approx_better), each (1/Ncal) times the
    cross-correlation of the elementwise products on the original periodic grid."""
    xis = [_grid(v, lat) for v in np.asarray(xis)]
    Gxis = [_grid(v, lat) for v in np.asarray(Gxis)]
    n = len(xis)
    out = np.zeros((3, lat.Ltau, lat.L, lat.L))
    ax = (-3, -2, -1)
    npairs = 0
    for a in range(n):
        for b in range(a + 1, n):
            out[0] += cross_correlation(xis[a] * xis[b], Gxis[a] * Gxis[b], ax)
            out[1] += cross_correlation(xis[a] * Gxis[a], xis[b] * Gxis[b], ax)
            out[2] += cross_correlation(xis[a] * Gxis[b], xis[b] * Gxis[a], ax)
            npairs += 1
    return out / (npairs * lat.N * lat.Ltau)


def pair_products_direct(lat, xis, Gxis):
    """The pair-averaged products by direct summation, for small grids."""
    L, T, N = lat.L, lat.Ltau, lat.N
    xs = np.asarray(xis)
    gs = np.asarray(Gxis)
    n = len(xs)
    out = np.zeros((3, T, L, L))
    npairs = 0
    for a in range(n):
        for b in range(a + 1, n):
            npairs += 1
            for dt in range(T):
                for dy in range(L):
                    for dx in range(L):
                        s = np.zeros(3)
                        for tau in range(T):
                            t2 = (tau + dt) % T
                            for y in range(L):
                                for xx in range(L):
                                    i = xx + L * y
                                    j = (xx + dx) % L + L * ((y + dy) % L)
                                    s[0] += xs[a][tau, i] * xs[b][tau, i] * gs[a][t2, j] * gs[b][t2, j]
                                    s[1] += xs[a][tau, i] * gs[a][tau, i] * xs[b][t2, j] * gs[b][t2, j]
                                    s[2] += xs[a][tau, i] * gs[b][tau, i] * xs[b][t2, j] * gs[a][t2, j]
                        out[:, dt, dy, dx] += s
    return out / (npairs * N * T)


def pair_products_exact(lat, G):
    """T1, T2, T3 from the full matrix G by their definitions."""
    L, T, N = lat.L, lat.Ltau, lat.N
    out = np.zeros((3, T, L, L))
    d = np.diag(G)
    for dt in range(T):
        for dy in range(L):
            for dx in range(L):
                s = np.zeros(3)
                for tau in range(T):
                    t2 = (tau + dt) % T
                    for y in range(L):
                        for xx in range(L):
                            i = tau * N + xx + L * y
                            j = t2 * N + (xx + dx) % L + L * ((y + dy) % L)
                            s[0] += G[j, i] ** 2
                            s[1] += d[j] * d[i]
                            s[2] += G[j, i] * G[i, j]
                out[:, dt, dy, dx] = s / (N * T)
    return out
