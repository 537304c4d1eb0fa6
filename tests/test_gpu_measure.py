"""GPU parity of the stochastic Green's-function measurements (Sec. VI) against the CPU oracle.

Through the C ABI.  Tolerances: the 3-D transforms agree with numpy's FFT to
1e-12 of the largest coefficient (sums of up to a few hundred FP64 terms);
estimators computed from the same vectors agree with the oracle's to 1e-12
of the largest entry; G xi from the GPU solves agree with the oracle's LU
solves to the solve tolerance; end to end, the estimators from GPU vectors
agree with the oracle's from its own vectors to 1e-8.
"""

import numpy as np
import pytest

from oracle import lattice as OL
from oracle import measure as OM
from workloads import get_config, phonon_field, rademacher_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def relmax(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def make(lat, max_rhs=2):
    from paper_2203_01291_amd.measure import GreenMeasurement
    from paper_2203_01291_amd.solver import FermionSolver
    s = FermionSolver(lat.L, lat.Ltau, lat.dtau, lat.t, lat.mu, lat.alpha, max_rhs=max_rhs)
    return s, GreenMeasurement(s)


SHAPES = [(4, 40, 0.1, 1.0, 0.0, 1.0), (6, 42, 0.1, 1.0, 0.2, 1.3), (10, 2, 0.1, 1.0, 0.0, 1.0),
          (8, 100, 0.1, 1.0, 0.0, 1.0), (32, 400, 0.05, 1.0, -0.2, 1.2), (64, 100, 0.05, 1.0, 0.0, 1.5)]
IDS = [f"L{s[0]}_T{s[1]}" for s in SHAPES]


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_fft_matches_numpy(shape):
    lat = OL.Lattice(*shape)
    rng = np.random.default_rng(lat.L * 1000 + lat.Ltau)
    z = rng.standard_normal((lat.Ltau, lat.N)) + 1j * rng.standard_normal((lat.Ltau, lat.N))
    s, m = make(lat)
    zg = tgpu(z)
    g = z.reshape(lat.Ltau, lat.L, lat.L)
    ref = np.fft.fftn(g).reshape(lat.Ltau, lat.N)
    assert relmax(m.fft(zg).cpu().numpy(), ref) < 1e-12
    refi = (np.fft.ifftn(g) * g.size).reshape(lat.Ltau, lat.N)
    assert relmax(m.fft(zg, inverse=True).cpu().numpy(), refi) < 1e-12
    # twisted: the odd frequencies of the antiperiodic extension to 2 Ltau slices, halved
    ext = np.concatenate([g, -g], axis=0)
    reft = (np.fft.fftn(ext)[1::2] / 2).reshape(lat.Ltau, lat.N)
    Zt = m.fft(zg, twist=True)
    assert relmax(Zt.cpu().numpy(), reft) < 1e-12
    back = m.fft(Zt, inverse=True, twist=True).cpu().numpy() / g.size
    assert relmax(back, z) < 1e-12


EST = [("c1", (4, 40, 0.1, 1.0, 0.0, 1.0), 4), ("L6_T42", (6, 42, 0.1, 1.0, 0.2, 1.3), 3),
       ("L10_T2", (10, 2, 0.1, 1.0, 0.0, 1.0), 3), ("c3", (32, 400, 0.05, 1.0, -0.2, 1.2), 3)]


@pytest.mark.parametrize("case", EST, ids=[c[0] for c in EST])
def test_estimators_match_oracle(case):
    """Same vectors in, the GPU estimators against the oracle's FFT estimators."""
    name, shape, n = case
    lat = OL.Lattice(*shape)
    rng = np.random.default_rng(sum(map(ord, name)))
    xis = 2.0 * rng.integers(0, 2, size=(n, lat.Ltau, lat.N)) - 1.0
    gxs = rng.standard_normal((n, lat.Ltau, lat.N))
    s, m = make(lat)
    xg, gg = tgpu(xis), tgpu(gxs)
    ga = m.green_average(xg, gg).cpu().numpy()
    assert relmax(ga, OM.green_average_estimate(lat, xis, gxs)) < 1e-12
    pp = m.pair_products(xg, gg).cpu().numpy()
    ref = OM.pair_products_estimate(lat, xis, gxs)
    for k in range(3):
        assert relmax(pp[k], ref[k]) < 1e-12, k


@pytest.mark.parametrize("key", ["c1", "c2"])
def test_green_vectors_and_estimators_end_to_end(key):
    """Rademacher xi, G xi from GPU solves (FP64 to 1e-12) against the oracle's LU solves, and the
    estimators from them against the oracle's from its own vectors."""
    p = get_config(key)
    lat = OL.Lattice.from_params(p)
    C = OL.sparse_C(lat).toarray() if lat.N > 16 else None
    x = phonon_field(p)
    xis = rademacher_rhs(p, 4)
    ref_g = OM.green_vectors(lat, x, xis, C)
    s, m = make(lat, max_rhs=3)          # chunks of 3 and 1
    s.set_field(tgpu(x))
    xg = tgpu(xis)
    gg, st = m.green_vectors(xg, tol=1e-12, prec="f64", maxiter=20000)
    assert all(v["status"] == 1 for v in st)
    assert relmax(gg.cpu().numpy(), ref_g) < 1e-8
    assert relmax(m.green_average(xg, gg).cpu().numpy(), OM.green_average_estimate(lat, xis, ref_g)) < 1e-8
    pp = m.pair_products(xg, gg).cpu().numpy()
    ref = OM.pair_products_estimate(lat, xis, ref_g)
    for k in range(3):
        assert relmax(pp[k], ref[k]) < 1e-8, k


def test_complete_set_reproduces_exact_green_function():
    """c1 lattice: with xi_n = sqrt(Ncal) e_n for all n the GPU average equals the exact average of
    G^ext from a dense inverse (a check independent of random vectors)."""
    lat = OL.Lattice(4, 8, 0.1, 1.0, 0.1, 1.0)
    x = np.random.default_rng(9).standard_normal((lat.Ltau, lat.N))
    G = OM.green_dense(lat, x)
    n = lat.dim
    xis = np.sqrt(n) * np.eye(n).reshape(n, lat.Ltau, lat.N)
    gxs = np.sqrt(n) * G.T.reshape(n, lat.Ltau, lat.N)
    s, m = make(lat)
    ga = m.green_average(tgpu(xis), tgpu(gxs)).cpu().numpy()
    assert relmax(ga, OM.gext_average_exact(lat, G)) < 1e-12
