"""CPU pins of the rank-1 action-change identity used by the large-lattice
finite-difference force check (tests/_rank1.py): it must equal the direct
difference of two dense-LU actions, for small and for large changes of one
field component, at slice 0 (antiperiodic wrap) and inside."""

import numpy as np
import pytest

from oracle import force as OF
from oracle import lattice as OL
from oracle import solve as OS
from workloads import gaussian_rhs, get_config, perturbed_field, phonon_field

from ._rank1 import action_change, c_row


def _setup():
    p = get_config("c1")
    lat = OL.Lattice.from_params(p)
    x0 = phonon_field(p)
    x = perturbed_field(p, x0)
    Phi = OS.rhs_from_phi(lat, x0, gaussian_rhs(p, 1))[0]
    C = OL.checkerboard_C(lat)
    return lat, x, Phi, C


@pytest.mark.parametrize("k", [(0, 0), (0, 13), (7, 5), (39, 15)])
@pytest.mark.parametrize("h", [1e-3, 0.7])
def test_rank1_identity_equals_direct_difference(k, h):
    import scipy.sparse as sp
    lat, x, Phi, C = _setup()
    u = OS.solve_dense(lat, x, Phi[None], C)[0]
    xn = x.copy()
    xn[k] += h
    un = OS.solve_dense(lat, xn, Phi[None], C)[0]
    direct = float(np.sum(Phi * un) - np.sum(Phi * u))
    E = OL.E_field(lat, x)
    ident = action_change(lat, E, c_row(sp.csr_matrix(C), k[1]), k, xn[k], u, un)
    assert ident == pytest.approx(direct, rel=1e-9, abs=1e-12 * abs(np.sum(Phi * u)))


def test_rank1_central_difference_matches_adjoint_force():
    import scipy.sparse as sp
    lat, x, Phi, C = _setup()
    u = OS.solve_dense(lat, x, Phi[None], C)[0]
    g = OF.force_from_solution(lat, x, u[None], C)[0]
    E = OL.E_field(lat, x)
    Cs = sp.csr_matrix(C)
    h = 1e-4
    for k in [(0, 3), (11, 7), (39, 0)]:
        ds = []
        for sgn in (1.0, -1.0):
            xn = x.copy()
            xn[k] += sgn * h
            un = OS.solve_dense(lat, xn, Phi[None], C)[0]
            ds.append(action_change(lat, E, c_row(Cs, k[1]), k, xn[k], u, un))
        fd = (ds[0] - ds[1]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-7)
