"""The SSH solve in FP32-refined mode (FP32 iterations on a correction with
FP64 residual replacement) against the oracle's direct solves: small lattices
(dense LU), L = 8 with Ltau = 40 and L = 40 / 64 (sparse LU of M and M^T), the
unfused operator path (L = 64), right-hand sides of very different scales and
a zero one, the preconditioned solve, the iteration and evaluation caps, and
the argument checks."""

import numpy as np
import pytest

from oracle import lattice as Lm
from oracle import ssh as S
from workloads import gaussian_rhs, get_config, phonon_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def relmax(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def make(L, Ltau, g, alpha=0.9, max_rhs=3, seed=0, dtau=0.1, mu=-0.2):
    from paper_2203_01291_amd.ssh import SSHSolver
    lat = Lm.Lattice(L=L, Ltau=Ltau, dtau=dtau, t=1.0, mu=mu, alpha=alpha)
    x = 0.6 * np.random.default_rng(seed).standard_normal((Ltau, L * L))
    s = SSHSolver(L, Ltau, dtau, 1.0, mu, alpha, g, max_rhs=max_rhs)
    s.set_field(tgpu(x))
    return lat, x, s


@pytest.mark.parametrize("L,T,g", [(4, 6, 0.45), (6, 4, 0.3), (8, 40, 0.3), (40, 4, 0.35), (64, 2, 0.35)])
def test_refined_solve_against_direct(L, T, g):
    lat, x, s = make(L, T, g, max_rhs=3, dtau=0.1 if L < 40 else 0.05)
    phi = np.random.default_rng(11).standard_normal((3, T, L * L)) * np.array([1.0, 1e-3, 1e3])[:, None, None]
    u, st = s.solve(tgpu(phi), tol=1e-12, prec="f32_refined")
    uo = S.solve(lat, g, x, phi) if lat.dim <= 2000 else S.sparse_solve(lat, g, x, phi)
    for r in range(3):
        assert st[r]["status"] == 1, st[r]
        assert st[r]["rel_resid"] < 1e-12 and st[r]["outer_iters"] >= 1
        assert relmax(u[r].cpu().numpy(), uo[r]) < 1e-8, r
        assert st[r]["action"] == pytest.approx(float(np.sum(phi[r] * uo[r])), rel=1e-10)
    # the same solve in FP64: same solution to the tolerance
    u64, st64 = s.solve(tgpu(phi), tol=1e-12)
    assert relmax(u.cpu().numpy(), u64.cpu().numpy()) < 1e-8
    print(f"L={L} T={T}: FP32-refined iterations {[v['iters'] for v in st]} "
          f"(evaluations {[v['outer_iters'] for v in st]}), FP64 {[v['iters'] for v in st64]}")


def test_refined_zero_rhs_warm_start_and_caps():
    lat, x, s = make(8, 40, 0.3, max_rhs=2)
    phi = np.random.default_rng(12).standard_normal((2, 40, 64))
    phi[0] = 0.0
    u, st = s.solve(tgpu(phi), tol=1e-12, prec="f32_refined")
    assert st[0]["status"] == 1 and st[0]["iters"] == 0 and torch.count_nonzero(u[0]) == 0
    assert st[1]["status"] == 1
    # warm start at the solution: converged at the first FP64 evaluation
    u2, st2 = s.solve(tgpu(phi[1:]), u=u[1:].clone(), tol=1e-10, prec="f32_refined")
    assert st2[0]["status"] == 1 and st2[0]["iters"] == 0
    # iteration cap and evaluation cap
    _, st3 = s.solve(tgpu(phi[1:]), tol=1e-14, maxiter=5, chunk=5, prec="f32_refined")
    assert st3[0]["status"] == 2 and st3[0]["iters"] == 5
    _, st4 = s.solve(tgpu(phi[1:]), tol=1e-14, max_outer=1, prec="f32_refined", ru_delta=0.5, chunk=1)
    assert st4[0]["status"] == 2 and st4[0]["outer_iters"] == 1
    from paper_2203_01291_amd._lib import FphError
    with pytest.raises(FphError):
        s.solve(tgpu(phi), prec="f32_refined", max_outer=-1)


@pytest.mark.parametrize("key,g", [("c1", 0.3), ("c2", 0.2)])
def test_refined_preconditioned(key, g):
    """FP32-refined PCG with the Holstein adiabatic preconditioner (FP32 applies): the oracle's
    solution (c1: dense LU) or the FP64 preconditioned solve (c2), in fewer iterations than
    without the preconditioner."""
    from paper_2203_01291_amd.solver import FermionSolver
    from paper_2203_01291_amd.ssh import SSHSolver
    p = get_config(key)
    x = phonon_field(p)
    s = SSHSolver.from_params(p, g, max_rhs=2)
    fs = FermionSolver.from_params(p, max_rhs=2)
    s.attach_preconditioner(fs, a1=0.15, a2=12.0)
    s.set_field(tgpu(x))
    phi = gaussian_rhs(p, 2)
    u1, st1 = s.solve(tgpu(phi), tol=1e-11, precond=True, prec="f32_refined")
    u0, st0 = s.solve(tgpu(phi), tol=1e-11, precond=False, prec="f32_refined")
    u64, st64 = s.solve(tgpu(phi), tol=1e-11, precond=True)
    assert all(v["status"] == 1 for v in st1 + st0 + st64), (st1, st0, st64)
    assert all(a["iters"] < b["iters"] for a, b in zip(st1, st0)), (st1, st0)
    if key == "c1":
        lat = Lm.Lattice.from_params(p)
        assert relmax(u1.cpu().numpy(), S.solve(lat, g, x, phi)) < 1e-8
    else:
        assert relmax(u1.cpu().numpy(), u64.cpu().numpy()) < 1e-7
    print(f"{key}: FP32-refined PCG {[v['iters'] for v in st1]} ({[v['outer_iters'] for v in st1]} evaluations), "
          f"FP64 PCG {[v['iters'] for v in st64]}, FP32-refined CG {[v['iters'] for v in st0]}")
