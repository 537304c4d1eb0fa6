"""The solve as a stream-ordered sequence of kernels (pcg_solve).

pcg_solve enqueues a fixed sequence of launches and reads nothing back:
convergence, FP64 residual evaluations and stopping are decided on the
device, and the statistics land in device memory.  These tests check that
(a) it gives bit for bit the result of the blocking driver (which runs the
same kernels and only stops enqueueing early), (b) an exhausted iteration
budget is reported, and (c) one whole step -- set-field, preconditioned
FP32-refined solve, S_F, force -- captured in a graph and replayed on new
inputs matches the oracle on every replay (Sec. II D, Eq. CG; Sec. V A;
Eq. dSF_dx).
"""

import numpy as np
import pytest

from oracle import force as OF
from oracle import lattice as OL
from oracle import solve as OS
from workloads import gaussian_rhs, get_config, perturbed_field, phonon_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def c2_problem(k=0):
    p = get_config("c2")
    lat = OL.Lattice.from_params(p)
    x0 = phonon_field(p)
    Cs = OL.sparse_C(lat).tocsr()
    phi = gaussian_rhs(p, 2)
    Phi = OL.apply_MT(lat, x0, phi, Cs)
    x = perturbed_field(p, x0) + 0.05 * k
    return p, lat, Cs, x, Phi


def make_solver(lat, max_rhs):
    from paper_2203_01291_amd.solver import FermionSolver
    return FermionSolver(lat.L, lat.Ltau, lat.dtau, lat.t, lat.mu, lat.alpha, max_rhs=max_rhs)


@pytest.mark.parametrize("prec", ["f64", "f32_refined"])
@pytest.mark.parametrize("precond", [False, True])
def test_enqueue_only_equals_blocking(prec, precond):
    from paper_2203_01291_amd._lib import stats_from_device
    p, lat, Cs, x, Phi = c2_problem()
    s = make_solver(lat, 2)
    s.set_field(tgpu(x), a1=0.15, a2=12.0)
    b = tgpu(Phi)
    u1, st1 = s.solve(b, tol=1e-11, maxiter=20000, precond=precond, prec=prec)
    budget = max(v["iters"] for v in st1) + 40
    u2, sd = s.solve_async(b, tol=1e-11, maxiter=budget, precond=precond, prec=prec)
    st2 = stats_from_device(sd)
    assert torch.equal(u1, u2)
    assert st1 == st2
    u_ref = OS.solve_sparse(lat, x, Phi, Cs)
    for r in range(2):
        assert st2[r]["status"] == 1, st2[r]
        assert relmax(u2[r].cpu().numpy(), u_ref[r]) < 1e-8


def test_enqueue_only_budget_and_zero_rhs():
    from paper_2203_01291_amd._lib import stats_from_device
    p, lat, Cs, x, Phi = c2_problem()
    s = make_solver(lat, 2)
    s.set_field(tgpu(x))
    B = np.stack([np.zeros_like(Phi[0]), Phi[1]])
    u, sd = s.solve_async(tgpu(B), u=tgpu(np.ones_like(B)), zero_guess=False, tol=1e-12,
                          maxiter=7, prec="f32_refined")
    st = stats_from_device(sd)
    assert st[0]["status"] == 1 and torch.count_nonzero(u[0]) == 0   # b = 0: u = 0 exactly
    assert st[1]["status"] & 2 and st[1]["iters"] == 7               # budget exhausted


def test_graph_captured_step_matches_oracle():
    """set_field + FP32-refined preconditioned pcg_solve + S_F + force captured
    once in a hipGraph (through torch.cuda.graph) and replayed on three new
    fields; every replay against the oracle, with eager work in between."""
    from paper_2203_01291_amd._lib import stats_from_device
    p, lat, Cs, x, Phi = c2_problem()
    s = make_solver(lat, 2)
    a1, a2 = 0.15, 12.0
    x_in = tgpu(x)
    Phi_in = tgpu(Phi)
    u = torch.zeros_like(Phi_in)
    stats = torch.zeros(2 * 4, dtype=torch.float64, device=DEV)
    S = torch.zeros(2, dtype=torch.float64, device=DEV)
    grad = torch.zeros(lat.Ltau, lat.N, dtype=torch.float64, device=DEV)
    kw = dict(tol=1e-11, maxiter=400, precond=True, prec="f32_refined", zero_guess=True)

    def step():
        s.set_field(x_in, a1=a1, a2=a2)
        s.solve_async(Phi_in, u=u, stats=stats, **kw)
        s.action(Phi_in, u, out=S)
        grad.zero_()
        s.force(u, grad=grad)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                      # eager warm-up: launch configurations cached
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    other = make_solver(lat, 1)
    for k in (1, 2, 3):
        _, _, _, xk, _ = c2_problem(k)
        x_in.copy_(tgpu(xk))
        g.replay()
        torch.cuda.synchronize()
        st = stats_from_device(stats)
        u_ref = OS.solve_sparse(lat, xk, Phi, Cs)
        g_ref = OF.force_from_solution(lat, xk, u_ref, Cs).sum(axis=0)
        for r in range(2):
            assert st[r]["status"] == 1, (k, st[r])
            assert relmax(u[r].cpu().numpy(), u_ref[r]) < 1e-8, k
            assert float(S[r]) == pytest.approx(float(np.sum(Phi[r] * u_ref[r])), rel=1e-10)
            assert st[r]["action"] == pytest.approx(float(S[r]), rel=1e-14)
        assert relmax(grad.cpu().numpy(), g_ref) < 1e-8, k
        # eager work on the same device between replays
        other.set_field(tgpu(xk))
        other.solve(tgpu(Phi[:1]), tol=1e-8)
        torch.cuda.synchronize()
