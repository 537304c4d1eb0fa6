"""Independent solves and HMC chains run side by side (pcg_solve_concurrent,
hmc_trajectory_concurrent) give the same results, bit for bit, as the same
calls made one after the other; a repeated handle is refused."""

import numpy as np
import pytest

from workloads import gaussian_rhs, get_config, hmc_draws, hmc_params, phonon_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_concurrent_solves_equal_sequential():
    from paper_2203_01291_amd.solver import FermionSolver, solve_concurrent
    p = get_config("c2")
    items, seq = [], []
    for k in range(3):
        s = FermionSolver.from_params(p, max_rhs=2)
        x = tgpu(phonon_field(p) + 0.05 * k)
        s.set_field(x, a1=0.15, a2=12.0)
        b = s.matvec(tgpu(gaussian_rhs(p, 2) * (1 + k)), "MT")
        u, st = s.solve(b, tol=1e-9, prec="f32_refined", precond=True)
        seq.append((u.cpu().numpy(), st))
        items.append((s, b))
    out = solve_concurrent(items, tol=1e-9, prec="f32_refined", precond=True)
    for (u, st), (u0, st0) in zip(out, seq):
        assert np.array_equal(u.cpu().numpy(), u0)
        assert [v["iters"] for v in st] == [v["iters"] for v in st0]
        assert all(v["status"] == 1 for v in st)
    from paper_2203_01291_amd._lib import FphError
    with pytest.raises(FphError):
        solve_concurrent([items[0], items[0]])


def test_concurrent_chains_equal_sequential():
    from paper_2203_01291_amd.hmc import PhononHMC, trajectories_concurrent
    from paper_2203_01291_amd.solver import FermionSolver
    p = get_config("c1")
    hp = hmc_params(p, Nt=20)
    ctx, args = [], []
    for k in range(3):
        s = FermionSolver.from_params(p, max_rhs=2)
        h = PhononHMC(s, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, force_tol=hp.tol_force,
                      action_tol=hp.tol_action, lambda_action=(k == 1))
        Rf, Rm, r = hmc_draws(p, 2, traj=k)
        ctx.append((s, h))
        args.append((phonon_field(p) + 0.1 * k, Rf, Rm, r))
    seq = []
    for (s, h), (x, Rf, Rm, r) in zip(ctx, args):
        xg = tgpu(x)
        st = h.trajectory(xg, tgpu(Rf), tgpu(Rm), r)
        seq.append((xg.cpu().numpy(), st))
    xs = [tgpu(a[0]) for a in args]
    out = trajectories_concurrent([(h, xg, tgpu(Rf), tgpu(Rm), r)
                                   for (s, h), xg, (x, Rf, Rm, r) in zip(ctx, xs, args)])
    for xg, st, (x0, st0) in zip(xs, out, seq):
        assert np.array_equal(xg.cpu().numpy(), x0)
        assert st == st0
