"""Per-right-hand-side fields (fph_set_fields): independent systems of one lattice in the same
launches give, right-hand side by right-hand side, the results of the same systems set up one
field at a time (operators, preconditioner and forces to rounding; solves to their tolerance);
argument limits are enforced."""

import numpy as np
import pytest

from workloads import gaussian_rhs, get_config, hmc_draws, hmc_params, phonon_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES = [("c2", 3, 2), ("c1", 2, 1), ("c3", 2, 1)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_{c[1]}f_{c[2]}rpf" for c in CASES])
def test_multifield_equals_single_field(case):
    from paper_2203_01291_amd.solver import FermionSolver
    key, nf, rpf = case
    p = get_config(key)
    nr = nf * rpf
    xs = np.stack([phonon_field(p) + 0.07 * f for f in range(nf)])
    phi = gaussian_rhs(p, nr)
    sm = FermionSolver.from_params(p, max_rhs=max(nr, nf))
    ss = FermionSolver.from_params(p, max_rhs=rpf)
    # right-hand sides b = M(x_f)^T phi from the single-field path
    bs = []
    for f in range(nf):
        ss.set_field(tgpu(xs[f]))
        bs.append(ss.matvec(tgpu(phi[f * rpf:(f + 1) * rpf]), "MT"))
    b = torch.cat(bs).contiguous()
    sm.set_fields(tgpu(xs), rhs_per_field=rpf, a1=0.15, a2=12.0)
    v = tgpu(np.random.default_rng(1).standard_normal((nr, p.Ltau, p.N)))
    mv = {op: sm.matvec(v, op).cpu().numpy() for op in ("M", "MT", "MTM")}
    pcv = sm.precond(v, "FFT").cpu().numpy()
    sols = {}
    for prec, pre in (("f64", True), ("f32_refined", True), ("f64", False)):
        sols[(prec, pre)] = sm.solve(b, tol=1e-10, prec=prec, precond=pre)
    u_ref = sols[("f64", True)][0]
    g = sm.force(u_ref, scale=0.5).cpu().numpy()
    assert g.shape == (nf, p.Ltau, p.N)
    for f in range(nf):
        sl = slice(f * rpf, (f + 1) * rpf)
        ss.set_field(tgpu(xs[f]), a1=0.15, a2=12.0)
        for op in ("M", "MT", "MTM"):
            assert rel(mv[op][sl], ss.matvec(v[sl].contiguous(), op).cpu().numpy()) < 1e-14, op
        assert rel(pcv[sl], ss.precond(v[sl].contiguous(), "FFT").cpu().numpy()) < 1e-14
        for (prec, pre), (u, st) in sols.items():
            u1, st1 = ss.solve(b[sl].contiguous(), tol=1e-10, prec=prec, precond=pre)
            # Launch shapes (operator chunks, preconditioner tiles) follow the launch's
            # right-hand-side count, so partial sums are added in another order and CG's
            # iteration count near the tolerance can move by a few percent; the solutions
            # agree to the tolerance.
            it, it1 = [s["iters"] for s in st[sl]], [s["iters"] for s in st1]
            assert all(abs(a - c) <= max(2, 0.03 * c) for a, c in zip(it, it1)), (prec, pre, it, it1)
            assert rel(u[sl].cpu().numpy(), u1.cpu().numpy()) < 1e-7, (prec, pre)
            assert all(s["status"] == 1 and s["rel_resid"] < 1e-10 for s in st[sl])
        g1 = ss.force(u_ref[sl].contiguous(), scale=0.5).cpu().numpy()
        assert rel(g[f], g1) < 1e-13


def test_multifield_limits_and_reset():
    from paper_2203_01291_amd._lib import FphError
    from paper_2203_01291_amd.solver import FermionSolver
    p = get_config("c1")
    s = FermionSolver.from_params(p, max_rhs=4)
    xs = tgpu(np.stack([phonon_field(p), phonon_field(p) + 0.1]))
    s.set_fields(xs, rhs_per_field=2)
    b = tgpu(gaussian_rhs(p, 4))
    s.solve(b, tol=1e-8, precond=True)
    with pytest.raises(FphError):                      # more than nfields * rhs_per_field
        s.matvec(tgpu(gaussian_rhs(p, 5)), "M")
    with pytest.raises(FphError):                      # the one-launch solve takes one field
        s.solve(b[:1].contiguous(), tol=1e-8, prec="f32_refined", variant=2)
    s.set_field(xs[1].contiguous())                    # back to one shared field
    u, st = s.solve(b, tol=1e-10, prec="f64", precond=True)
    assert all(v["status"] == 1 for v in st)
    s2 = FermionSolver.from_params(p, max_rhs=4)
    s2.set_field(xs[1].contiguous())
    u2, _ = s2.solve(b, tol=1e-10, prec="f64", precond=True)
    assert np.array_equal(u.cpu().numpy(), u2.cpu().numpy())


@pytest.mark.parametrize("lam", [False, True], ids=["Sprime", "Lambda"])
def test_chains_equal_single_chain(lam):
    """K chains advanced together (hmc_trajectories) give, chain by chain, the single-chain
    trajectory: with FP64 solves to 1e-12 the fields, energies and accept decisions agree to
    the solves' rounding; with the paper's tolerances the energy changes stay close."""
    from paper_2203_01291_amd._lib import FphError
    from paper_2203_01291_amd.hmc import PhononHMC
    from paper_2203_01291_amd.solver import FermionSolver
    p = get_config("c1")
    hp = hmc_params(p, Nt=20)
    K, nf = 3, 2
    x0 = np.stack([phonon_field(p) + 0.1 * k for k in range(K)])
    draws = [hmc_draws(p, nf, traj=k) for k in range(K)]
    Rf = np.stack([d[0] for d in draws])
    Rm = np.stack([d[1] for d in draws])
    rs = [d[2] for d in draws]
    for tol, prec, xtol, htol in ((1e-12, "f64", 1e-8, 1e-7), (hp.tol_force, "f32_refined", None, 0.05)):
        kw = dict(Nt=hp.Nt, nt=hp.nt, force_tol=tol, action_tol=hp.tol_action, prec=prec,
                  lambda_action=lam)
        sm = FermionSolver.from_params(p, max_rhs=K * nf)
        hm = PhononHMC(sm, hp.omega0, hp.m_reg, hp.dt, nchains=K, **kw)
        xg = tgpu(x0)
        pm = torch.empty_like(xg)
        st = hm.trajectories(xg, tgpu(Rf), tgpu(Rm), rs, p_out=pm)
        assert len(st) == K
        with pytest.raises(FphError):                      # one-chain entry points refuse K > 1
            hm.trajectory(xg[0].contiguous(), tgpu(Rf[0]), tgpu(Rm[0]), 0.5)
        with pytest.raises(FphError):
            hm.global_update(xg[0].contiguous(), "reflect", 0, 0, tgpu(Rf[0]), 0.5)
        ss = FermionSolver.from_params(p, max_rhs=nf)
        hs = PhononHMC(ss, hp.omega0, hp.m_reg, hp.dt, **kw)
        for k in range(K):
            x1 = tgpu(x0[k])
            p1 = torch.empty_like(x1)
            s1 = hs.trajectory(x1, tgpu(Rf[k]), tgpu(Rm[k]), rs[k], p_out=p1)
            dh, dh1 = st[k]["H_f"] - st[k]["H_i"], s1["H_f"] - s1["H_i"]
            assert st[k]["H_i"] == pytest.approx(s1["H_i"], rel=1e-12)
            if xtol is not None:
                assert st[k]["accepted"] == s1["accepted"]
                assert abs(dh - dh1) < htol, (k, dh, dh1)
                assert rel(pm[k].cpu().numpy(), p1.cpu().numpy()) < xtol
                if s1["accepted"]:
                    assert rel(xg[k].cpu().numpy(), x1.cpu().numpy()) < xtol
                else:
                    assert np.array_equal(xg[k].cpu().numpy(), x0[k])
            else:
                assert abs(dh - dh1) < htol, (k, dh, dh1)
            assert st[k]["solves"] == s1["solves"]
        hm.close()
        hs.close()
