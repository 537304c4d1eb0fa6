"""GPU parity of the Lambda reformulation (A = M Lambda) and of the reflection and swap
updates (Secs. II C, IV) against the CPU oracle, through the C ABI.

Tolerances: Lambda applies and the Lambda force term agree to rounding
(1e-14 relative); forces from FP64 solves to 1e-12 to 1e-9; whole
trajectories (FP64 solves to 1e-13) and global updates (1e-12) match the
oracle's LU-based ones to 1e-8 (fields) and 1e-8 absolute (energies,
actions).  The single-site adiabatic limit checks the paper's symmetry
claim on the GPU: a reflection is free with the action S and costly with S'.
"""

import numpy as np
import pytest

from oracle import hmc as OH
from oracle import lam as OLA
from oracle import lattice as OL
from workloads import get_config, hmc_draws, hmc_params, phonon_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def tgpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def make(lat, omega0, m_reg=None, dt=0.01, Nt=10, nt=2, nfields=2, **kw):
    from paper_2203_01291_amd.hmc import PhononHMC
    from paper_2203_01291_amd.solver import FermionSolver
    s = FermionSolver(lat.L, lat.Ltau, lat.dtau, lat.t, lat.mu, lat.alpha, max_rhs=max(nfields, 2))
    return s, PhononHMC(s, omega0, m_reg, dt, Nt=Nt, nt=nt, nfields=nfields, **kw)


SHAPES = [(4, 40, 0.1, 1.0, 0.0, 1.0), (6, 42, 0.1, 1.0, 0.2, 1.3), (10, 2, 0.1, 1.0, 0.0, 1.0),
          (32, 400, 0.05, 1.0, -0.2, 1.2)]
IDS = [f"L{s[0]}_T{s[1]}" for s in SHAPES]


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_lambda_apply_and_force_term(shape):
    lat = OL.Lattice(*shape)
    rng = np.random.default_rng(lat.L + lat.Ltau)
    x = rng.standard_normal((lat.Ltau, lat.N))
    v = rng.standard_normal((2, lat.Ltau, lat.N))
    s, h = make(lat, 1.0)
    xg, vg = tgpu(x), tgpu(v)
    Lm = OLA.lambda_sparse(lat, x)
    Li = OLA.lambda_inv_sparse(lat, x)
    for op, mat in (("L", Lm), ("Linv", Li), ("LT", Lm.T), ("LinvT", Li.T)):
        ref = np.stack([(mat @ r.ravel()).reshape(lat.Ltau, lat.N) for r in v])
        assert relmax(h.lambda_apply(xg, vg, op).cpu().numpy(), ref) < 1e-14, op
    b, u = v, rng.standard_normal((2, lat.Ltau, lat.N))
    g0 = rng.standard_normal((lat.Ltau, lat.N))
    grad = tgpu(g0)
    h.lambda_force(tgpu(b), tgpu(u), grad, scale=0.7)
    ref = g0 + 0.7 * (-lat.dtau * lat.alpha) * np.roll(np.sum(b * u, axis=0), 1, axis=0)
    assert relmax(grad.cpu().numpy(), ref) < 1e-14


@pytest.mark.parametrize("key", ["c1", "c2"])
def test_lambda_force_end_to_end(key):
    """b = Lambda^{-T} Phi, FP64 solve, fermion_force + lambda_force (1/2 per field) against
    the oracle's force of the Lambda action."""
    p = get_config(key)
    lat = OL.Lattice.from_params(p)
    x0 = phonon_field(p)
    R, _, _ = hmc_draws(p, 2)
    C = OL.sparse_C(lat).toarray() if lat.N > 16 else None
    Phis = OLA.pseudofermions(lat, x0, R, C)
    x = x0 + 0.1 * np.random.default_rng(3).standard_normal(x0.shape)
    ref = OLA.fermion_force(lat, x, Phis, C)
    s, h = make(lat, p.omega)
    xg = tgpu(x)
    s.set_field(xg)
    b = h.lambda_apply(xg, tgpu(Phis), "LinvT")
    u, st = s.solve(b, tol=1e-12, prec="f64", precond=True, maxiter=20000)
    assert st[0]["status"] == 1 and st[1]["status"] == 1
    g = s.force(u, scale=0.5)
    h.lambda_force(b, u, g, scale=0.5)
    assert relmax(g.cpu().numpy(), ref) < 1e-9


LTRAJ = [("c1_lambda", (4, 40, 0.1, 1.0, 0.0, 1.0), 1.0, "w0", 100, 10),
         ("L6_T42_lambda_inf", (6, 42, 0.1, 1.0, 0.2, 1.3), 0.7, None, 20, 4)]


@pytest.mark.parametrize("case", LTRAJ, ids=[c[0] for c in LTRAJ])
def test_lambda_trajectory_parity(case):
    name, shape, w0, mreg, Nt, nt = case
    lat = OL.Lattice(*shape)
    m_reg = w0 if mreg == "w0" else mreg
    rng = np.random.default_rng(sum(map(ord, name)))
    x = 0.5 * rng.standard_normal((lat.Ltau, lat.N))
    R = rng.standard_normal((2, lat.Ltau, lat.N))
    Rm = rng.standard_normal((lat.Ltau, lat.N))
    dt = 1.0 / (100 * w0)
    ref = OH.hmc_update(lat, w0, m_reg, dt, Nt, nt, x, R, Rm, 0.0, lam=True)
    s, h = make(lat, w0, m_reg, dt, Nt=Nt, nt=nt, force_tol=1e-13, action_tol=1e-13, precond=False,
                prec="f64", maxiter=20000, lambda_action=True)
    xg = tgpu(x)
    pg = torch.empty_like(xg)
    st = h.trajectory(xg, tgpu(R), tgpu(Rm), 0.0, p_out=pg)
    assert st["status"] == 1, st
    assert relmax(pg.cpu().numpy(), ref["p_f"]) < 1e-8
    assert relmax(xg.cpu().numpy(), ref["x_f"]) < 1e-8
    for k, gk in (("S_B", "SB"), ("S_F", "SF"), ("K", "K")):
        assert st[gk + "_i"] == pytest.approx(ref["H_i"][k], abs=1e-8, rel=1e-12), k
        assert st[gk + "_f"] == pytest.approx(ref["H_f"][k], abs=1e-8, rel=1e-12), k
    assert st["H_f"] - st["H_i"] == pytest.approx(ref["dH"], abs=1e-8)


MOVES = [("c1", "reflect", (5, -1), True), ("c1", "swap", (2, 3), True), ("c1", "reflect", (9, -1), False),
         ("c1", "swap", (0, 15), False), ("c2", "reflect", (77, -1), True), ("c2", "swap", (40, 41), True)]


@pytest.mark.parametrize("case", MOVES, ids=[f"{c[0]}_{c[1]}_{'S' if c[3] else 'Sprime'}" for c in MOVES])
def test_global_update_parity(case):
    key, kind, (i, j), lam = case
    p = get_config(key)
    lat = OL.Lattice.from_params(p)
    C = OL.sparse_C(lat).toarray() if lat.N > 16 else None
    x = phonon_field(p)
    R, _, r = hmc_draws(p, 2, traj=7)
    sites = (i,) if kind == "reflect" else (i, j)
    ref = OLA.global_update(lat, p.omega, x, kind, sites, R, r, lam=lam, C=C)
    s, h = make(lat, p.omega, action_tol=1e-12, prec="f64", precond=True, maxiter=20000, lambda_action=lam)
    xg = tgpu(x)
    st = h.global_update(xg, kind, i, j if kind == "swap" else 0, tgpu(R), r)
    print(key, kind, lam, st, "oracle dS", ref["dS"], flush=True)
    assert st["status"] == 1
    assert st["dS_B"] == pytest.approx(ref["dS_B"], abs=1e-8)
    assert st["SF_old"] == pytest.approx(ref["S_F_old"], rel=1e-11)
    assert st["SF_new"] == pytest.approx(ref["S_F_new"], rel=1e-11)
    assert st["dS"] == pytest.approx(ref["dS"], abs=1e-6)
    assert st["accepted"] == int(ref["accepted"])
    assert np.array_equal(xg.cpu().numpy(), ref["x_out"])


def test_reflection_free_in_adiabatic_single_site_limit():
    """t = 0, mu = 0, tau-constant field (App. B): reflecting a site leaves S unchanged to the
    solve tolerance for any Phi drawn at x (accepted with probability 1), while with S' the
    same move costs a large action (Sec. IV)."""
    lat = OL.Lattice(4, 40, 0.1, 0.0, 0.0, 2.0)
    x = np.full((lat.Ltau, lat.N), 2.0)          # x0 = alpha / omega0^2
    R = np.random.default_rng(4).standard_normal((2, lat.Ltau, lat.N))
    out = {}
    for lam in (True, False):
        s, h = make(lat, 1.0, action_tol=1e-12, prec="f64", precond=False, lambda_action=lam)
        xg = tgpu(x)
        out[lam] = h.global_update(xg, "reflect", 6, 0, tgpu(R), 0.999)
    assert abs(out[True]["dS"]) < 1e-6 and out[True]["accepted"] == 1
    assert out[False]["dS"] > 5.0 and out[False]["accepted"] == 0


def test_lambda_trajectory_c3_paper_settings():
    """c3 with the Lambda action and the paper's HMC settings and solver tolerances: solves
    converge; energies of the returned state match the oracle's; S_F(x_i) = |R|^2/2."""
    p = get_config("c3")
    lat = OL.Lattice.from_params(p)
    hp = hmc_params(p)
    x = phonon_field(p)
    R, Rm, r = hmc_draws(p, 2)
    s, h = make(lat, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, force_tol=hp.tol_force,
                action_tol=hp.tol_action, a1=0.15, a2=12.0, lambda_action=True)
    xg = tgpu(x)
    pf = torch.empty_like(xg)
    st = h.trajectory(xg, tgpu(R), tgpu(Rm), 0.0, p_out=pf)
    print("c3 lambda trajectory", st, flush=True)
    assert st["status"] == 1
    mt = OH.mass_tilde(lat.Ltau, lat.dtau, hp.omega0, hp.m_reg)
    assert st["SB_f"] == pytest.approx(OH.bosonic_action(lat, xg.cpu().numpy(), hp.omega0), rel=1e-11)
    assert st["K_f"] == pytest.approx(OH.kinetic_energy(pf.cpu().numpy(), mt), rel=1e-11)
    assert st["SF_i"] == pytest.approx(0.5 * np.sum(R ** 2), rel=1e-12)
    assert abs(st["H_f"] - st["H_i"]) < 5.0


def test_reflection_acceptance_single_site_paper_values():
    """The paper's printed acceptance of single-site reflections (Sec. IV): omega0 = 1,
    alpha = 2, beta = 4, half filling; about 68 % with S and about 2 % with S'.  Sixteen
    independent sites (t = 0) are sampled by this library's HMC with the action S (paper
    settings, 40 trajectories to equilibrate from x = alpha/omega0^2), then after each of 60
    further trajectories every site's reflection is proposed with fresh Phi under both actions
    and the Metropolis probabilities are averaged (960 proposals each).  Statistical: the
    bounds allow about four standard errors of a correlated sample."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))[
        "reflection_acceptance"]
    dtau = 0.1
    Ltau = int(round(g["beta"] / dtau))
    lat = OL.Lattice(4, Ltau, dtau, g["t"], g["mu"], g["alpha"])
    w0 = g["omega0"]
    kw = dict(Nt=100, nt=10, force_tol=1e-8, action_tol=1e-10, precond=False, prec="f64")
    s, hS = make(lat, w0, w0, 0.01 / w0, lambda_action=True, **kw)
    from paper_2203_01291_amd.hmc import PhononHMC
    hP = PhononHMC(s, w0, w0, 0.01 / w0, nfields=2, lambda_action=False, **kw)
    rng = np.random.default_rng(2203)
    x = tgpu(g["alpha"] / w0 ** 2 + 0.1 * rng.standard_normal((Ltau, lat.N)))
    accS, accP = [], []
    for it in range(100):
        st = hS.trajectory(x, tgpu(rng.standard_normal((2, Ltau, lat.N))),
                           tgpu(rng.standard_normal((Ltau, lat.N))), rng.random())
        assert st["status"] == 1
        if it < 40:
            continue
        for i in range(lat.N):
            R2 = tgpu(rng.standard_normal((2, Ltau, lat.N)))
            accS.append(hS.global_update(x, "reflect", i, 0, R2, 1.0)["accept_prob"])
            accP.append(hP.global_update(x, "reflect", i, 0, R2, 1.0)["accept_prob"])
    aS, aP = float(np.mean(accS)), float(np.mean(accP))
    print("reflection acceptance: S", aS, "S'", aP, flush=True)
    assert abs(aS - g["S"]) < 0.08
    assert abs(aP - g["S_prime"]) < 0.015
