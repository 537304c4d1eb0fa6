#!/usr/bin/env python3
"""Benchmark of the Holstein fermion solve on one MI355X.

One step = one pass of the hot path over the workload: per-field setup
(E, dbar, preconditioner bounds and Chebyshev tables), the FP32-refined
preconditioned CG solve of (M^T M) u = Phi to relative residual 1e-8, the
action S_F = Phi . u and the phonon force dS_F/dx.  Default workload:
L = 32 (N = 1024), Ltau = 400 (d = 409600), dtau = 0.05, mu = -0.2,
alpha = 1.2, AR(1)-correlated field.  The Chebyshev orders use
N_P = floor(db (a1/phi + a2)) with a1 = 0.15, a2 = 12 (--a1, --a2): the
fastest pair of a sweep (a1 from 0.05 to 0.5, a2 from 1 to 32) in mean
solve time over four synthetic fields of this shape.

Prints one JSON line: the headline (FP32-refined solves/s), the same step
with FP64 CG, one step of every solver variant, the fused M^T M roofline
(HIP events on the stream the kernel runs on) on a working set above the
Infinity Cache and at the workload shape, the batched persistent solve,
one full HMC update with the paper's settings, the stochastic Green's-function
measurements, and the CPU oracle timed on a bounded sample.
"""

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MᵀM matvec GB/s (% HBM peak) + PCG solves/s, FP32-refined vs FP64 @1e-8"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--precond", type=int, default=1,
                    help="1: preconditioned CG in the timed step (default); 0: plain CG; "
                         "-1: the faster of one trial each")
    ap.add_argument("--a1", type=float, default=0.15,
                    help="Chebyshev order coefficient a1 of N_P = floor(db (a1/phi + a2))")
    ap.add_argument("--a2", type=float, default=12.0)
    ap.add_argument("--matvec-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the one-step timing of every solver variant")
    ap.add_argument("--no-hmc", action="store_true", help="skip the HMC trajectory leg")
    ap.add_argument("--hmc-only", action="store_true",
                    help="only the HMC trajectory leg (one warm-up and one timed trajectory)")
    ap.add_argument("--no-meas", action="store_true", help="skip the measurement leg")
    ap.add_argument("--meas-only", action="store_true",
                    help="only the stochastic Green's-function measurement leg")
    ap.add_argument("--nrv", type=int, default=10, help="random vectors of the measurement leg")
    ap.add_argument("--no-ssh", action="store_true", help="skip the SSH-coupling leg")
    ap.add_argument("--ssh-only", action="store_true", help="only the SSH-coupling leg")
    ap.add_argument("--ssh-g", type=float, default=0.2, help="SSH coupling g of the SSH leg")
    ap.add_argument("--ssh-hmc", action="store_true",
                    help="with --ssh-only: also time one HMC trajectory on the SSH operator (paper "
                         "settings, FP64 preconditioned solves; about 10 s)")
    ap.add_argument("--profile-roofline", action="store_true",
                    help="only the roofline kernel (M^T M at L=64 Ltau=400: FP64 x 40 rhs, FP32 x "
                         "80 rhs) and a plain copy of the FP64 byte count, for hardware-counter runs")
    ap.add_argument("--profile-step", action="store_true",
                    help="only two steps (the first one a warm-up) of the workload's timed step, "
                         "for kernel traces and hardware-counter runs")
    return ap.parse_args()


def time_steps(step, steps, warmup, torch):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def event_time_matvec(solver, v, op, reps, torch, isolated=False):
    """Average duration (s) of one apply, HIP events on the stream the
    kernel runs on.  isolated=False: the median over 5 groups of `reps`
    back-to-back launches between two events (the figure used for
    rooflines; it agrees with the kernel trace's average duration); True:
    each launch between its own events and waited for (adds the start-up of
    an idle GPU to every launch)."""
    out = torch.empty_like(v)
    for _ in range(5):
        solver.matvec(v, op, out=out)
    stream = torch.cuda.current_stream()
    if not isolated:
        # median over 5 groups of `reps` back-to-back launches
        groups = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                solver.matvec(v, op, out=out)
            e1.record(stream)
            e1.synchronize()
            groups.append(e0.elapsed_time(e1) / 1e3 / reps)
        return sorted(groups)[2]
    tot = 0.0
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        solver.matvec(v, op, out=out)
        e1.record(stream)
        e1.synchronize()
        tot += e0.elapsed_time(e1) / 1e3
    return tot / reps


def bench_batched(torch, dev, log):
    """The batched workload: 64 systems with L drawn from {8, ..., 24},
    Ltau = 100, 8 Gaussian pseudofermion and 32 Rademacher right-hand sides
    each (2560 solves), FP32 CG with FP64 residual replacement to 1e-8, one
    persistent graph-replayed launch with an autotuned shape."""
    import time as _t

    from paper_2203_01291_amd.solver import FermionBatch, FermionSolver
    from workloads import (batched_systems, gaussian_rhs, get_config, phonon_field,
                           rademacher_rhs)
    import numpy as np

    p = get_config("c4")
    Ls = batched_systems(p)
    ops = {}
    systems = []
    for k, L in enumerate(Ls):
        if L not in ops:
            ops[L] = FermionSolver.from_params(p, L=L, max_rhs=1)
        s = ops[L]
        x = torch.from_numpy(phonon_field(p, L=L, system=k)).to(dev)
        rhs = np.concatenate([gaussian_rhs(p, p.n_gauss, L=L, system=k),
                              rademacher_rhs(p, p.n_rademacher, L=L, system=k)])
        s.set_field(x)
        b = s.matvec(torch.from_numpy(rhs).to(dev), "MT").contiguous()   # b = M(x)^T (phi, xi)
        systems.append((type("P", (), dict(L=L, Ltau=p.Ltau, dtau=p.dtau, t=p.t, mu=p.mu,
                                           alpha=p.alpha)), x, b))
    torch.cuda.synchronize()
    for s in ops.values():
        s.close()
    bt = FermionBatch(systems)
    t0 = _t.perf_counter()
    best = bt.tune(tol=p.tol)
    tune_s = _t.perf_counter() - t0
    bt.solve(tol=p.tol)
    torch.cuda.synchronize()
    reps = 3
    t0 = _t.perf_counter()
    for _ in range(reps):
        st = bt.solve(tol=p.tol)
    torch.cuda.synchronize()
    dt = (_t.perf_counter() - t0) / reps
    nrhs = len(st)
    iters = [v["iters"] for v in st]
    conv = sum(1 for v in st if v["status"] & 1)
    dsum = sum(L * L * p.Ltau * (p.n_gauss + p.n_rademacher) for L in Ls)
    # Algorithmic traffic of the whole batch: per FP32 CG iteration the
    # operator pass (read r, p_old, E; write p, Ap) and the update pass (read
    # u, p, r, Ap; write u, r), 11 vectors of 4 bytes; per FP64 residual
    # replacement the FP64 operator on u with b (read u, E, b; write r32)
    # and the accumulation of u (read u32, u; write u), 7 vectors of 8 bytes.
    per_rhs_d = [L * L * p.Ltau for L in Ls for _ in range(p.n_gauss + p.n_rademacher)]
    alg_bytes = sum(d_i * (44 * v["iters"] + 56 * v["outer_iters"]) for d_i, v in zip(per_rhs_d, st))
    res = {
        "workload": f"{p.name}: 64 systems, L in {sorted(set(Ls))}, Ltau={p.Ltau}, "
                    f"{p.n_gauss}+{p.n_rademacher} rhs each, FP32 CG + FP64 residual "
                    f"replacement to {p.tol}, one persistent graph-replayed launch",
        "solves": nrhs, "converged": conv,
        "seconds": dt, "solves_per_s": nrhs / dt, "systems_per_s": len(Ls) / dt,
        "unknowns_total": dsum,
        "algorithmic_bytes": alg_bytes, "algorithmic_GB/s": alg_bytes / dt / 1e9,
        "algorithmic_GB/s_note": "bytes the method moves per second through the caches: about "
                                 "512 items of ~0.6 MB of live vectors stay in the 256 MB "
                                 "Infinity Cache, so this is not a fraction of HBM",
        "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
        "max_rel_resid": float(max(v["rel_resid"] for v in st)),
        "tuned_shape": best, "tune_seconds": tune_s,
    }
    log(f"batched: {res}")
    # The same batch preconditioned by F F^T inside each item's workgroup
    # (per-system tables; the paper's order-one Chebyshev constants, whose
    # total series length is the smallest).
    t0 = _t.perf_counter()
    best_p = bt.tune(tol=p.tol, precond=True)
    tune_p = _t.perf_counter() - t0
    bt.solve(tol=p.tol, precond=True)
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    for _ in range(reps):
        stp = bt.solve(tol=p.tol, precond=True)
    torch.cuda.synchronize()
    dtp = (_t.perf_counter() - t0) / reps
    itp = [v["iters"] for v in stp]
    res["preconditioned"] = {
        "chebyshev_a1_a2": [1.0, 1.0], "seconds": dtp, "solves_per_s": nrhs / dtp,
        "systems_per_s": len(Ls) / dtp, "speedup_vs_plain": dt / dtp,
        "converged": sum(1 for v in stp if v["status"] & 1),
        "iters_mean": float(np.mean(itp)), "iters_max": int(np.max(itp)),
        "max_rel_resid": float(max(v["rel_resid"] for v in stp)),
        "tuned_shape": best_p, "tune_seconds": tune_p}
    log(f"batched preconditioned: {res['preconditioned']}")
    bt.close()
    return res


def bench_hmc(torch, dev, p, a1, a2, log, batch_chains=8):
    """One HMC trial update (Algorithm 1) on the workload's lattice with the
    paper's settings: dt = 1/(100 omega0), Nt = 100 steps of nt = 10 bosonic
    sub-steps, Fourier acceleration with m_reg = omega0, two pseudofermion
    fields, FP32-refined preconditioned solves to 1e-5 for the forces (each
    from a zero guess) and to 1e-10 for the final action, FP64 energies.
    Starts from the workload's synthetic field; one warm-up trajectory, then
    one timed, with the action S' (A = M); then one with the action S
    (A = M Lambda) and four reflection / swap updates with it; and
    `batch_chains` independent chains in the same launches (one trajectory
    each)."""
    from paper_2203_01291_amd.hmc import PhononHMC
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import hmc_draws, hmc_params, phonon_field

    hp = hmc_params(p)
    s = FermionSolver.from_params(p, max_rhs=hp.nfields)
    x0 = torch.from_numpy(phonon_field(p)).to(dev)
    Rf, Rm, r = hmc_draws(p, hp.nfields)
    Rf = torch.from_numpy(Rf).to(dev)
    Rm = torch.from_numpy(Rm).to(dev)
    h = PhononHMC(s, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, nfields=hp.nfields, a1=a1, a2=a2,
                  force_tol=hp.tol_force, action_tol=hp.tol_action)
    x = x0.clone()
    h.trajectory(x, Rf, Rm, r)
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.trajectory(x, Rf, Rm, r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the bosonic sub-steps of one time step (composed map, two circulant
    # passes over x and p, plus two device copies back in place)
    xb, pb = x0.clone(), torch.randn_like(x0)
    for _ in range(3):
        h.boson_steps(xb, pb)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(50):
        h.boson_steps(xb, pb)
    e1.record(stream)
    e1.synchronize()
    boson_us = e0.elapsed_time(e1) / 50 * 1e3
    # The same update with the action S (A = M Lambda), and global updates
    # (reflection of one site, swap of two neighbours) with that action: one
    # solve to the action tolerance each.
    hl = PhononHMC(s, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, nfields=hp.nfields, a1=a1, a2=a2,
                   force_tol=hp.tol_force, action_tol=hp.tol_action, lambda_action=True)
    x = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stl = hl.trajectory(x, Rf, Rm, r)
    torch.cuda.synchronize()
    dtl = time.perf_counter() - t0
    moves = []
    for kind, i, j in (("reflect", 0, 0), ("reflect", 517, 0), ("swap", 0, 1), ("swap", 517, 549)):
        xm = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su = hl.global_update(xm, kind, i, j, Rf, r)
        torch.cuda.synchronize()
        moves.append({"kind": kind, "sites": [i, j] if kind == "swap" else [i],
                      "ms": (time.perf_counter() - t0) * 1e3, "dS": su["dS"], "cg_iters": su["cg_iters"],
                      "status": su["status"]})
    hl.close()
    # The same chains in the same launches: chain k's pseudofermions are
    # right-hand sides of its own field in every solve.
    batched = None
    if batch_chains > 1:
        nb = batch_chains
        sb = FermionSolver.from_params(p, max_rhs=nb * hp.nfields)
        hb = PhononHMC(sb, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, nfields=hp.nfields, a1=a1,
                       a2=a2, force_tol=hp.tol_force, action_tol=hp.tol_action, nchains=nb)
        Rfb = Rf.unsqueeze(0).expand(nb, *Rf.shape).contiguous()
        Rmb = Rm.unsqueeze(0).expand(nb, *Rm.shape).contiguous()
        xb = x0.unsqueeze(0).expand(nb, *x0.shape).contiguous()
        hb.trajectories(xb.clone(), Rfb, Rmb, [r] * nb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stb = hb.trajectories(xb, Rfb, Rmb, [r] * nb)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        batched = {"chains": nb, "seconds": dtb, "trajectories_per_s": nb / dtb,
                   "speedup_vs_one": (nb / dtb) * dt, "cg_iters": [v["cg_iters"] for v in stb],
                   "dH": [v["H_f"] - v["H_i"] for v in stb], "status": [v["status"] for v in stb]}
        hb.close()
        sb.close()
    res = {
        "workload": f"{p.name}: one HMC update, dt={hp.dt:g}, Nt={hp.Nt}, nt={hp.nt}, "
                    f"m_reg={hp.m_reg}, {hp.nfields} fields, FP32-refined PCG (a1={a1}, a2={a2}) "
                    f"to {hp.tol_force:g} (forces, zero guess) and {hp.tol_action:g} (action)",
        "ms_per_trajectory": dt * 1e3, "trajectories_per_s": 1.0 / dt,
        "solves": st["solves"], "cg_iters": st["cg_iters"],
        "cg_iters_per_force_solve_and_field": st["cg_iters"] / st["solves"] / hp.nfields,
        "dH": st["H_f"] - st["H_i"], "accept_prob": st["accept_prob"], "accepted": st["accepted"],
        "status": st["status"], "boson_step_us": boson_us,
        "boson_fraction": boson_us * 1e-6 * hp.Nt / dt,
        "chains_per_launch": batched,
        "lambda_action": {"ms_per_trajectory": dtl * 1e3, "cg_iters": stl["cg_iters"],
                          "dH": stl["H_f"] - stl["H_i"], "status": stl["status"],
                          "global_updates": moves},
    }
    log(f"hmc: {res}")
    h.close()
    s.close()
    return res


def bench_measure(torch, dev, p, a1, a2, nrv, log):
    """Stochastic Green's-function measurements (Sec. VI) on the workload's
    field: nrv Rademacher vectors, G xi from FP32-refined preconditioned
    solves to 1e-8 (nrv right-hand sides in one call), the space-time
    average of G^ext and the three pair-averaged four-point products by FFT
    cross-correlation; each part timed once after a warm-up."""
    from paper_2203_01291_amd.measure import GreenMeasurement
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import phonon_field, rademacher_rhs

    s = FermionSolver.from_params(p, max_rhs=nrv)
    s.set_field(torch.from_numpy(phonon_field(p)).to(dev), a1=a1, a2=a2)
    m = GreenMeasurement(s)
    xi = torch.from_numpy(rademacher_rhs(p, nrv)).to(dev)
    gx, _ = m.green_vectors(xi)
    m.green_average(xi, gx)
    m.pair_products(xi[:2], gx[:2])
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, r

    t_vec, (gx, st) = timed(lambda: m.green_vectors(xi))
    t_avg, _ = timed(lambda: m.green_average(xi, gx))
    t_pair, _ = timed(lambda: m.pair_products(xi, gx))
    z = torch.randn(p.Ltau, p.N, dtype=torch.complex128, device=dev)
    for _ in range(3):
        m.fft(z)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        m.fft(z)
    e1.record(stream)
    e1.synchronize()
    fft_us = e0.elapsed_time(e1) / 20 * 1e3
    npairs = nrv * (nrv - 1) // 2
    res = {
        "workload": f"{p.name}: {nrv} Rademacher vectors, G xi by FP32-refined PCG to 1e-8 "
                    f"(a1={a1}, a2={a2}), average of G^ext and {npairs}-pair four-point products",
        "green_vectors_ms": t_vec, "iters": [v["iters"] for v in st],
        "green_average_ms": t_avg, "pair_products_ms": t_pair,
        "fft3_us": fft_us, "grid": [p.Ltau, p.L, p.L],
        "fft3_per_pair_products": 4 * npairs + nrv,
    }
    log(f"measure: {res}")
    m.close()
    s.close()
    return res


def bench_ssh(torch, dev, p, g, a1, a2, log, hmc=False):
    """SSH-type coupling (x in the bond hoppings) on the workload's lattice and
    field: the M and M^T kernels timed with events (one and eight right-hand
    sides), and one step of set-field + FP64 CG to 1e-8 (no preconditioner)
    + S_F + force, the same step preconditioned with the Holstein adiabatic
    preconditioner of the field (uniform hopping), in FP64 and FP32-refined,
    and the preconditioned step with eight right-hand sides in both."""
    from paper_2203_01291_amd.solver import FermionSolver
    from paper_2203_01291_amd.ssh import SSHSolver
    from workloads import gaussian_rhs, phonon_field

    nr = 8
    s = SSHSolver.from_params(p, g, max_rhs=nr)
    x = torch.from_numpy(phonon_field(p)).to(dev)
    s.set_field(x)
    v = torch.from_numpy(gaussian_rhs(p, nr)).to(dev)
    stream = torch.cuda.current_stream()

    def kernel_us(op, n, reps=50):
        vin = v[:n].contiguous()
        out = torch.empty_like(vin)
        for _ in range(3):
            s.matvec(vin, op, out=out)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            s.matvec(vin, op, out=out)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    # algorithmic bytes of one M (or M^T) launch: per right-hand side read v_tau
    # and the transported slice, write out (3 d doubles); once per launch the
    # field's tables, bond (cosh, sinh) and E (5 d doubles)
    kern = {}
    for op in ("M", "MT"):
        for n in (1, nr):
            us = kernel_us(op, n)
            byts = (3.0 * n + 5.0) * p.dim * 8
            kern[f"{op}_rhs{n}"] = {"us": us, "GB/s": byts / us * 1e-3, "frac": byts / us * 1e-3 / HBM_PEAK_GBS}
    b = s.matvec(v[:1].contiguous(), "MT")
    s.solve(b, tol=1e-8, chunk=128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_field(x)
    u, st = s.solve(b, tol=1e-8, chunk=128)
    grad = s.force(u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fs = FermionSolver.from_params(p, max_rhs=nr)
    s.attach_preconditioner(fs, a1=a1, a2=a2)

    def pc_step(bv, prec):
        s.set_field(x)
        s.solve(bv, tol=1e-8, chunk=32, precond=True, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_field(x)
        uu, ss = s.solve(bv, tol=1e-8, chunk=32, precond=True, prec=prec)
        gg = s.force(uu)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, uu, ss, gg

    dtp, up, stp, gradp = pc_step(b, "f64")
    dtr, ur, str_, gradr = pc_step(b, "f32_refined")
    b8 = s.matvec(v, "MT")
    dt8, u8, st8, _ = pc_step(b8, "f64")
    dt8r, u8r, st8r, _ = pc_step(b8, "f32_refined")
    res = {
        "workload": f"{p.name}: SSH coupling g={g} (t_b = t - g (x_j - x_i)) with the Holstein on-site "
                    f"factor, FP64 CG to 1e-8 without preconditioner, S_F and force",
        "ms_per_step": dt * 1e3, "iters": st[0]["iters"], "rel_resid": st[0]["rel_resid"],
        "us_per_iteration": dt * 1e6 / max(1, st[0]["iters"]), "status": st[0]["status"],
        "grad_norm": float(grad.norm()), "kernels": kern,
        "preconditioned": {"ms_per_step": dtp * 1e3, "iters": stp[0]["iters"],
                           "rel_resid": stp[0]["rel_resid"], "status": stp[0]["status"],
                           "us_per_iteration": dtp * 1e6 / max(1, stp[0]["iters"]),
                           "grad_rel_diff": float((gradp - grad).norm() / grad.norm()),
                           "a1_a2": [a1, a2]},
        "preconditioned_f32_refined": {
            "ms_per_step": dtr * 1e3, "iters": str_[0]["iters"], "fp64_evaluations": str_[0]["outer_iters"],
            "rel_resid": str_[0]["rel_resid"], "status": str_[0]["status"],
            "speedup_vs_fp64": dtp / dtr,
            "u_rel_diff_vs_fp64": float((ur - up).abs().max() / up.abs().max()),
            "grad_rel_diff_vs_fp64": float((gradr - gradp).norm() / gradp.norm())},
        "preconditioned_rhs8": {
            "f64": {"ms_per_step": dt8 * 1e3, "solves_per_s": nr / dt8, "iters": [q["iters"] for q in st8],
                    "status": [q["status"] for q in st8]},
            "f32_refined": {"ms_per_step": dt8r * 1e3, "solves_per_s": nr / dt8r,
                            "iters": [q["iters"] for q in st8r], "status": [q["status"] for q in st8r],
                            "fp64_evaluations": [q["outer_iters"] for q in st8r]},
            "speedup_fp32_refined": dt8 / dt8r,
            "u_rel_diff": float((u8r - u8).abs().max() / u8.abs().max())},
    }
    if hmc:
        from paper_2203_01291_amd.hmc import PhononHMC
        from workloads import hmc_draws, hmc_params
        hp = hmc_params(p)
        s2 = SSHSolver.from_params(p, g, max_rhs=hp.nfields)
        fs2 = FermionSolver.from_params(p, max_rhs=hp.nfields)
        s2.attach_preconditioner(fs2, a1=a1, a2=a2)
        hh = PhononHMC(s2, hp.omega0, hp.m_reg, hp.dt, Nt=hp.Nt, nt=hp.nt, nfields=hp.nfields,
                       force_tol=hp.tol_force, action_tol=hp.tol_action, precond=True, prec="f64")
        Rf, Rm, r = hmc_draws(p, hp.nfields)
        xh = x.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sth = hh.trajectory(xh, torch.from_numpy(Rf).to(dev), torch.from_numpy(Rm).to(dev), r)
        torch.cuda.synchronize()
        res["hmc_trajectory"] = {
            "seconds": time.perf_counter() - t0, "solves": sth["solves"], "cg_iters": sth["cg_iters"],
            "dH": sth["H_f"] - sth["H_i"], "accepted": sth["accepted"], "status": sth["status"],
            "settings": f"dt={hp.dt:g}, Nt={hp.Nt}, nt={hp.nt}, m_reg={hp.m_reg}, {hp.nfields} fields, "
                        f"FP64 PCG to {hp.tol_force:g} (forces) and {hp.tol_action:g} (action)"}
        hh.close()
        s2.close()
        fs2.close()
    fs.close()
    log(f"ssh: {res}")
    s.close()
    return res


def cpu_baseline(p, golden_iters):
    """Oracle CG (scipy CSR, FP64) on the workload for a bounded number of
    iterations; scaled to solves/s with the oracle's own iteration count."""
    import numpy as np

    from oracle import lattice as OL
    from oracle import solve as OS
    from workloads import gaussian_rhs, perturbed_field, phonon_field

    lat = OL.Lattice.from_params(p)
    x0 = phonon_field(p)
    x = perturbed_field(p, x0)
    Cs = OL.sparse_C(lat)
    phi = gaussian_rhs(p, 1)[0]
    Phi = (OL.sparse_M(lat, x0, Cs).T @ phi.reshape(-1)).reshape(lat.Ltau, lat.N)
    mv = OS.normal_matvec_sparse(lat, x, Cs)
    n = 50
    while True:
        t0 = time.perf_counter()
        OS.cg(mv, Phi, tol=0.0, maxiter=n)
        dt = time.perf_counter() - t0
        if dt > 8.0 or n >= 4000:
            break
        n = int(n * max(2.0, 10.0 / max(dt, 1e-3)))
    per_iter = dt / n
    return {
        "value": 1.0 / (per_iter * golden_iters),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n} iterations of the oracle's textbook FP64 CG on the CSR M^T M "
                  f"(scipy, single-threaded SpMV) on the {p.name} system, "
                  f"{per_iter * 1e3:.2f} ms/iteration, scaled by the oracle's "
                  f"{golden_iters} iterations to 1e-8 (tests/golden/oracle_iterations.json)",
        "host_threads_available": os.cpu_count(),
        "host_cpu": host_cpu_model(),
        "blas_threads": blas_threads(),
    }


def host_cpu_model():
    """CPU model of the host: lscpu's model name (else /proc/cpuinfo's), with
    the family / model / stepping numbers appended when the name carries no
    model number (virtual machines often report only the brand)."""
    import subprocess
    name = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                name = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    ids = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # first processor only
                k, _, v = line.partition(":")
                ids[k.strip()] = v.strip()
    except Exception:
        pass
    if name is None:
        name = ids.get("model name")
    if name is not None and not any(c.isdigit() for c in name):
        extra = ", ".join(f"{k} {ids[k]}" for k in ("cpu family", "model", "stepping") if k in ids)
        if extra:
            name = f"{name} ({extra})"
    return name


def blas_threads():
    """Threads of the BLAS numpy links against (the CG's SpMV is scipy's own
    single-threaded code; BLAS serves only its dot products)."""
    try:
        from threadpoolctl import threadpool_info
        return [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    except Exception:
        return None


# HBM traffic of the roofline kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of `bench.py --profile-roofline`, each scaled by the same
# counter read for a copy kernel of known size.  Valid only while the
# kernel sources hash to `source_sha1`; otherwise reported as null.
# FETCH_SIZE scale 518400 / 259212.56 = 1.99990 (a copy of 518 400 KiB reads
# that much), WRITE_SIZE scale 1.0; bytes per launch = (FETCH * 1.99990 +
# WRITE) KiB * 1024, means over 10 launches.
TRAFFIC = {"f64_bytes_per_launch": 1091013026, "f32_bytes_per_launch": 1088841079,
           "fetch_scale": 1.99990, "write_scale": 1.0,
           "source_sha1": "7ebe70fca504328e6af8a94048a62e021c1fd05e",
           "profile": "profiles/mtm_L64_Ltau400_roofline_counters.md"}
KERNEL_SOURCES = ["paper_2203_01291_amd/csrc/fph_matvec.h", "paper_2203_01291_amd/csrc/fph_common.h",
                  "paper_2203_01291_amd/csrc/fph_lib.hip"]


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# Right-hand sides of the roofline applies: (2R + 1) d w bytes per launch at
# L = 64, Ltau = 400 (d = 1 638 400) must exceed 4 x the 256 MB Infinity
# Cache (1.03 GB): FP32 R = 80 -> 1.055 GB, FP64 R = 40 -> 1.062 GB.
ROOF_R32 = 80
ROOF_R64 = 40


def large_matvec_setup(torch, dev, R5=ROOF_R32):
    """The roofline workload: fused M^T M at L = 64, Ltau = 400 (c5 shape)
    with R5 right-hand sides sharing one field (FP64 values; slices of it
    serve the smaller FP64 leg)."""
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import get_config, phonon_field
    p5 = get_config("c5")
    s5 = FermionSolver.from_params(p5, max_rhs=1)
    s5.set_field(torch.from_numpy(phonon_field(p5)).to(dev))
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    vl = torch.randn(R5, p5.Ltau, p5.N, device=dev, dtype=torch.float64, generator=g)
    return p5, R5, s5, vl


def error_vs_golden(key, u, g, S, tol):
    """Relative error of a solution u, force g and action S of the workload
    `key` (x = x0 + 0.1 N(0,1), Phi = M(x0)^T phi) against the oracle's
    stored values (its FP64 CG to relative residual 1e-13) at the stored
    sample components: 2-norm over the samples and largest element-wise
    error over the largest sample."""
    import numpy as np
    from workloads import get_config
    p = get_config(key)
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_{key}.json")
    if not os.path.exists(gold_path):
        return None
    gold = json.load(open(gold_path))
    idx = np.array(gold["samples"])
    uh = u.reshape(p.Ltau, p.N).cpu().numpy()[idx[:, 0], idx[:, 1]]
    gh = g.reshape(p.Ltau, p.N).cpu().numpy()[idx[:, 0], idx[:, 1]]
    ur, gr = np.array(gold["u_samples"]), np.array(gold["force_samples"])
    return {"reference": "oracle FP64 CG to relative residual 1e-13, same inputs (tests/golden)",
            "components": int(len(idx)), "solve_tol": tol,
            "u_rel": float(np.linalg.norm(uh - ur) / np.linalg.norm(ur)),
            "u_maxrel": float(np.max(np.abs(uh - ur)) / np.max(np.abs(ur))),
            "force_rel": float(np.linalg.norm(gh - gr) / np.linalg.norm(gr)),
            "force_maxrel": float(np.max(np.abs(gh - gr)) / np.max(np.abs(gr))),
            "S_F_rel": float(abs(float(S) - gold["S_F"]) / abs(gold["S_F"]))}


def bench_workload_tols(torch, dev, key, tols, steps, log):
    """The step (set-field + preconditioned PCG + S_F + force) of workload
    `key` with its tuned Chebyshev constants, FP32-refined and FP64, at each
    solve tolerance of `tols`: ms per step, iterations and the error against
    the oracle's stored values."""
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import gaussian_rhs, get_config, perturbed_field, phonon_field
    p = get_config(key)
    a1, a2 = p.cheb
    s = FermionSolver.from_params(p)
    x0 = torch.from_numpy(phonon_field(p)).to(dev)
    x = torch.from_numpy(perturbed_field(p, phonon_field(p))).to(dev)
    s.set_field(x0)
    Phi = s.matvec(torch.from_numpy(gaussian_rhs(p, 1)).to(dev), "MT")
    torch.cuda.synchronize()
    out = {"workload": f"{p.name}: L={p.L} Ltau={p.Ltau} d={p.dim}, preconditioned "
                       f"(a1={a1}, a2={a2}), set-field + PCG + S_F + force per step"}
    for tol in tols:
        row = {}
        for prec in ("f32_refined", "f64"):
            last = {}

            def step():
                s.set_field(x, a1=a1, a2=a2)
                u, st = s.solve(Phi, tol=tol, prec=prec, precond=True)
                last["S"], last["g"], last["u"] = s.action(Phi, u), s.force(u), u
                return st
            t, st = time_steps(step, steps, 1, torch)
            row[prec] = {"ms_per_step": t * 1e3, "solves_per_s": 1.0 / t, "iters": st[0]["iters"],
                         "outer": st[0]["outer_iters"], "status": st[0]["status"],
                         "rel_resid": st[0]["rel_resid"],
                         "error_vs_oracle": error_vs_golden(key, last["u"], last["g"],
                                                            float(last["S"][0]), tol)}
        row["speedup_fp32_refined"] = row["f64"]["ms_per_step"] / row["f32_refined"]["ms_per_step"]
        out[f"tol_{tol:g}"] = row
        log(f"{key} tol {tol:g}: {row}")
    s.close()
    return out


def bench_graph_step(torch, dev, p, a1, a2, log, replays=3):
    """The step as a hipGraph: set-field + enqueue-only pcg_solve
    (FP32-refined, preconditioned, tol 1e-8) + S_F + force captured once and
    replayed.  pcg_solve enqueues 1 + maxiter + max_outer slots, so maxiter
    is an iteration budget: here 1.05 x the iterations the blocking solve
    needed on this field, max_outer 16."""
    from paper_2203_01291_amd._lib import stats_from_device
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import gaussian_rhs, perturbed_field, phonon_field
    s = FermionSolver.from_params(p)
    x0 = torch.from_numpy(phonon_field(p)).to(dev)
    x = torch.from_numpy(perturbed_field(p, phonon_field(p))).to(dev)
    s.set_field(x0)
    Phi = s.matvec(torch.from_numpy(gaussian_rhs(p, 1)).to(dev), "MT")
    s.set_field(x, a1=a1, a2=a2)
    _, st = s.solve(Phi, tol=1e-8, prec="f32_refined", precond=True)
    budget = int(1.05 * st[0]["iters"]) + 1
    u = torch.zeros_like(Phi)
    stats = torch.zeros(4, dtype=torch.float64, device=dev)
    S = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(p.Ltau, p.N, dtype=torch.float64, device=dev)

    def step():
        s.set_field(x, a1=a1, a2=a2)
        s.solve_async(Phi, u=u, stats=stats, tol=1e-8, maxiter=budget, precond=True,
                      prec="f32_refined", zero_guess=True, max_outer=16)
        s.action(Phi, u, out=S)
        g.zero_()
        s.force(u, grad=g)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / replays
    sd = stats_from_device(stats)[0]
    res = {"iteration_budget": budget, "blocking_iters": st[0]["iters"], "status": sd["status"],
           "iters": sd["iters"], "rel_resid": sd["rel_resid"],
           "eager_enqueue_only_ms": t_eager * 1e3, "graph_replay_ms": t_graph * 1e3,
           "error_vs_oracle": error_vs_golden(p_key(p), u, g, float(S[0]), 1e-8)}
    log(f"graph step: {res}")
    del graph
    s.close()
    return res


# Workgroups of the block-contiguous copies: the grids of the FP64 (40 rhs x
# 6 chunks) and FP32 (80 rhs x 6 chunks) roofline applies.
CEILING_BLOCKS = (240, 480)


def hbm_ceilings(torch, dev, nbytes):
    """Bandwidth of copies moving `nbytes` (half read, half written): the
    runtime's own copy, and fph_hbm_copy with every workgroup sweeping one
    window (the best pattern for HBM) and with each workgroup copying its own
    contiguous part (the operator's pattern), at the operator's grids.
    Median over 5 groups of 10 launches, HIP events on the launch stream."""
    from paper_2203_01291_amd import _lib
    lib = _lib.load()
    src = torch.empty(nbytes // 8, dtype=torch.float32, device=dev).normal_()
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    half = src.numel() * 4

    def fph_copy(pattern, nblocks):
        def f():
            rc = lib.fph_hbm_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  half, nblocks, pattern, sp)
            if rc != 0:
                raise RuntimeError(f"fph_hbm_copy: {lib.fph_strerror(rc).decode()}")
        return f

    def timed(f):
        f()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                f()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 10 * 1e-3)
        t = sorted(ts)[2]
        return {"us": t * 1e6, "GB/s": nbytes / t / 1e9, "frac": nbytes / t / 1e9 / HBM_PEAK_GBS}

    out = {"bytes": nbytes, "runtime_copy": timed(lambda: dst.copy_(src)),
           "window_copy": timed(fph_copy(0, 0))}
    for g in CEILING_BLOCKS:
        out[f"block_copy_{g}wg"] = timed(fph_copy(1, g))
    if not torch.equal(src, dst):
        raise RuntimeError("fph_hbm_copy: copy differs from its source")
    del src, dst
    return out


def p_key(p):
    from workloads import CONFIGS
    return next(k for k, v in CONFIGS.items() if v.name == p.name)


def profile_roofline(torch, dev):
    """For hardware-counter runs: 10 FP64 applies (ROOF_R64 rhs), 10 FP32
    applies (ROOF_R32 rhs) of the roofline kernel, then 10 runtime copies of
    the FP64 apply's byte count (the reference for the counter scale) and 10
    of each of the library's copy patterns on the same buffers."""
    p5, R5, s5, vl = large_matvec_setup(torch, dev)
    v64 = vl[:ROOF_R64].contiguous()
    out = torch.empty_like(v64)
    for _ in range(10):
        s5.matvec(v64, "MTM", out=out)
    del v64, out
    v32 = vl.float()
    del vl
    out = torch.empty_like(v32)
    for _ in range(10):
        s5.matvec(v32, "MTM", out=out)
    del v32, out
    nbytes64 = (2 * ROOF_R64 + 1) * p5.dim * 8
    nbytes32 = (2 * R5 + 1) * p5.dim * 4
    src = torch.empty(nbytes64 // 8, dtype=torch.float32, device=dev).normal_()
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    # the library's copies of the same buffer: one window, then block-contiguous
    from paper_2203_01291_amd import _lib
    lib = _lib.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for pattern, nblocks in [(0, 0)] + [(1, g) for g in CEILING_BLOCKS]:
        for _ in range(10):
            rc = lib.fph_hbm_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  src.numel() * 4, nblocks, pattern, sp)
            if rc != 0:
                raise RuntimeError(f"fph_hbm_copy: {lib.fph_strerror(rc).decode()}")
    torch.cuda.synchronize()
    print(json.dumps({"mtm_f64_launches": 10, "mtm_f64_bytes": nbytes64, "mtm_f32_launches": 10,
                      "mtm_f32_bytes": nbytes32, "copy_launches": 10,
                      "copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))


def profile_step(torch, dev, p, a1, a2):
    """For kernel traces and counter runs: two steps of the timed path
    (set-field + FP32-refined PCG to 1e-8 + S_F + force, one right-hand
    side), the first one a warm-up."""
    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import gaussian_rhs, perturbed_field, phonon_field
    s = FermionSolver.from_params(p, max_rhs=1)
    x0 = torch.from_numpy(phonon_field(p)).to(dev)
    x = torch.from_numpy(perturbed_field(p, phonon_field(p))).to(dev)
    s.set_field(x0)
    Phi = s.matvec(torch.from_numpy(gaussian_rhs(p, 1)).to(dev), "MT")
    out = []
    for _ in range(2):
        s.set_field(x, a1=a1, a2=a2)
        u, st = s.solve(Phi, tol=1e-8, prec="f32_refined", precond=True)
        s.action(Phi, u)
        s.force(u)
        torch.cuda.synchronize()
        out.append({"iters": st[0]["iters"], "status": st[0]["status"],
                    "rel_resid": st[0]["rel_resid"]})
    print(json.dumps({"workload": p.name, "steps": out}), flush=True)
    s.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: --gpus must be 1 (see the sharding notes for several GPUs)"}))
        sys.exit(2)
    import numpy as np
    import torch

    if args.profile_roofline:
        profile_roofline(torch, torch.device("cuda:0"))
        return
    if args.profile_step:
        from workloads import get_config as _gc
        profile_step(torch, torch.device("cuda:0"), _gc(args.workload), args.a1, args.a2)
        return
    if args.meas_only:
        from workloads import get_config as _gc
        print(json.dumps(bench_measure(torch, torch.device("cuda:0"), _gc(args.workload), args.a1, args.a2,
                                       args.nrv, log)), flush=True)
        return
    if args.ssh_only:
        from workloads import get_config as _gc
        print(json.dumps(bench_ssh(torch, torch.device("cuda:0"), _gc(args.workload), args.ssh_g, args.a1,
                                   args.a2, log, hmc=args.ssh_hmc)),
              flush=True)
        return
    if args.hmc_only:
        from workloads import get_config as _gc
        print(json.dumps(bench_hmc(torch, torch.device("cuda:0"), _gc(args.workload), args.a1, args.a2,
                                   log)), flush=True)
        return

    from paper_2203_01291_amd.solver import FermionSolver
    from workloads import gaussian_rhs, get_config, perturbed_field, phonon_field

    dev = torch.device("cuda:0")
    p = get_config(args.workload)
    R = args.nrhs
    s = FermionSolver.from_params(p, max_rhs=max(R, 1))
    x0 = torch.from_numpy(phonon_field(p)).to(dev)
    x = torch.from_numpy(perturbed_field(p, phonon_field(p))).to(dev)
    phi = torch.from_numpy(gaussian_rhs(p, R)).to(dev)
    s.set_field(x0)
    Phi = s.matvec(phi, "MT")          # Phi = M(x0)^T phi
    torch.cuda.synchronize()
    tol = 1e-8
    last = {}

    def make_step(prec, pre, variant=0, a1=args.a1, a2=args.a2):
        def step():
            s.set_field(x, a1=a1, a2=a2)                     # setup
            u, st = s.solve(Phi, tol=tol, prec=prec, precond=pre, variant=variant)   # PCG
            S = s.action(Phi, u)                             # S_F
            g = s.force(u)                                   # dS_F/dx
            last["st"], last["S"], last["g"], last["u"] = st, S, g, u
            return st
        return step

    # One step of each solver variant: FP32-refined and FP64, with and
    # without the preconditioner (Chebyshev coefficients a1 as chosen, and
    # a1 = a2 = 1), the one-launch FP32 solve.
    variants = {}
    all_variants = (("f32_refined_plain", "f32_refined", False, 0, args.a1),
                    ("f32_refined_precond", "f32_refined", True, 0, args.a1),
                    ("f32_refined_precond_a1_a2_1", "f32_refined", True, 0, 1.0),
                    ("f64_plain", "f64", False, 0, args.a1),
                    ("f32_refined_plain_one_launch", "f32_refined", False, 2, args.a1),
                    ("f64_precond", "f64", True, 0, args.a1))
    for name, prec, pre_v, var, a1v in (() if args.no_variants else all_variants):
        if var == 2 and R != 1:
            continue
        t, st = time_steps(make_step(prec, pre_v, var, a1=a1v, a2=1.0 if a1v == 1.0 else args.a2),
                           1, 0, torch)
        variants[name] = {"ms": t * 1e3, "iters": st[0]["iters"], "status": st[0]["status"],
                          "rel_resid": st[0]["rel_resid"]}
        log(f"variant {name}: {t * 1e3:.1f} ms, {st[0]['iters']} iterations, status {st[0]['status']}")
    # The paper's action sums over two pseudofermion fields (spin up and
    # down) sharing one phonon field: both solves in one call (two
    # right-hand sides), action and force of both.
    two_fields = None
    if not args.no_variants and R == 1:
        s2 = FermionSolver.from_params(p, max_rhs=2)
        s2.set_field(x0)
        Phi2 = s2.matvec(torch.from_numpy(gaussian_rhs(p, 2)).to(dev), "MT")

        def step2():
            s2.set_field(x, a1=args.a1, a2=args.a2)
            u2, st = s2.solve(Phi2, tol=tol, prec="f32_refined", precond=True)
            s2.action(Phi2, u2)
            s2.force(u2, scale=0.5)
            return st
        t2, st2 = time_steps(step2, 1, 1, torch)
        two_fields = {"ms_per_step": t2 * 1e3, "solves_per_s": 2 / t2,
                      "iters": [v["iters"] for v in st2], "status": [v["status"] for v in st2]}
        log(f"two fields: {two_fields}")
        s2.close()
    # Several independent systems of the workload's shape in the same launches
    # (per-right-hand-side fields, fph_set_fields): K fields x0 + 0.01 k with
    # Phi_k = M(x0 + 0.01 k)^T phi, solved at x + 0.01 k; one step = set the
    # K fields + FP32-refined PCG of the K systems + their actions and forces.
    multi = None
    if not args.no_variants and R == 1:
        multi = {}
        for K in (4, 8):
            sm = FermionSolver.from_params(p, max_rhs=K)
            x0s = torch.stack([x0 + 0.01 * k for k in range(K)]).contiguous()
            xs = torch.stack([x + 0.01 * k for k in range(K)]).contiguous()
            sm.set_fields(x0s)
            PhiK = sm.matvec(phi.expand(K, -1, -1).contiguous(), "MT")

            def stepm():
                sm.set_fields(xs, 1, a1=args.a1, a2=args.a2)
                uK, stK = sm.solve(PhiK, tol=tol, prec="f32_refined", precond=True)
                sm.action(PhiK, uK)
                sm.force(uK)
                return stK
            tm, stm = time_steps(stepm, 2, 1, torch)
            multi[f"fields_{K}"] = {"ms_per_step": tm * 1e3, "solves_per_s": K / tm,
                                   "iters": [v["iters"] for v in stm], "status": [v["status"] for v in stm]}
            log(f"multi-field K={K}: {multi[f'fields_{K}']}")
            sm.close()
    if args.precond < 0 and variants:
        pre = variants["f32_refined_precond"]["ms"] < variants["f32_refined_plain"]["ms"]
    else:
        pre = args.precond > 0

    t32, st32 = time_steps(make_step("f32_refined", pre), args.steps, args.warmup, torch)
    st32 = [dict(v) for v in st32]
    S32 = last["S"].cpu().numpy().tolist()
    # Error of the timed step's solution and force against the oracle's
    # stored values (its FP64 CG to relative residual 1e-13, same inputs).
    err = None
    if R == 1:
        err = error_vs_golden(args.workload, last["u"], last["g"], S32[0], tol)
        log(f"error vs oracle: {err}")
    log(f"f32_refined: {t32 * 1e3:.2f} ms/step {st32}")
    t64, st64 = time_steps(make_step("f64", pre), max(1, args.steps // 2), min(args.warmup, 1), torch)
    st64 = [dict(v) for v in st64]
    S64 = last["S"].cpu().numpy().tolist()
    log(f"f64: {t64 * 1e3:.2f} ms/step {st64}")

    # The same step at a solve tolerance whose error against the oracle is
    # below 1e-8 (1e-11; the rigorous bound kappa * tol would need ~4e-15,
    # below what an FP64 residual resolves), and the L = 64 workload at both
    # tolerances; the step captured as a graph with the enqueue-only solve.
    accuracy = c5 = graph_step = None
    if not args.no_variants and R == 1:
        accuracy = bench_workload_tols(torch, dev, args.workload, (1e-11,), 2, log)
        c5 = bench_workload_tols(torch, dev, "c5", (1e-8, 1e-11), 3, log)
        graph_step = bench_graph_step(torch, dev, p, args.a1, args.a2, log)

    # M^T M apply at the workload shape: the bandwidth-bound kernel of the path.
    d = p.dim
    v32 = torch.randn(R, p.Ltau, p.N, device=dev, dtype=torch.float32)
    v64 = v32.double()
    s.set_field(x)
    tm32 = event_time_matvec(s, v32, "MTM", args.matvec_reps, torch)
    tm64 = event_time_matvec(s, v64, "MTM", args.matvec_reps, torch)
    bytes32 = (2 * R + 1) * d * 4
    bytes64 = (2 * R + 1) * d * 8
    gbs32 = bytes32 / tm32 / 1e9
    gbs64 = bytes64 / tm64 / 1e9
    log(f"MTM fp32 {tm32 * 1e6:.2f} us {gbs32:.0f} GB/s; fp64 {tm64 * 1e6:.2f} us {gbs64:.0f} GB/s")

    large = None
    if not args.no_large:
        # Same kernel on working sets above 4 x the 256 MB Infinity Cache:
        # FP32 with ROOF_R32 right-hand sides, FP64 with ROOF_R64.
        p5, R5, s5, vl = large_matvec_setup(torch, dev)
        vl64 = vl[:ROOF_R64].contiguous()
        tl64 = event_time_matvec(s5, vl64, "MTM", 20, torch)
        del vl64
        vl32 = vl.float()
        del vl
        tl32 = event_time_matvec(s5, vl32, "MTM", 20, torch)
        tl32_iso = event_time_matvec(s5, vl32, "MTM", 20, torch, isolated=True)
        bl64 = (2 * ROOF_R64 + 1) * p5.dim * 8
        bl32 = (2 * R5 + 1) * p5.dim * 4
        ceil = hbm_ceilings(torch, dev, bl64)
        large = {
            "workload": f"{p5.name}: {R5} rhs (FP32), {ROOF_R64} rhs (FP64) sharing one field",
            "copy_ceilings": ceil,
            "working_set_MB": {"f64": bl64 / 1e6, "f32": bl32 / 1e6},
            "mall_MB": 256, "working_set_over_mall": {"f64": bl64 / 256e6, "f32": bl32 / 256e6},
            "f64": {"us": tl64 * 1e6, "GB/s": bl64 / tl64 / 1e9, "frac": bl64 / tl64 / 1e9 / HBM_PEAK_GBS},
            "f32": {"us": tl32 * 1e6, "GB/s": bl32 / tl32 / 1e9, "frac": bl32 / tl32 / 1e9 / HBM_PEAK_GBS,
                    "isolated_launch_us": tl32_iso * 1e6},
        }
        log(f"large: {large}")
        s5.close()
        del vl32

    batch = None
    if not args.no_batch:
        batch = bench_batched(torch, dev, log)

    hmc = None
    if not args.no_hmc and R == 1:
        hmc = bench_hmc(torch, dev, p, args.a1, args.a2, log)

    meas = None
    if not args.no_meas and R == 1:
        meas = bench_measure(torch, dev, p, args.a1, args.a2, args.nrv, log)

    ssh = None
    if not args.no_ssh and R == 1:
        ssh = bench_ssh(torch, dev, p, args.ssh_g, args.a1, args.a2, log)

    cpu = None
    if not args.no_cpu_baseline:
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_iterations.json")))
        cpu = cpu_baseline(p, gold[args.workload]["iters_tol_1e-8"])
        log(f"cpu baseline: {cpu}")

    if large is not None:
        valid = TRAFFIC is not None and TRAFFIC["source_sha1"] == kernel_sources_sha1()
        roofline = {"bound": "hbm", "achieved": large["f64"]["GB/s"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": large["f64"]["frac"],
                    "traffic": TRAFFIC["f64_bytes_per_launch"] if valid else None,
                    "kernel": "fused M^T M apply, FP64 (k_mtm<double, 1024, 1, InPlain, EpiStream>)",
                    "workload": f"holstein_L64_Ltau400 x {ROOF_R64} rhs sharing one field "
                                f"({large['working_set_over_mall']['f64']:.2f} x the 256 MB Infinity Cache)",
                    "bytes_per_launch": large["working_set_MB"]["f64"] * 1e6,
                    "avg_launch_us": large["f64"]["us"],
                    "f32": {"kernel": "k_mtm<float, 1024, 1, InPlain, EpiStream>",
                            "workload": f"holstein_L64_Ltau400 x {ROOF_R32} rhs sharing one field "
                                        f"({large['working_set_over_mall']['f32']:.2f} x the MALL)",
                            "achieved": large["f32"]["GB/s"], "frac": large["f32"]["frac"],
                            "bytes_per_launch": large["working_set_MB"]["f32"] * 1e6,
                            "avg_launch_us": large["f32"]["us"],
                            "traffic": TRAFFIC["f32_bytes_per_launch"] if valid else None},
                    "ceilings": {k: v["frac"] for k, v in large["copy_ceilings"].items() if k != "bytes"},
                    "frac_of_window_copy": large["f64"]["frac"] / large["copy_ceilings"]["window_copy"]["frac"],
                    "profile": TRAFFIC["profile"] if TRAFFIC else None}
    else:
        roofline = {"bound": "hbm", "achieved": gbs32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs32 / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "fused M^T M apply, FP32 (k_mtm<float, 256, 1, InPlain, EpiStore>)",
                    "workload": p.name, "bytes_per_launch": bytes32, "avg_launch_us": tm32 * 1e6}

    value = R / t32
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{p.name}: L={p.L} N={p.N} Ltau={p.Ltau} d={p.dim} dtau={p.dtau} "
                        f"mu={p.mu} alpha={p.alpha}; FP32-refined PCG to 1e-8 + S_F + force",
            "nrhs": R,
            "precond": pre,
            "chebyshev_a1_a2": [args.a1, args.a2] if pre else None,
            "iters": [v["iters"] for v in st32],
            "fp64_refreshes": [v["outer_iters"] for v in st32],
            "rel_resid": [v["rel_resid"] for v in st32],
        },
        "error_vs_oracle": err,
        "accuracy_1e-8_error": accuracy,
        "c5": c5,
        "graph_step": graph_step,
        "fp64_cg": {"solves_per_s": R / t64, "ms_per_step": t64 * 1e3,
                    "iters": [v["iters"] for v in st64],
                    "speedup_fp32_refined": t64 / t32,
                    "action_rel_diff": float(np.max(np.abs(np.array(S32) - np.array(S64)) / np.abs(np.array(S64))))},
        "roofline": roofline,
        "matvec_workload": {
            "note": "single system at the workload shape: cache resident, latency bound",
            "f32": {"GB/s": gbs32, "frac": gbs32 / HBM_PEAK_GBS, "avg_launch_us": tm32 * 1e6,
                    "bytes_per_launch": bytes32},
            "f64": {"GB/s": gbs64, "frac": gbs64 / HBM_PEAK_GBS, "avg_launch_us": tm64 * 1e6,
                    "bytes_per_launch": bytes64}},
        "matvec_large": large,
        "batched": batch,
        "variants": variants,
        "two_fields": two_fields,
        "multi_field": multi,
        "hmc_trajectory": hmc,
        "measurements": meas,
        "ssh": ssh,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
