"""Write the oracle's reference values for the full-size workloads.

Calls only ``oracle/`` and ``workloads/`` (never the HIP path).  For each
workload it solves (M^T M) u = Phi with the oracle's textbook FP64 CG on
the CSR matrix to a tight tolerance and stores, as small JSON fixtures:

* the iteration counts at which the oracle's CG first reached relative
  residuals 1e-8 and 1e-10 (used to scale the CPU baseline);
* S_F = Phi . u, |u|, and u at sampled components;
* the force dS_F/dx (Eq. dSF_dx) at the same sampled components;
* the final relative residual and a Lanczos estimate of kappa(M^T M).

The field is x = x0 + 0.1 N(0,1) and Phi = M(x0)^T phi (workloads.inputs).

Usage: python tests/golden/make_golden.py c3 [c5 ...]
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import force as OF  # noqa: E402
from oracle import lattice as OL  # noqa: E402
from oracle import solve as OS  # noqa: E402
from workloads import (fd_sample_indices, gaussian_rhs, get_config,  # noqa: E402
                       perturbed_field, phonon_field)


def run(key, tol=1e-13, nsample=100):
    p = get_config(key)
    lat = OL.Lattice.from_params(p)
    x0 = phonon_field(p)
    x = perturbed_field(p, x0)
    Cs = OL.sparse_C(lat)
    phi = gaussian_rhs(p, 1)[0]
    Phi = (OL.sparse_M(lat, x0, Cs).T @ phi.reshape(-1)).reshape(lat.Ltau, lat.N)
    mv = OS.normal_matvec_sparse(lat, x, Cs)
    t0 = time.time()
    u, it, hist = OS.cg(mv, Phi, tol=tol, maxiter=400000)
    dt = time.time() - t0
    hist = np.array(hist)
    first = lambda eps: int(np.argmax(hist < eps)) if np.any(hist < eps) else None  # noqa: E731
    res = OS.relative_residual(mv, Phi, u)
    # force at sampled components from the oracle's own solution
    Mu = (OL.sparse_M(lat, x, Cs) @ u.reshape(-1)).reshape(lat.Ltau, lat.N)
    E = OL.E_field(lat, x)
    comps = fd_sample_indices(p, nsample)
    g = []
    for tau, i in comps:
        prev = u[tau - 1] if tau >= 1 else -u[lat.Ltau - 1]
        y = E[tau, i] * float((Cs[i] @ prev).item())
        g.append(float(-2.0 * lat.dtau * lat.alpha * Mu[tau, i] * y))
    # cross-check the sampled formula against the full-vector oracle force on a few slices
    full_g = OF.force_from_solution(lat, x, u[None], Cs.toarray() if lat.N <= 1024 else None)[0] \
        if lat.N <= 1024 else None
    if full_g is not None:
        scale = float(np.max(np.abs(full_g)))
        for (tau, i), gv in zip(comps, g):
            assert abs(full_g[tau, i] - gv) <= 1e-11 * scale
    kappa = OS.lanczos_condition_estimate(mv, Phi, iters=min(it, 2000))
    return {
        "workload": p.name,
        "field": "x = phonon_field + 0.1 N(0,1) (workloads.perturbed_field); Phi = M(x0)^T phi",
        "iters_tol_1e-8": first(1e-8),
        "iters_tol_1e-10": first(1e-10),
        "iters_total": it,
        "final_rel_resid": res,
        "kappa_lanczos": kappa,
        "S_F": float(np.sum(Phi * u)),
        "u_norm": float(np.linalg.norm(u)),
        "samples": [[int(tau), int(i)] for tau, i in comps],
        "u_samples": [float(u[tau, i]) for tau, i in comps],
        "force_samples": g,
        "oracle_seconds": dt,
    }


def main(keys):
    for key in keys:
        print(f"solving {key} ...", flush=True)
        rec = run(key)
        print(json.dumps({k: v for k, v in rec.items() if not k.endswith("samples")}), flush=True)
        json.dump(rec, open(os.path.join(HERE, f"oracle_{key}.json"), "w"), indent=1)
    its = {}
    for key in sorted(["c1", "c2", "c3", "c4", "c5"]):
        f = os.path.join(HERE, f"oracle_{key}.json")
        if os.path.exists(f):
            v = json.load(open(f))
            its[key] = {"iters_tol_1e-8": v["iters_tol_1e-8"], "iters_tol_1e-10": v["iters_tol_1e-10"]}
    json.dump(its, open(os.path.join(HERE, "oracle_iterations.json"), "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3"])
