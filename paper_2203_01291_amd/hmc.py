"""Python binding of the hybrid Monte Carlo update (Sec. III, Algorithm 1).

Argument marshalling only: every step runs in the HIP library; tensors give
device pointers and the current torch stream gives the hipStream_t.
"""

import ctypes
import math

import torch

from . import _lib
from ._lib import (FPH_LAMBDA, FPH_LAMBDA_INV, FPH_LAMBDA_INV_T, FPH_LAMBDA_T, FPH_MASS, FPH_MASS_INV,
                   FPH_MASS_SQRT, FPH_MOVE_REFLECT, FPH_MOVE_SWAP, HmcOpts, HmcStats, PcgOpts, UpdateStats,
                   check)
from .solver import _PRECS, _ptr, _stream

_MASS_OPS = {"inv": FPH_MASS_INV, "sqrt": FPH_MASS_SQRT, "mass": FPH_MASS}
_GUESS = {"zero": 0, "previous": 1, "extrapolate": 2}
_LAMBDA_OPS = {"L": FPH_LAMBDA, "Linv": FPH_LAMBDA_INV, "LT": FPH_LAMBDA_T, "LinvT": FPH_LAMBDA_INV_T}
_MOVES = {"reflect": FPH_MOVE_REFLECT, "swap": FPH_MOVE_SWAP}


def _pcg_opts(tol, precond=True, prec="f32_refined", maxiter=100000, ru_delta=0.0):
    return PcgOpts(float(tol), int(maxiter), int(bool(precond)), _PRECS[prec], 1, float(ru_delta), 0, 0)


class PhononHMC:
    """HMC and global updates of the phonon field of one ``FermionSolver`` or
    ``SSHSolver`` (which must outlive this object; with an SSHSolver prec is
    "f64" or "f32_refined" as well).  m_reg=None disables Fourier
    acceleration; lambda_action=True samples the action with A = M Lambda,
    False the action S' with A = M."""

    def __init__(self, solver, omega0, m_reg, dt, Nt=100, nt=10, nfields=2, a1=1.0, a2=1.0,
                 force_tol=1e-5, action_tol=1e-10, precond=True, prec="f32_refined",
                 maxiter=100000, guess="zero", lambda_action=False, nchains=1):
        self.lib = _lib.load()
        self.solver = solver
        self.nfields = int(nfields)
        self.nchains = int(nchains)
        mr = math.inf if m_reg is None else float(m_reg)
        self.opts = HmcOpts(float(omega0), mr, float(dt), int(Nt), int(nt), self.nfields, float(a1),
                            float(a2), _GUESS[guess], int(bool(lambda_action)), self.nchains, 0,
                            _pcg_opts(force_tol, precond, prec, maxiter),
                            _pcg_opts(action_tol, precond, prec, maxiter))
        h = ctypes.c_void_p()
        from .ssh import SSHSolver
        create = self.lib.fph_hmc_create_ssh if isinstance(solver, SSHSolver) else self.lib.fph_hmc_create
        check(create(ctypes.byref(h), solver.h, ctypes.byref(self.opts), _stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.fph_hmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _v(self, t, n=1):
        if t.numel() != n * self.solver.dim:
            raise ValueError(f"expected {n} vector(s) of N*Ltau values")
        self.solver._vec(t)
        return t

    def bosonic_action(self, x):
        """Tensor [S_B(x), -dtau*alpha*sum x] (FP64, on the device)."""
        out = torch.empty(2, dtype=torch.float64, device=x.device)
        check(self.lib.bosonic_action(self.h, _ptr(self._v(x)), _ptr(out), _stream()))
        return out

    def bosonic_force(self, x, grad=None, scale=1.0):
        """grad += scale * (dS_B/dx - dtau*alpha)."""
        grad = torch.zeros_like(x) if grad is None else grad
        check(self.lib.bosonic_force(self.h, _ptr(self._v(x)), _ptr(self._v(grad)), float(scale),
                                     _stream()))
        return grad

    def mass_apply(self, v, op="inv"):
        """Mass^{-1} v, sqrt(Mass) v or Mass v for one or more vectors [..., Ltau, N]."""
        n = self.solver._vec(v)
        out = torch.empty_like(v)
        check(self.lib.hmc_mass_apply(self.h, _MASS_OPS[op], n, _ptr(v), _ptr(out), _stream()))
        return out

    def boson_steps(self, x, p):
        """The nt bosonic sub-steps of one time step, in place on x and p."""
        check(self.lib.hmc_boson_steps(self.h, _ptr(self._v(x)), _ptr(self._v(p)), _stream()))
        return x, p

    def trajectory(self, x, R_fields, R_mom, r_uniform, p_out=None):
        """One HMC trial update of x (in place if accepted).  Returns the stats dict."""
        self._v(x)
        self._v(R_fields, self.nfields)
        self._v(R_mom)
        st = HmcStats()
        pp = _ptr(p_out) if p_out is not None else None
        check(self.lib.hmc_trajectory(self.h, _ptr(x), _ptr(R_fields), _ptr(R_mom), float(r_uniform),
                                      pp, ctypes.byref(st), _stream()))
        return st.as_dict()

    def trajectories(self, x, R_fields, R_mom, r_uniform, p_out=None):
        """One HMC update of each of the nchains chains at once: x [nchains, Ltau, N] (accepted
        chains updated in place), R_fields [nchains, nfields, Ltau, N], R_mom [nchains, Ltau, N],
        r_uniform a sequence of nchains draws.  Returns one stats dict per chain."""
        K = self.nchains
        self._v(x, K)
        self._v(R_fields, K * self.nfields)
        self._v(R_mom, K)
        r_uniform = [float(v) for v in r_uniform]
        if len(r_uniform) != K:
            raise ValueError(f"expected {K} uniform draws")
        rs = (ctypes.c_double * K)(*r_uniform)
        st = (HmcStats * K)()
        pp = _ptr(p_out) if p_out is not None else None
        check(self.lib.hmc_trajectories(self.h, _ptr(x), _ptr(R_fields), _ptr(R_mom), rs, pp, st,
                                        _stream()))
        return [v.as_dict() for v in st]

    def lambda_apply(self, x, v, op="LinvT"):
        """Lambda(x) v, Lambda^{-1} v, Lambda^T v or Lambda^{-T} v (op 'L', 'Linv', 'LT', 'LinvT')."""
        n = self.solver._vec(v)
        self._v(x)
        out = torch.empty_like(v)
        check(self.lib.lambda_apply(self.h, _LAMBDA_OPS[op], _ptr(x), n, _ptr(v), _ptr(out), _stream()))
        return out

    def lambda_force(self, b, u, grad, scale=1.0):
        """grad += scale * (-dtau alpha) * shift_tau(sum_r b_r * u_r)."""
        n = self.solver._vec(b)
        check(self.lib.lambda_force(self.h, n, _ptr(b), _ptr(u), _ptr(self._v(grad)), float(scale),
                                    _stream()))
        return grad

    def global_update(self, x, kind, i, j, R_fields, r_uniform):
        """One reflection ('reflect', site i) or swap ('swap', sites i, j) Metropolis update of
        x (in place if accepted).  Returns the stats dict."""
        self._v(x)
        self._v(R_fields, self.nfields)
        st = UpdateStats()
        check(self.lib.hmc_global_update(self.h, _MOVES[kind], int(i), int(j), _ptr(x), _ptr(R_fields),
                                         float(r_uniform), ctypes.byref(st), _stream()))
        return st.as_dict()
