"""Python binding of the SSH-type coupling (x in the bond hoppings).

The paper (Sec. II C, closing remark; Sec. III A) only names the SSH model:
its phonon coordinates enter the hopping matrix, and the force follows by
the product rule through the checkerboard factors.  The library reads the
coupling as t_b(x_tau) = t - g (x_{j,tau} - x_{i,tau}) on bond b = (i, j = i + x^
or i + y^), keeps the Holstein on-site factor exp(-dtau (alpha x - mu)) and the
four bond families of the checkerboard (F_xe F_ye F_xo F_yo); g = 0 is the
Holstein matrix.  Argument marshalling only: every step runs in the HIP
library; tensors give device pointers and the current torch stream the
hipStream_t.  FP64 only.  ``solver.fermion_action(x, Phi, ssh_solver)`` gives
a differentiable S_F on this operator (its gradient is ``force``).
"""

import ctypes

import torch

from . import _lib
from ._lib import FPH_OP_M, FPH_OP_MT, FPH_OP_MTM, Lattice, PcgOpts, PcgStats, check
from .solver import _ptr, _scale_ptr, _stream

_OPS = {"M": FPH_OP_M, "MT": FPH_OP_MT, "MTM": FPH_OP_MTM}


class SSHSolver:
    """One lattice, SSH coupling g and up to ``max_rhs`` right-hand sides."""

    def __init__(self, L, Ltau, dtau, t, mu, alpha, g, max_rhs=1):
        self.lib = _lib.load()
        self.L, self.Ltau = int(L), int(Ltau)
        self.N = self.L * self.L
        self.dim = self.N * self.Ltau
        self.g = float(g)
        self.max_rhs = int(max_rhs)
        lat = Lattice(self.L, self.Ltau, float(dtau), float(t), float(mu), float(alpha))
        h = ctypes.c_void_p()
        check(self.lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(lat), self.g, self.max_rhs))
        self.h = h
        self._pc = None
        self._field = None
        self.field_version = 0

    @classmethod
    def from_params(cls, p, g, L=None, max_rhs=1):
        return cls(p.L if L is None else L, p.Ltau, p.dtau, p.t, p.mu, p.alpha, g, max_rhs=max_rhs)

    def close(self):
        if getattr(self, "h", None):
            self.lib.fph_ssh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, v):
        if not (v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()):
            raise ValueError("expected a contiguous float64 CUDA tensor")
        if v.numel() % self.dim:
            raise ValueError(f"size {v.numel()} is not a multiple of N*Ltau = {self.dim}")
        return v.numel() // self.dim

    def attach_preconditioner(self, fermion_solver, a1=1.0, a2=1.0):
        """Precondition solves with the adiabatic preconditioner of a FermionSolver of the
        same lattice (uniform hopping, on-site factor of the field); set_field then sets
        that solver's field too (in the library), with Chebyshev-order constants a1, a2.
        None detaches."""
        h = fermion_solver.h if fermion_solver is not None else None
        check(self.lib.ssh_set_preconditioner(self.h, h, float(a1), float(a2)))
        self._pc = fermion_solver  # kept alive while attached

    def set_field(self, x):
        if self._vec(x) != 1:
            raise ValueError("expected one field of N*Ltau values")
        check(self.lib.ssh_set_field(self.h, _ptr(x), _stream()))
        self._field = x
        self.field_version += 1

    def field_state(self):
        return self._field

    def restore_field(self, state):
        if state is not None:
            self.set_field(state)

    def matvec(self, v, op="M", out=None):
        """M v, M^T v or M^T M v for every vector of v."""
        nrhs = self._vec(v)
        out = torch.empty_like(v) if out is None else out
        check(self.lib.ssh_matvec(self.h, _OPS[op], nrhs, _ptr(v), _ptr(out), _stream()))
        return out

    def solve(self, b, u=None, tol=1e-10, maxiter=100000, chunk=0, precond=False, prec="f64",
              ru_delta=0.0, max_outer=0):
        """(P)CG on (M^T M) u = b (precond: the attached preconditioner), FP64
        or FP32-refined (prec="f32_refined": FP32 iterations with FP64
        residual replacement).  Returns (u, [stats dict per rhs]).  Blocks
        until done."""
        from .solver import _PRECS
        nrhs = self._vec(b)
        zero = u is None
        u = torch.empty_like(b) if u is None else u
        opts = PcgOpts(float(tol), int(maxiter), int(bool(precond)), _PRECS[prec], int(zero), float(ru_delta),
                       int(chunk), 0, int(max_outer))
        stats = (PcgStats * nrhs)()
        check(self.lib.ssh_solve(self.h, nrhs, _ptr(b), _ptr(u), ctypes.byref(opts), stats, _stream()))
        return u, [s.as_dict() for s in stats]

    def action(self, b, u):
        """S_F = b . u per right-hand side, FP64 on the device."""
        nrhs = self._vec(b)
        out = torch.empty(nrhs, dtype=torch.float64, device=b.device)
        check(self.lib.ssh_action(self.h, nrhs, _ptr(b), _ptr(u), _ptr(out), _stream()))
        return out

    def force(self, u, grad=None, scale=1.0, scale_dev=None):
        """grad += scale * s * sum_r dS_F/dx for solutions u (S_F = b . (M^T M)^{-1} b);
        s = scale_dev (one-element float64 CUDA tensor, read on the device) or 1."""
        nrhs = self._vec(u)
        grad = torch.zeros(self.Ltau, self.N, dtype=torch.float64, device=u.device) if grad is None else grad
        if self._vec(grad) != 1:
            raise ValueError("grad must hold one field")
        check(self.lib.ssh_force(self.h, nrhs, _ptr(u), _ptr(grad), float(scale), _scale_ptr(scale_dev),
                                 _stream()))
        return grad
