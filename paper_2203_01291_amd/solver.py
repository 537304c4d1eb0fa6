"""Python binding of the gfx950 Holstein fermion solver.

Argument marshalling only: tensors provide device pointers and the current
torch stream provides the hipStream_t; every step of the computation runs
in the HIP library (``lib/libholstein_hmc.so``).
"""

import ctypes

import torch

from . import _lib
from ._lib import (FPH_F32, FPH_F32_REFINED, FPH_F64, FPH_OP_M, FPH_OP_MT, FPH_OP_MTM,
                   FPH_PC_F, FPH_PC_FFT, FPH_PC_FT, Lattice, PcgOpts, PcgStats, System, check,
                   stats_from_device)

_OPS = {"M": FPH_OP_M, "MT": FPH_OP_MT, "MTM": FPH_OP_MTM}
_PC_OPS = {"F": FPH_PC_F, "FT": FPH_PC_FT, "FFT": FPH_PC_FFT}
_PRECS = {"f64": FPH_F64, "f32_refined": FPH_F32_REFINED}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _scale_ptr(scale_dev):
    """Device pointer of a one-element float64 CUDA tensor, or NULL."""
    if scale_dev is None:
        return ctypes.c_void_p(None)
    if not (scale_dev.is_cuda and scale_dev.dtype == torch.float64 and scale_dev.numel() == 1
            and scale_dev.is_contiguous()):
        raise ValueError("scale_dev must be a one-element contiguous float64 CUDA tensor")
    return _ptr(scale_dev)


class FermionSolver:
    """One lattice (L, Ltau, dtau, t, mu, alpha) and up to ``max_rhs``
    right-hand sides; owns the library handle and its workspace."""

    def __init__(self, L, Ltau, dtau, t, mu, alpha, max_rhs=1):
        self.lib = _lib.load()
        self.L, self.Ltau = int(L), int(Ltau)
        self.N = self.L * self.L
        self.dim = self.N * self.Ltau
        self.params = dict(L=L, Ltau=Ltau, dtau=dtau, t=t, mu=mu, alpha=alpha)
        self.max_rhs = int(max_rhs)
        lat = Lattice(self.L, self.Ltau, float(dtau), float(t), float(mu), float(alpha))
        h = ctypes.c_void_p()
        check(self.lib.fph_create(ctypes.byref(h), ctypes.byref(lat), self.max_rhs))
        self.h = h
        self._x = None
        self._field = None
        self.field_version = 0

    @classmethod
    def from_params(cls, p, L=None, max_rhs=1):
        return cls(p.L if L is None else L, p.Ltau, p.dtau, p.t, p.mu, p.alpha, max_rhs=max_rhs)

    def close(self):
        if getattr(self, "h", None):
            self.lib.fph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- checks
    def _vec(self, v, dtype=torch.float64):
        if not (v.is_cuda and v.dtype == dtype and v.is_contiguous()):
            raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
        if v.numel() % self.dim:
            raise ValueError(f"size {v.numel()} is not a multiple of N*Ltau = {self.dim}")
        return v.numel() // self.dim

    # ---------------------------------------------------------------- API
    def set_field(self, x, a1=1.0, a2=1.0):
        """E = exp(-dtau V(x)), dbar, spectral bounds and Chebyshev tables."""
        if self._vec(x) != 1:
            raise ValueError("x must hold exactly N*Ltau values")
        self._x = x
        self._nfields = 0
        check(self.lib.fph_set_field(self.h, _ptr(x), float(a1), float(a2), _stream()))
        self._field = ("one", x, dict(a1=a1, a2=a2))
        self.field_version += 1

    def set_fields(self, xs, rhs_per_field=1, a1=1.0, a2=1.0):
        """Per-right-hand-side fields: xs [nfields, Ltau, N]; right-hand side r of later calls
        uses field r // rhs_per_field.  force() then returns one gradient per field."""
        nf = self._vec(xs)
        self._x = xs
        self._nfields = nf
        check(self.lib.fph_set_fields(self.h, nf, int(rhs_per_field), _ptr(xs), float(a1), float(a2),
                                      _stream()))
        self._field = ("many", xs, dict(rhs_per_field=rhs_per_field, a1=a1, a2=a2))
        self.field_version += 1

    def field_state(self):
        """What the last set_field / set_fields call installed (see restore_field)."""
        return self._field

    def restore_field(self, state):
        """Install again a field recorded by field_state (no-op for None)."""
        if state is None:
            return
        kind, x, kw = state
        if kind == "one":
            self.set_field(x, **kw)
        else:
            self.set_fields(x, **kw)

    def matvec(self, v, op="MTM", out=None):
        """out = op(v) for op in {'M', 'MT', 'MTM'}; float64 or float32."""
        prec = FPH_F64 if v.dtype == torch.float64 else FPH_F32
        nrhs = self._vec(v, v.dtype)
        out = torch.empty_like(v) if out is None else out
        check(self.lib.fermion_matvec(self.h, _OPS[op], prec, nrhs, _ptr(v), _ptr(out), _stream()))
        return out

    def precond(self, v, op="FFT", out=None):
        """out = F v, F^T v or F F^T v (adiabatic preconditioner)."""
        prec = FPH_F64 if v.dtype == torch.float64 else FPH_F32
        nrhs = self._vec(v, v.dtype)
        out = torch.empty_like(v) if out is None else out
        check(self.lib.fph_precond_apply(self.h, _PC_OPS[op], prec, nrhs, _ptr(v), _ptr(out),
                                         _stream()))
        return out

    def precond_info(self):
        b = (ctypes.c_double * 2)()
        npt = (ctypes.c_int32 * self.Ltau)()
        check(self.lib.fph_precond_info(self.h, b, npt, _stream()))
        return (b[0], b[1]), list(npt)

    def _opts(self, zero, tol, maxiter, precond, prec, ru_delta, chunk, variant, max_outer):
        return PcgOpts(float(tol), int(maxiter), int(bool(precond)), _PRECS[prec], int(zero),
                       float(ru_delta), int(chunk), int(variant), int(max_outer), 0)

    def solve(self, b, u=None, tol=1e-10, maxiter=100000, precond=False, prec="f64",
              ru_delta=0.0, chunk=0, variant=0, max_outer=0):
        """Solve (M^T M) u = b for every right-hand side of b (float64).
        Returns (u, [stats dict per rhs]).  Blocks until done (pcg_solve_sync:
        the slots are enqueued in chunks until the device reports every
        right-hand side finished)."""
        nrhs = self._vec(b)
        if nrhs > self.max_rhs:
            raise ValueError("more right-hand sides than max_rhs")
        zero = u is None
        u = torch.empty_like(b) if u is None else u
        opts = self._opts(zero, tol, maxiter, precond, prec, ru_delta, chunk, variant, max_outer)
        stats = (PcgStats * nrhs)()
        check(self.lib.pcg_solve_sync(self.h, nrhs, _ptr(b), _ptr(u), ctypes.byref(opts), stats,
                                      _stream()))
        return u, [s.as_dict() for s in stats]

    def solve_async(self, b, u=None, stats=None, tol=1e-10, maxiter=2000, precond=False,
                    prec="f64", ru_delta=0.0, variant=0, max_outer=0, zero_guess=None):
        """Enqueue the solve on the current stream and return at once
        (pcg_solve): (u, stats) with stats a device tensor of nrhs
        fph_pcg_stats_t entries (decode with _lib.stats_from_device once the
        stream has reached it).  1 + maxiter + max_outer slots are enqueued,
        so maxiter is the iteration budget.  u is the initial guess unless
        zero_guess (default: u is None).  Allocates nothing when u and stats
        are given (the call can then be captured in a graph)."""
        nrhs = self._vec(b)
        if nrhs > self.max_rhs:
            raise ValueError("more right-hand sides than max_rhs")
        zero = (u is None) if zero_guess is None else bool(zero_guess)
        u = torch.empty_like(b) if u is None else u
        if stats is None:
            stats = torch.empty(nrhs * 4, dtype=torch.float64, device=b.device)
        if not (stats.is_cuda and stats.is_contiguous() and stats.numel() * stats.element_size() >= 32 * nrhs):
            raise ValueError("stats must be a contiguous CUDA tensor of at least 32 bytes per right-hand side")
        opts = self._opts(zero, tol, maxiter, precond, prec, ru_delta, 0, variant, max_outer)
        check(self.lib.pcg_solve(self.h, nrhs, _ptr(b), _ptr(u), ctypes.byref(opts), _ptr(stats),
                                 _stream()))
        return u, stats

    def force(self, u, grad=None, scale=1.0, scale_dev=None):
        """grad += scale * s * sum_r dS_F/dx for solutions u (float64); s is the
        one-element float64 CUDA tensor scale_dev, read on the device (no host
        synchronisation), or 1."""
        nrhs = self._vec(u)
        nf = getattr(self, "_nfields", 0) or 1
        shape = (self.Ltau, self.N) if nf == 1 and not getattr(self, "_nfields", 0) else (nf, self.Ltau, self.N)
        grad = torch.zeros(*shape, dtype=torch.float64, device=u.device) if grad is None else grad
        sd = _scale_ptr(scale_dev)
        check(self.lib.fermion_force(self.h, nrhs, _ptr(u), _ptr(grad), float(scale), sd, _stream()))
        return grad

    def action(self, b, u, out=None):
        """S_F = b . u per right-hand side, FP64 on the device."""
        nrhs = self._vec(b)
        out = torch.empty(nrhs, dtype=torch.float64, device=b.device) if out is None else out
        check(self.lib.fermion_action(self.h, nrhs, _ptr(b), _ptr(u), _ptr(out), _stream()))
        return out


class FermionBatch:
    """Many independent systems (lattice, field x, right-hand sides b) solved
    in one persistent launch.  ``systems`` is a list of (params, x, b) with
    params having L, Ltau, dtau, t, mu, alpha; x [Ltau, N] and b
    [nrhs, Ltau, N] float64 CUDA tensors.  Solutions land in ``self.u``
    (one tensor per system, same shape as b).  The tensors are referenced
    by the library: keep them alive and update them in place."""

    def __init__(self, systems):
        self.lib = _lib.load()
        self.keep = []
        self.u = []
        arr = (System * len(systems))()
        self.nrhs_total = 0
        for k, (p, x, b) in enumerate(systems):
            L, Ltau = int(p.L), int(p.Ltau)
            d = L * L * Ltau
            for t in (x, b):
                if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                    raise ValueError("x and b must be contiguous float64 CUDA tensors")
            if x.numel() != d or b.numel() % d:
                raise ValueError("shape mismatch between lattice and tensors")
            u = torch.zeros_like(b)
            nrhs = b.numel() // d
            self.keep += [x, b]
            self.u.append(u)
            arr[k] = System(Lattice(L, Ltau, float(p.dtau), float(p.t), float(p.mu), float(p.alpha)),
                            x.data_ptr(), nrhs, b.data_ptr(), u.data_ptr())
            self.nrhs_total += nrhs
        h = ctypes.c_void_p()
        check(self.lib.fph_batch_create(ctypes.byref(h), arr, len(systems)))
        self.h = h

    def _opts(self, tol, maxiter, ru_delta, precond=False, a1=1.0, a2=1.0):
        return PcgOpts(float(tol), int(maxiter), int(bool(precond)), FPH_F32_REFINED, 1,
                       float(ru_delta), 0, 0, 0, 0, float(a1), float(a2))

    def solve_async(self, tol=1e-8, maxiter=100000, ru_delta=0.0, stats=None, precond=False,
                    a1=1.0, a2=1.0):
        """Enqueue the batched solve (fph_batch_solve) and return the device
        statistics tensor (nrhs_total entries; see _lib.stats_from_device).
        precond: F F^T preconditioning with Chebyshev constants a1, a2."""
        if stats is None:
            stats = torch.empty(self.nrhs_total * 4, dtype=torch.float64, device=self.u[0].device)
        opts = self._opts(tol, maxiter, ru_delta, precond, a1, a2)
        check(self.lib.fph_batch_solve(self.h, ctypes.byref(opts), _ptr(stats), _stream()))
        return stats

    def solve(self, tol=1e-8, maxiter=100000, ru_delta=0.0, precond=False, a1=1.0, a2=1.0):
        """The batched solve, waiting for it: one stats dict per right-hand side."""
        return stats_from_device(self.solve_async(tol, maxiter, ru_delta, precond=precond, a1=a1,
                                                  a2=a2))

    def tune(self, tol=1e-8, maxiter=100000, ru_delta=0.0, precond=False, a1=1.0, a2=1.0):
        best = (ctypes.c_int32 * 3)()
        opts = self._opts(tol, maxiter, ru_delta, precond, a1, a2)
        check(self.lib.fph_batch_tune(self.h, ctypes.byref(opts), best, _stream()))
        return {"threads": best[0], "plaquettes_per_thread": best[1], "blocks_per_cu": best[2]}

    def close(self):
        if getattr(self, "h", None):
            self.lib.fph_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FermionAction(torch.autograd.Function):
    """S_F(x; Phi) = sum_r Phi_r^T (M(x)^T M(x))^{-1} Phi_r with the hand-written
    adjoint force as its gradient (Eq. dSF_dx; ``solver`` is a FermionSolver,
    or an SSHSolver, whose force is the product rule through its bond factors):
        dS_F/dx = sum_r -2 dtau alpha (M u_r) * (E * C u~_r),
        dS_F/dPhi_r = 2 u_r.
    forward installs x in the solver (field_kw: the Chebyshev constants a1, a2
    of a FermionSolver) and raises if a right-hand side did not converge.
    backward scales the force by the upstream gradient on the device; if the
    solver holds another field by then (a later set_field or a second
    action on the same solver), it installs x again for the force and then
    puts the other field back.
    """

    @staticmethod
    def forward(ctx, x, Phi, solver, field_kw, solve_kw):
        xc = x.detach().contiguous()
        Pc = Phi.detach().contiguous()
        solver.set_field(xc, **field_kw)
        u, stats = solver.solve(Pc, **solve_kw)
        bad = [k for k, st in enumerate(stats) if not (st["status"] & _lib.ST_CONVERGED)]
        if bad:
            raise RuntimeError("fermion_action: the solve did not converge for right-hand side(s) "
                               f"{bad}: {[stats[k] for k in bad]}")
        ctx.solver = solver
        ctx.field_kw = field_kw
        ctx.version = solver.field_version
        ctx.save_for_backward(u, xc)
        return solver.action(Pc, u).sum()

    @staticmethod
    def backward(ctx, g):
        u, xc = ctx.saved_tensors
        solver = ctx.solver
        gx = gphi = None
        gd = g.detach().to(torch.float64).reshape(1).contiguous()
        if ctx.needs_input_grad[0]:
            other = None
            if solver.field_version != ctx.version:
                other = solver.field_state()
                solver.set_field(xc, **ctx.field_kw)
            gx = solver.force(u, scale_dev=gd)
            if other is not None:
                solver.restore_field(other)
        if ctx.needs_input_grad[1]:
            gphi = (2.0 * gd) * u
        return gx, gphi, None, None, None


def fermion_action(x, Phi, solver, a1=None, a2=None, **solve_kw):
    """Differentiable S_F(x; Phi) (see FermionAction).  a1, a2: Chebyshev
    order constants of the preconditioner (FermionSolver only); solve_kw go
    to solver.solve."""
    field_kw = {}
    if a1 is not None:
        field_kw["a1"] = a1
    if a2 is not None:
        field_kw["a2"] = a2
    return FermionAction.apply(x, Phi, solver, field_kw, solve_kw)
