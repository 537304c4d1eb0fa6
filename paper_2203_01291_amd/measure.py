"""Python binding of the stochastic Green's-function measurements (Sec. VI).

Argument marshalling only: every step runs in the HIP library; tensors give
device pointers and the current torch stream gives the hipStream_t.
"""

import ctypes

import torch

from . import _lib
from ._lib import PcgStats, check
from .hmc import _pcg_opts
from .solver import _ptr, _stream


class GreenMeasurement:
    """Green's-function estimators on the lattice of one ``FermionSolver``
    (which must outlive this object).  Vectors are float64 CUDA tensors
    [nvec, Ltau, N]; results are [Ltau, L, L] (one average) or [3, Ltau, L, L]
    (the three four-point products), indexed [dtau, dy, dx]."""

    def __init__(self, solver):
        self.lib = _lib.load()
        self.solver = solver
        h = ctypes.c_void_p()
        check(self.lib.fph_meas_create(ctypes.byref(h), solver.h, _stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.fph_meas_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fft(self, z, inverse=False, twist=False):
        """Unnormalised 3-D DFT of a complex128 CUDA tensor [Ltau, N]."""
        if not (z.is_cuda and z.dtype == torch.complex128 and z.is_contiguous()):
            raise ValueError("expected a contiguous complex128 CUDA tensor")
        if z.numel() != self.solver.dim:
            raise ValueError("expected N*Ltau values")
        out = torch.empty_like(z)
        check(self.lib.meas_fft(self.h, int(bool(inverse)), int(bool(twist)), _ptr(z), _ptr(out), _stream()))
        return out

    def green_vectors(self, xi, tol=1e-8, precond=True, prec="f32_refined", maxiter=100000):
        """G xi for every vector of xi (the solver's field must be set).  Returns (Gxi, stats)."""
        n = self.solver._vec(xi)
        gx = torch.empty_like(xi)
        st = (PcgStats * n)()
        opts = _pcg_opts(tol, precond, prec, maxiter)
        check(self.lib.green_vectors(self.h, n, _ptr(xi), _ptr(gx), ctypes.byref(opts), st, _stream()))
        return gx, [v.as_dict() for v in st]

    def green_average(self, xi, gxi):
        n = self.solver._vec(xi)
        out = torch.empty(self.solver.Ltau, self.solver.L, self.solver.L, dtype=torch.float64, device=xi.device)
        check(self.lib.green_average(self.h, n, _ptr(xi), _ptr(gxi), _ptr(out), _stream()))
        return out

    def pair_products(self, xi, gxi):
        n = self.solver._vec(xi)
        out = torch.empty(3, self.solver.Ltau, self.solver.L, self.solver.L, dtype=torch.float64,
                          device=xi.device)
        check(self.lib.green_pair_products(self.h, n, _ptr(xi), _ptr(gxi), _ptr(out), _stream()))
        return out
