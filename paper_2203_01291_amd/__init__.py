"""MI355X (gfx950) fermion solver for the Holstein-model hybrid Monte Carlo
of arXiv:2203.01291: M / M^T / M^T M applies, (preconditioned) conjugate
gradients on M^T M in FP64 or FP32 with FP64 residual replacement, the
action S_F and the adjoint phonon force, behind the C ABI of
``include/holstein_hmc.h``."""

from ._lib import LIB_PATH, load  # noqa: F401


def __getattr__(name):
    # torch-dependent pieces are imported lazily so that `import` works
    # without initialising a GPU.
    if name in ("FermionSolver", "FermionAction", "fermion_action"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
