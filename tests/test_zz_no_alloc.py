"""fermion_action_noalloc (the no-allocation variant of fermion_action,
partial sums in the library's static device array) against fermion_action
through the C ABI: bit for bit, on two calls in a row, the second with a
smaller input, plus the host-side size check."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_noalloc_action_equals_action():
    from paper_2203_01291_amd import _lib
    from paper_2203_01291_amd.solver import FermionSolver
    lib = _lib.load()
    cases = [(16, 160, 3, 11), (4, 40, 1, 12)]   # second call: smaller lattice, fewer rhs
    for L, Ltau, nrhs, seed in cases:
        s = FermionSolver(L, Ltau, 0.1, 1.0, 0.0, 1.0, max_rhs=3)
        s.set_field(torch.zeros(Ltau * L * L, dtype=torch.float64, device=DEV))
        rng = np.random.default_rng(seed)
        b = torch.from_numpy(rng.standard_normal((nrhs, Ltau, L * L))).to(DEV)
        u = torch.from_numpy(rng.standard_normal((nrhs, Ltau, L * L))).to(DEV)
        ref = torch.empty(nrhs, dtype=torch.float64, device=DEV)
        got = torch.full((nrhs,), float("nan"), dtype=torch.float64, device=DEV)
        _lib.check(lib.fermion_action(s.h, nrhs, _p(b), _p(u), _p(ref), _stream()))
        _lib.check(lib.fermion_action_noalloc(s.h, nrhs, _p(b), _p(u), _p(got), _stream()))
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (L, got, ref)
        want = np.sum(b.cpu().numpy() * u.cpu().numpy(), axis=(1, 2))
        np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-12)
        s.close()


def test_noalloc_action_rejects_too_many_rhs():
    from paper_2203_01291_amd import _lib
    from paper_2203_01291_amd.solver import FermionSolver
    lib = _lib.load()
    s = FermionSolver(4, 2, 0.1, 1.0, 0.0, 1.0, max_rhs=65)
    b = torch.zeros(65 * 2 * 16, dtype=torch.float64, device=DEV)
    out = torch.zeros(65, dtype=torch.float64, device=DEV)
    assert lib.fermion_action_noalloc(s.h, 65, _p(b), _p(b), _p(out), _stream()) == _lib.FPH_E_NRHS
    assert lib.fermion_action_noalloc(s.h, 0, _p(b), _p(b), _p(out), _stream()) == _lib.FPH_E_NRHS
    s.close()
