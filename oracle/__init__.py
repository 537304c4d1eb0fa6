"""Plain FP64 CPU oracle for the Holstein-model fermion solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything under
``oracle/``.  The product path (the HIP library and its Python binding)
never imports, links or calls it, and it shares no code with that path: the
only common module is ``workloads`` (seeded random draws, no arithmetic of
the method).

Every routine is a direct, slow, obviously checkable transcription of a
definition in the paper (arXiv:2203.01291):

* ``lattice``  - hopping matrix K, checkerboard factors of exp(-dtau K),
                 the blocks B_tau and the space-time matrix M
                 (Sec. II C, Eqs. M_def, B_def, V_K_def).
* ``solve``    - direct solves of (M^T M) u = Phi via LU of M, and a
                 textbook (P)CG for sizes where LU does not fit
                 (Sec. II D, Eqs. psi_def, CG; Sec. V, Eq. CG_precon).
* ``force``    - the phonon force dS_F/dx (Sec. III A, Eq. dSF_dx), and
                 complex-step / finite-difference derivatives of S_F.
* ``precond``  - the adiabatic preconditioner P, its Fourier-space block
                 form and its Chebyshev (KPM) apply (Sec. V A, Eqs. P_def,
                 Bbar, udef, Mww, P_change_basis; App. C).
* ``hmc``      - the hybrid Monte Carlo update with A = M: bosonic action
                 and force, Fourier-acceleration mass, time-step splitting
                 leapfrog and the Metropolis test (Sec. III, Algorithm 1).
* ``lam``      - the Lambda reformulation A = M Lambda of the action, its
                 force, and the reflection and swap updates (Secs. II C, IV;
                 App. B).
* ``measure``  - stochastic Green's-function estimates and their space-time
                 averages by FFT cross-correlation (Sec. VI).
* ``ssh``      - the space-time matrix, action and product-rule force of an
                 SSH-type coupling, where x enters the hopping inside the
                 checkerboard factors (Sec. II C closing remark; Sec. III A).

Parity status of each function is stated in its docstring; a function with
no independent pin says "parity unpinned".
"""

from . import lattice, solve, force, precond, hmc, lam, measure, ssh  # noqa: F401
