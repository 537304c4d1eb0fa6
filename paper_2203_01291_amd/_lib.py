"""ctypes declarations of the C ABI in include/holstein_hmc.h.

Loading fails loudly when the shared library has not been built: there is
no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libholstein_hmc.so")

FPH_OK = 0
FPH_E_NULL, FPH_E_LATTICE, FPH_E_NRHS, FPH_E_PREC, FPH_E_NOFIELD, FPH_E_ALIGN, FPH_E_ARG = -1, -2, -3, -4, -5, -6, -7
FPH_OP_M, FPH_OP_MT, FPH_OP_MTM = 0, 1, 2
FPH_F64, FPH_F32, FPH_F32_REFINED = 0, 1, 2
FPH_PC_F, FPH_PC_FT, FPH_PC_FFT = 0, 1, 2
ST_CONVERGED, ST_MAXITER, ST_BREAKDOWN, ST_NONFINITE, ST_ABORTED = 1, 2, 4, 8, 16


class Lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("Ltau", ctypes.c_int32), ("dtau", ctypes.c_double),
                ("t", ctypes.c_double), ("mu", ctypes.c_double), ("alpha", ctypes.c_double)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32),
                ("use_precond", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("zero_guess", ctypes.c_int32), ("ru_delta", ctypes.c_double),
                ("chunk", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cheb_a1", ctypes.c_double), ("cheb_a2", ctypes.c_double)]


class PcgStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32), ("matvecs", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("action", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def stats_from_device(t):
    """Decode a device array of fph_pcg_stats_t (a CUDA tensor of 32-byte
    entries, as written by pcg_solve or fph_batch_solve) into dicts.
    Copies to the host, so it waits for the stream."""
    raw = t.detach().cpu().contiguous().numpy().tobytes()
    n = len(raw) // ctypes.sizeof(PcgStats)
    arr = (PcgStats * n).from_buffer_copy(raw[:n * ctypes.sizeof(PcgStats)])
    return [s.as_dict() for s in arr]


class System(ctypes.Structure):
    _fields_ = [("lat", Lattice), ("x_dev", ctypes.c_void_p), ("nrhs", ctypes.c_int32),
                ("b_dev", ctypes.c_void_p), ("u_dev", ctypes.c_void_p)]


class HmcOpts(ctypes.Structure):
    _fields_ = [("omega0", ctypes.c_double), ("m_reg", ctypes.c_double), ("dt", ctypes.c_double),
                ("Nt", ctypes.c_int32), ("nt", ctypes.c_int32), ("nfields", ctypes.c_int32),
                ("a1", ctypes.c_double), ("a2", ctypes.c_double),
                ("guess", ctypes.c_int32), ("lambda_action", ctypes.c_int32),
                ("nchains", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("force_solve", PcgOpts), ("action_solve", PcgOpts)]


class HmcStats(ctypes.Structure):
    _fields_ = [("H_i", ctypes.c_double), ("H_f", ctypes.c_double),
                ("SB_i", ctypes.c_double), ("SB_f", ctypes.c_double),
                ("SF_i", ctypes.c_double), ("SF_f", ctypes.c_double),
                ("K_i", ctypes.c_double), ("K_f", ctypes.c_double),
                ("accept_prob", ctypes.c_double), ("accepted", ctypes.c_int32),
                ("status", ctypes.c_int32), ("solves", ctypes.c_int32),
                ("cg_iters", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class UpdateStats(ctypes.Structure):
    _fields_ = [("dS", ctypes.c_double), ("dS_B", ctypes.c_double), ("SF_old", ctypes.c_double),
                ("SF_new", ctypes.c_double), ("accept_prob", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("status", ctypes.c_int32),
                ("cg_iters", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


FPH_MASS_INV, FPH_MASS_SQRT, FPH_MASS = 0, 1, 2
FPH_LAMBDA, FPH_LAMBDA_INV, FPH_LAMBDA_T, FPH_LAMBDA_INV_T = 0, 1, 2, 3
FPH_MOVE_REFLECT, FPH_MOVE_SWAP = 0, 1

EXPORTS = {
    "fph_ssh_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Lattice), ctypes.c_double,
                                      ctypes.c_int32]),
    "fph_ssh_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ssh_set_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ssh_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "ssh_set_preconditioner": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                              ctypes.c_double]),
    "fph_hmc_create_ssh": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                          ctypes.POINTER(HmcOpts), ctypes.c_void_p]),
    "ssh_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgStats), ctypes.c_void_p]),
    "ssh_action": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "ssh_force": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "fph_hbm_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p]),
    "fph_version": (ctypes.c_char_p, []),
    "fph_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fph_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Lattice), ctypes.c_int32]),
    "fph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fph_get_lattice": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Lattice),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "fph_set_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_void_p]),
    "fph_set_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_void_p]),
    "fermion_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pcg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(PcgOpts), ctypes.c_void_p, ctypes.c_void_p]),
    "pcg_solve_sync": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgStats), ctypes.c_void_p]),
    "fermion_force": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "fermion_action": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fermion_action_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fph_precond_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fph_precond_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "fph_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(System),
                                        ctypes.c_int32]),
    "fph_batch_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PcgOpts),
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "fph_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PcgOpts),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "fph_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fph_hmc_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                      ctypes.POINTER(HmcOpts), ctypes.c_void_p]),
    "fph_hmc_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "bosonic_action": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "bosonic_force": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_void_p]),
    "hmc_mass_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hmc_boson_steps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "hmc_trajectory": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.POINTER(HmcStats), ctypes.c_void_p]),
    "hmc_trajectories": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                        ctypes.POINTER(HmcStats), ctypes.c_void_p]),
    "lambda_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lambda_force": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "hmc_global_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.POINTER(UpdateStats), ctypes.c_void_p]),
    "fph_meas_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_void_p]),
    "fph_meas_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "meas_fft": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]),
    "green_vectors": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgStats), ctypes.c_void_p]),
    "green_average": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "green_pair_products": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


def load(path=None):
    """Load the library and declare every exported entry point."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"HIP library {p} is missing; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (no CPU fallback exists)")
    # The library and PyTorch must share one HIP runtime: torch ships its
    # own libamdhip64.so.7 and HSA runtime, and the library's dependency of
    # the same soname resolves to whichever copy is loaded first.  Loading
    # the library first would bring in the system runtime beside torch's
    # HSA runtime, after which torch finds no GPU.  So torch comes first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class FphError(RuntimeError):
    pass


def check(code):
    if code != FPH_OK:
        msg = load().fph_strerror(code).decode()
        raise FphError(f"fph error {code}: {msg}")
