"""The C-ABI library loads and exports every symbol declared in include/*.h
(no compute calls: this runs without a GPU)."""

import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(hdr).read()
        names += re.findall(r"^(?:const\s+char\s*\*|int|void)\s+(\w+)\s*\(", text, re.M)
    return names


def test_header_declares_required_entry_points():
    names = declared_symbols()
    for required in ("fermion_matvec", "pcg_solve", "fermion_force"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2203_01291_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert lib.fph_version().startswith(b"holstein")


def test_argument_errors_are_reported_on_the_host():
    """Argument checks happen before any device work: null pointers and bad
    lattices return negative codes without touching the GPU."""
    import ctypes
    from paper_2203_01291_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    h = ctypes.c_void_p()
    bad = _lib.Lattice(5, 40, 0.1, 1.0, 0.0, 1.0)       # odd L
    assert lib.fph_create(ctypes.byref(h), ctypes.byref(bad), 1) == -2
    bad = _lib.Lattice(4, 39, 0.1, 1.0, 0.0, 1.0)       # odd Ltau
    assert lib.fph_create(ctypes.byref(h), ctypes.byref(bad), 1) == -2
    good = _lib.Lattice(4, 40, 0.1, 1.0, 0.0, 1.0)
    assert lib.fph_create(ctypes.byref(h), ctypes.byref(good), 0) == -3
    assert lib.fph_create(None, ctypes.byref(good), 1) == -1
    assert lib.fermion_matvec(None, 0, 0, 1, None, None, None) == -1
    assert lib.pcg_solve(None, 1, None, None, None, None, None) == -1
    assert lib.pcg_solve_sync(None, 1, None, None, None, None, None) == -1
    assert lib.fermion_force(None, 1, None, None, 1.0, None, None) == -1
    assert b"NULL" in lib.fph_strerror(-1)
    # the bandwidth copy checks pointers, alignment, size and pattern first
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    assert lib.fph_hbm_copy(None, b, 16, 0, 0, None) == -1
    assert lib.fph_hbm_copy(ctypes.c_void_p((1 << 20) + 8), b, 16, 0, 0, None) == -6
    assert lib.fph_hbm_copy(a, b, 24, 0, 0, None) == -7
    assert lib.fph_hbm_copy(a, b, -16, 0, 0, None) == -7
    assert lib.fph_hbm_copy(a, b, 16, 0, 2, None) == -7
    assert lib.fph_hbm_copy(a, b, 16, (1 << 20) + 1, 1, None) == -7
    assert lib.fph_hbm_copy(a, b, 0, 0, 0, None) == 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2203_01291_amd import _lib
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load(str(tmp_path / "missing.so"))


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and offsets
    (checked with a host program compiled by gcc against include/holstein_hmc.h)."""
    import ctypes
    import shutil
    import subprocess
    from paper_2203_01291_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"fph_lattice_t": _lib.Lattice, "fph_pcg_opts_t": _lib.PcgOpts,
               "fph_pcg_stats_t": _lib.PcgStats, "fph_system_t": _lib.System,
               "fph_hmc_opts_t": _lib.HmcOpts, "fph_hmc_stats_t": _lib.HmcStats,
               "fph_update_stats_t": _lib.UpdateStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "holstein_hmc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_hmc_and_measurement_argument_errors_on_host():
    """The HMC, Lambda and measurement entry points check their arguments before any device
    work: null handles and pointers return FPH_E_NULL without touching the GPU."""
    from paper_2203_01291_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import ctypes
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.fph_hmc_create(ctypes.byref(h), None, None, None) == -1
    assert lib.fph_hmc_create(None, None, None, None) == -1
    assert lib.bosonic_action(None, None, None, None) == -1
    assert lib.bosonic_force(None, None, None, 1.0, None) == -1
    assert lib.hmc_mass_apply(None, 0, 1, None, None, None) == -1
    assert lib.hmc_boson_steps(None, None, None, None) == -1
    assert lib.hmc_trajectory(None, None, None, None, 0.5, None, None, None) == -1
    assert lib.lambda_apply(None, 0, None, 1, None, None, None) == -1
    assert lib.lambda_force(None, 1, None, None, None, 1.0, None) == -1
    assert lib.hmc_global_update(None, 0, 0, 0, None, None, 0.5, None, None) == -1
    assert lib.fph_meas_create(ctypes.byref(h), None, None) == -1
    assert lib.meas_fft(None, 0, 0, None, None, None) == -1
    assert lib.green_vectors(None, 1, None, None, None, None, None) == -1
    assert lib.green_average(None, 1, None, None, None, None) == -1
    assert lib.green_pair_products(None, 2, None, None, None, None) == -1
    assert lib.fph_get_lattice(None, None, None) == -1


def test_ssh_argument_errors_on_host():
    """The SSH entry points check their arguments before any device work: bad lattices, a
    non-finite coupling, bad right-hand-side counts and null pointers return negative codes."""
    from paper_2203_01291_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import ctypes
    lib = _lib.load()
    h = ctypes.c_void_p()
    good = _lib.Lattice(4, 8, 0.1, 1.0, 0.0, 1.0)
    assert lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(_lib.Lattice(5, 8, 0.1, 1.0, 0.0, 1.0)),
                              0.2, 1) == -2
    assert lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(_lib.Lattice(66, 8, 0.1, 1.0, 0.0, 1.0)),
                              0.2, 1) == -2
    assert lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(_lib.Lattice(4, 7, 0.1, 1.0, 0.0, 1.0)),
                              0.2, 1) == -2
    assert lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(good), float("nan"), 1) == -7
    assert lib.fph_ssh_create(ctypes.byref(h), ctypes.byref(good), 0.2, 0) == -3
    assert lib.fph_ssh_create(None, ctypes.byref(good), 0.2, 1) == -1
    assert lib.fph_ssh_destroy(None) == -1
    assert lib.ssh_set_field(None, None, None) == -1
    assert lib.ssh_matvec(None, 0, 1, None, None, None) == -1
    assert lib.ssh_solve(None, 1, None, None, None, None, None) == -1
    assert lib.ssh_force(None, 1, None, None, 1.0, None, None) == -1
    assert lib.ssh_action(None, 1, None, None, None, None) == -1
    assert lib.ssh_set_preconditioner(None, None, 1.0, 1.0) == -1
    assert lib.fph_hmc_create_ssh(ctypes.byref(h), None, None, None) == -1
    assert lib.fph_hmc_create_ssh(None, None, None, None) == -1
