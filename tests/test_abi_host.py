"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/sbd.h declares, and
reject invalid arguments on the host before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2601_16637_amd as sbd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sbd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sbd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = sbd.load()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), f"{n} declared in sbd.h but not exported"
    assert set(names) == set(sbd.EXPORTED)


def test_version_and_default_opts():
    L = sbd.load()
    assert L.sbd_version() >= 100
    o = sbd.default_opts()
    assert o.tol_residual == 1e-6 and o.max_space == 20 and o.max_iter == 200
    assert o.precond_delta == 1e-8 and o.sigma_prec == sbd.FP64


def _status(fn):
    try:
        fn()
    except sbd.SBDError as e:
        return e.status
    return 0


def test_basis_validation_on_host():
    ok = np.array([0b1111], dtype=np.uint64)
    assert _status(lambda: sbd.Basis(0, 0, 0, ok, ok)) == -2
    assert _status(lambda: sbd.Basis(65, 4, 4, ok, ok)) == -2
    assert _status(lambda: sbd.Basis(8, 9, 4, ok, ok)) == -1
    bad_pop = np.array([0b1111, 0b111], dtype=np.uint64)
    assert _status(lambda: sbd.Basis(8, 4, 4, bad_pop, ok)) == -3
    high = np.array([0b111 | (1 << 9)], dtype=np.uint64)
    assert _status(lambda: sbd.Basis(8, 4, 4, ok, high)) == -3
    empty = np.zeros(0, dtype=np.uint64)
    assert _status(lambda: sbd.Basis(8, 4, 4, empty, ok)) == -1
    assert "popcount" in sbd.last_error() or "string" in sbd.last_error()


def test_null_handles_rejected():
    L = sbd.load()
    out = ctypes.c_void_p()
    assert L.sbd_build_excitations(None, None, ctypes.byref(out)) == -1
    assert L.sbd_sigma(None, None, None, 1, 0, 0.0, None, None, 0, None) == -1
    e = np.zeros(1)
    assert L.sbd_davidson(None, None, None, 1, None, e.ctypes.data_as(ctypes.c_void_p),
                          None, None, None) == -1
    assert L.sbd_set_hamiltonian(None, None, None, None, 0.0, None, ctypes.byref(out)) == -1
    n = ctypes.c_int64()
    assert L.sbd_exc_count(None, 0, 1, ctypes.byref(n)) == -1


def test_norb64_strings_accepted_by_validation():
    """norb = 64 uses every bit; validation must not reject the top bit."""
    full = np.array([np.uint64((1 << 64) - 1)], dtype=np.uint64)
    st = _status(lambda: sbd.Basis(64, 64, 64, full, full))
    # on a machine without a GPU the call gets past validation and fails in HIP
    assert st in (0, -6)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the option, report, request and result structs
    have the C header's sizes and field offsets (compiled with gcc)."""
    import ctypes
    import shutil
    import subprocess
    from paper_2601_16637_amd import _native as nat
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"sbd_davidson_opts": nat.DavidsonOpts, "sbd_davidson_report": nat.DavidsonReport,
               "sbd_request": nat.Request, "sbd_result": nat.Result, "sbd_sqd_opts": nat.SqdOpts,
               "sbd_sqd_step": nat.SqdStep}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sbd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            c, f, v = line.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_recover_configurations_validation_on_host():
    ok = np.array([[0b0111, 0b0011]], dtype=np.uint64)
    assert _status(lambda: sbd.recover_configurations(0, 3, 2, ok)) == -2
    assert _status(lambda: sbd.recover_configurations(65, 3, 2, ok)) == -2
    assert _status(lambda: sbd.recover_configurations(4, 5, 2, ok)) == -1
    assert _status(lambda: sbd.recover_configurations(4, 3, 2, np.array([[0b10111, 0b0011]], dtype=np.uint64))) == -3
    assert "at or above norb" in sbd.last_error()
    assert _status(lambda: sbd.recover_configurations(4, 3, 2, ok, np.full(4, np.inf), np.zeros(4))) == -1


def test_full_basis_validation_on_host():
    ok = np.array([[0b1111, 0b1111]], dtype=np.uint64)
    assert _status(lambda: sbd.FullBasis(0, 4, 4, ok)) == -2
    assert _status(lambda: sbd.FullBasis(65, 4, 4, ok)) == -2
    assert _status(lambda: sbd.FullBasis(8, 9, 4, ok)) == -1
    assert _status(lambda: sbd.FullBasis(8, 4, 4, np.array([[0b1111, 0b111]], dtype=np.uint64))) == -3
    assert _status(lambda: sbd.FullBasis(8, 4, 4, np.array([[0b111 | (1 << 9), 0b1111]], dtype=np.uint64))) == -3
    assert _status(lambda: sbd.FullBasis(8, 4, 4, np.zeros((0, 2), dtype=np.uint64))) == -1
    assert "determinant" in sbd.last_error()
