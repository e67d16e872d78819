"""The C-ABI library loads and exports every symbol of include/invdft.h (CPU only).

Only argument-validation paths are called here: they return before any HIP call,
so no GPU is needed.
"""
import ctypes as C
import os
import re

import pytest

from paper_2510_10529_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "invdft.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def _lib_or_skip():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libinvdft.so not built")
    return _lib.load()


def test_header_lists_all_bound_symbols():
    decl = _declared()
    assert len(decl) >= 15
    assert set(decl) == set(_lib.SIGNATURES), (set(decl) ^ set(_lib.SIGNATURES))


def test_library_exports_every_declared_symbol():
    lib = _lib_or_skip()
    for name in _declared():
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.load()


def test_argument_checks_without_gpu():
    lib = _lib_or_skip()
    h = C.c_void_p()
    assert lib.fe_mesh_create(0, 4, 1.0, C.byref(h)) == _lib.FE_EINVAL
    assert b"p must be" in lib.fe_last_error()
    assert lib.fe_mesh_create(9, 4, 1.0, C.byref(h)) == _lib.FE_EINVAL
    assert lib.fe_mesh_create(2, 0, 1.0, C.byref(h)) == _lib.FE_EINVAL
    assert lib.fe_mesh_create(2, 4, -1.0, C.byref(h)) == _lib.FE_EINVAL
    assert lib.fe_mesh_create(2, 4, 1.0, None) == _lib.FE_EINVAL
    null = C.c_void_p()
    assert lib.ks_apply(null, None, None, None, None, 1, 1, 0, None) == _lib.FE_EINVAL
    assert lib.cheb_filter(null, None, 3, 0.0, 1.0, -1.0, None, 1, 1, 0, None, None) == _lib.FE_EINVAL
    assert lib.rayleigh_ritz(null, None, None, None, None, 1, 1, None, None) == _lib.FE_EINVAL
    assert lib.adjoint_solve(null, None, None, None, 1, None, None, 1e-8, 10, None, None, 0, None,
                             None) == _lib.FE_EINVAL
    assert lib.loss_grad(null, None, None, 1, None, None, 0.0, None, None, None, None, None, None) == _lib.FE_EINVAL
    assert lib.fe_workspace_bytes(null, 0, 4, 0) == 0
    assert lib.fe_mesh_destroy(null) == _lib.FE_OK
    out = C.c_double()
    assert lib.fe_dot(None, None, 10, C.byref(out), None, None) == _lib.FE_EINVAL
    assert lib.fe_axpby(C.c_double(1.0), None, C.c_double(1.0), None, 5, None) == _lib.FE_EINVAL
    assert lib.fe_axpby(C.c_double(1.0), None, C.c_double(1.0), None, 0, None) == _lib.FE_OK   # empty: nothing
    # apply timing: an empty record reads back as zero launches, a bad precision is rejected
    n, ms, b = C.c_int64(7), C.c_double(1.0), C.c_double(1.0)
    assert lib.fe_apply_timing(1) == _lib.FE_OK
    assert lib.fe_apply_timing_read(_lib.FE_F64, C.byref(n), C.byref(ms), C.byref(b), None) == _lib.FE_OK
    assert (n.value, ms.value, b.value) == (0, 0.0, 0.0)
    assert lib.fe_apply_timing(0) == _lib.FE_OK
    assert lib.fe_apply_timing_read(3, None, None, None, None) == _lib.FE_EINVAL     # no such precision
    assert lib.fe_sweep_timing_read(0, C.byref(n), C.byref(ms), C.byref(b), None) == _lib.FE_OK
    assert (n.value, ms.value, b.value) == (0, 0.0, 0.0)
    assert lib.fe_sweep_timing_read(3, None, None, None, None) == _lib.FE_EINVAL      # no such pass
    assert lib.ks_apply(null, None, None, None, None, 1, 1, _lib.FE_BF16, None) == _lib.FE_EINVAL   # NULL mesh
    # finite temperature: argument checks return before any arithmetic
    eig = (C.c_double * 3)(-1.0, 0.0, 1.0)
    bad = (C.c_double * 3)(0.0, -1.0, 1.0)
    occ = (C.c_double * 3)()
    assert lib.fermi_occupations(eig, 3, 2.0, 0.0, 2.0, 1e-12, occ, None, None, None) == _lib.FE_EINVAL
    assert lib.fermi_occupations(eig, 3, 6.0, 0.1, 2.0, 1e-12, occ, None, None, None) == _lib.FE_EINVAL
    assert lib.fermi_occupations(eig, 3, 0.0, 0.1, 2.0, 1e-12, occ, None, None, None) == _lib.FE_EINVAL
    assert lib.fermi_occupations(bad, 3, 2.0, 0.1, 2.0, 1e-12, occ, None, None, None) == _lib.FE_EINVAL
    assert b"ascend" in lib.fe_last_error()
    assert lib.fermi_occupations(eig, 3, 2.0, 0.1, 2.0, 1.0, occ, None, None, None) == _lib.FE_EINVAL
    assert lib.fermi_occupations(None, 3, 2.0, 0.1, 2.0, 1e-12, occ, None, None, None) == _lib.FE_EINVAL
    assert lib.adjoint_along_psi(null, None, 1, None, 0.0, 0.1, 2.0, None, None, None, None, None, None,
                                 None) == _lib.FE_EINVAL
    assert lib.fe_workspace_bytes(null, _lib.FE_OP_ALONG_PSI, 4, 0) == 0
    # linear XC mesh
    t = (C.c_double * 3)(-1.0, 0.0, 1.0)
    vmh = C.c_void_p()
    assert lib.vxc_mesh_create(null, 2, t, 2, t, 2, t, C.byref(vmh)) == _lib.FE_EINVAL
    assert lib.vxc_mesh_info(null, None, None) == _lib.FE_EINVAL
    assert lib.vxc_prolong(null, None, None, None, None) == _lib.FE_EINVAL
    assert lib.vxc_restrict(null, None, None, None) == _lib.FE_EINVAL
    assert lib.vxc_mesh_destroy(null) == _lib.FE_OK
    # physics front end
    assert lib.poisson_solve(null, None, 1.0, None, 1e-10, 10, None, None, None, None, None) == _lib.FE_EINVAL
    assert lib.xc_initial_guess(null, None, None, 10.0, 1e-2, 1.0, 0, None, None, None) == _lib.FE_EINVAL
    assert lib.fe_workspace_bytes(null, _lib.FE_OP_POISSON, 1, 0) == 0


def test_status_exceptions_carry_message():
    _lib_or_skip()
    err = None
    lib = _lib.load()
    st = lib.fe_mesh_create(0, 1, 1.0, C.byref(C.c_void_p()))
    try:
        _lib.check(st, "fe_mesh_create")
    except _lib.FEError as e:
        err = e
    assert err is not None and err.status == _lib.FE_EINVAL and "FE_EINVAL" in str(err)
