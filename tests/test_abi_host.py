"""Host-side checks of the C ABI (no GPU): the library loads, exports every function that
include/agca.h declares, and validates configurations without touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agca.h")
LIB = os.path.join(ROOT, "paper_2511_13109_amd", "libagca.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libagca.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(agca_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2511_13109_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_validate_config_rejects_bad_values():
    from paper_2511_13109_amd import _lib
    import paper_2511_13109_amd as p
    lib = _lib.load()
    cfg = p.default_config()
    assert p.validate_config(cfg) == _lib.AGCA_OK
    for field, value, frag in [("ncomp", 2, b"ncomp"), ("L", 0, b"L must"), ("L", 12, b"L must"),
                               ("omega", 2.5, b"omega"), ("flag_mode", 7, b"flag_mode"),
                               ("mg_dtype", _lib.BF16, b"mg_dtype"), ("pre_sweeps", -1, b"sweeps")]:
        c2 = p.default_config()
        setattr(c2, field, value)
        assert p.validate_config(c2) == _lib.AGCA_E_INVALID
        assert frag in lib.agca_last_error()
    c3 = p.default_config()
    c3.mg_dtype = _lib.F32
    c3.mg_nu_dtype = _lib.F64
    assert p.validate_config(c3) == _lib.AGCA_E_INVALID
    c3.mg_nu_dtype = _lib.BF16
    assert p.validate_config(c3) == _lib.AGCA_OK


def test_null_arguments_are_errors_not_crashes():
    from paper_2511_13109_amd import _lib
    lib = _lib.load()
    assert lib.agca_create(None, None, None, None, None) == _lib.AGCA_E_INVALID
    assert lib.agca_apply(None, 0, 0, None, None) == _lib.AGCA_E_INVALID
    assert lib.agca_destroy(None) == _lib.AGCA_OK
    assert lib.agca_device_bytes(None) == 0


def test_stokes_entry_points_reject_a_null_hierarchy():
    # the Stokes and pressure-multigrid entry points check the handle before any device
    # work (no GPU needed to call them this way)
    from paper_2511_13109_amd import _lib
    lib = _lib.load()
    assert lib.agca_stokes_schur_apply(None, _lib.SCHUR_BFBT_MG, 4, None, None) == _lib.AGCA_E_INVALID
    assert b"null hierarchy" in lib.agca_last_error()
    assert lib.agca_stokes_z_stencil(None, 0, None) == _lib.AGCA_E_INVALID
    assert lib.agca_stokes_z_vcycle(None, None, None) == _lib.AGCA_E_INVALID
    opts = _lib.StokesOpts()
    assert lib.agca_stokes_solve(None, opts, None, None, None, None, None) == _lib.AGCA_E_INVALID
