"""The C ABI library loads and exports every declared entry point (no GPU).

Also exercises argument and charge validation, which the library performs
on the host before it touches the device.
"""
import ctypes as C
import os
import re

import pytest

from paper_2303_11409_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "u1mps.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("mps_create", "mps_apply_gate", "mps_truncate", "mps_amplitude", "mps_norm"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == declared_symbols()


def test_default_options():
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert (o.chi_max, o.cutoff, o.zero_tol, o.max_sweeps, o.jacobi_tol) == (0, 0.0, 1e-13, 40, 0.0)


def _create(L, d, N, dims, charges):
    lib = binding.lib()
    h = C.c_void_p()
    cd = (C.c_int * len(dims))(*dims)
    cc = (C.c_int * len(charges))(*charges)
    st = lib.mps_create(L, d, N, cd, cc, None, None, None, None, C.byref(h))
    return st, lib.mps_last_error().decode(), h


def test_charge_validation_errors():
    # bond 0 must carry N, bond L must carry 0 (Eq. E4)
    st, msg, h = _create(3, 3, 2, [1, 1, 1, 1], [1, 1, 0, 0])
    assert st == -2 and "bond 0" in msg and not h.value
    st, msg, _ = _create(3, 3, 2, [1, 1, 1, 1], [2, 1, 0, 1])
    assert st == -2
    # a charge step larger than d-1 has no admissible partner (Eq. E2)
    st, msg, _ = _create(3, 2, 3, [1, 1, 1, 1], [3, 1, 0, 0])
    assert st == -2 and "partner" in msg
    # charge outside 0..N
    st, msg, _ = _create(3, 3, 2, [1, 1, 1, 1], [2, 5, 0, 0])
    assert st == -2


def test_argument_errors():
    lib = binding.lib()
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 5, 0)
    assert lib.mps_create_product(4, 3, occ, None, None, C.byref(h)) == -1
    assert lib.mps_create_product(1, 3, occ, None, None, C.byref(h)) == -1
    occ2 = (C.c_int * 4)(1, 0, 1, 0)
    assert lib.mps_create_product(4, 1, occ2, None, None, C.byref(h)) == -1
    assert lib.mps_apply_gate(None, 0, None, None) == -1
    assert lib.mps_norm(None, None) == -1
    assert lib.mps_destroy(None) == 0
    assert isinstance(lib.mps_last_error(), bytes)


def test_apply_batch_argument_errors():
    """mps_apply_batch rejects bad arguments before touching any device state."""
    lib = binding.lib()
    assert lib.mps_apply_batch(0, None, None, None, None, None) == 0
    assert lib.mps_apply_batch(-1, None, None, None, None, None) == -1
    hs = (C.c_void_p * 2)(None, None)
    counts = (C.c_int * 2)(1, 0)
    sites = (C.c_int * 1)(0)
    assert lib.mps_apply_batch(2, hs, counts, sites, None, None) == -1
    assert "invalid handle" in lib.mps_last_error().decode()
    assert lib.mps_apply_batch(2, hs, None, sites, None, None) == -1


def test_form_option():
    """The default form is plain complex128; an unknown form is rejected."""
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert o.form == binding.FORM_PLAIN_C128
    o.form = 7
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 1, 0)
    assert lib.mps_create_product(4, 3, occ, C.byref(o), None, C.byref(h)) == -1
    assert "form" in lib.mps_last_error().decode()


def test_modulus_option():
    """The default charge is U(1) (modulus 0); a Z_n charge needs n >= 2 and
    n >= d (each local occupation its own charge), and its bond charges must
    lie in 0..n-1 -- all refused before any device work."""
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert o.modulus == 0
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 1, 0)
    for bad, d in ((3, 4), (1, 2), (-2, 2)):
        o.modulus = bad
        assert lib.mps_create_product(4, d, occ, C.byref(o), None, C.byref(h)) == -1
        assert "Z_n" in lib.mps_last_error().decode() or "modulus" in lib.mps_last_error().decode()
    assert not h.value
    o.modulus = 2
    cd = (C.c_int * 4)(1, 1, 1, 1)
    cc = (C.c_int * 4)(0, 2, 1, 0)
    assert lib.mps_create(3, 2, 2, cd, cc, None, None, C.byref(o), None, C.byref(h)) == -2
    cc = (C.c_int * 4)(1, 1, 1, 0)                 # bond 0 must carry N mod 2 = 0
    assert lib.mps_create(3, 2, 2, cd, cc, None, None, C.byref(o), None, C.byref(h)) == -2
    assert "bond 0" in lib.mps_last_error().decode()


def test_diagnostic_options():
    """blocked_sweeps and select_scratch default to 0 and are range-checked on
    the host."""
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert (o.blocked_sweeps, o.select_scratch) == (0, 0)
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 1, 0)
    o.blocked_sweeps = -1
    assert lib.mps_create_product(4, 3, occ, C.byref(o), None, C.byref(h)) == -1
    assert "blocked_sweeps" in lib.mps_last_error().decode()
    o.blocked_sweeps = 0
    o.select_scratch = 2
    assert lib.mps_create_product(4, 3, occ, C.byref(o), None, C.byref(h)) == -1
    assert "select_scratch" in lib.mps_last_error().decode()


def test_jacobi_block_option():
    """jacobi_block defaults to 0 (chosen per update); only 0, 8 and 16 are accepted,
    checked on the host."""
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert o.jacobi_block == 0
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 1, 0)
    for bad in (-1, 4, 12, 32):
        o.jacobi_block = bad
        assert lib.mps_create_product(4, 3, occ, C.byref(o), None, C.byref(h)) == -1
        assert "jacobi_block" in lib.mps_last_error().decode()
    assert not h.value


def test_jacobi_lockstep_option():
    """jacobi_lockstep defaults to 0 (sectors sweep at their own pace); only 0 and
    1 are accepted, checked on the host."""
    lib = binding.lib()
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    assert o.jacobi_lockstep == 0
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 0, 1, 0)
    for bad in (-1, 2):
        o.jacobi_lockstep = bad
        assert lib.mps_create_product(4, 3, occ, C.byref(o), None, C.byref(h)) == -1
        assert "jacobi_lockstep" in lib.mps_last_error().decode()
    assert not h.value


def test_last_leaks_argument_errors():
    lib = binding.lib()
    n = C.c_int(-1)
    assert lib.mps_last_leaks(None, 0, C.byref(n), None) == -1


def test_charge_map_argument_errors():
    """mps_create_product_charges refuses bad maps before touching the device."""
    lib = binding.lib()
    h = C.c_void_p()
    occ = (C.c_int * 4)(1, 2, 0, 3)
    o = binding.mps_opts()
    lib.mps_default_opts(C.byref(o))
    good = (C.c_int * 8)(0, 0, 0, 1, 1, 0, 1, 1)
    dup = (C.c_int * 8)(0, 0, 0, 1, 0, 1, 1, 1)
    assert lib.mps_create_product_charges(4, 4, occ, 3, good, C.byref(o), None, C.byref(h)) == -1
    assert lib.mps_create_product_charges(4, 4, occ, 2, dup, C.byref(o), None, C.byref(h)) == -1
    assert "same charge" in lib.mps_last_error().decode()
    o.modulus = 4
    assert lib.mps_create_product_charges(4, 4, occ, 2, good, C.byref(o), None, C.byref(h)) == -1
    assert not h.value
