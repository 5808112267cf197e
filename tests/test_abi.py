"""The C-ABI library: it loads, exports every entry point the header
declares, and rejects invalid arguments with the documented status before
touching the device (these checks need no GPU)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_09578_amd import capi

    if not os.path.exists(capi.LIB_PATH):
        pytest.fail("libfm.so is not built (run __graft_entry__.build())")
    return capi.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), f"{name} declared in fm.h but not exported"
    from paper_1710_09578_amd import capi

    assert set(names) == set(capi.SIGNATURES), "binding and header disagree"


def test_version(lib):
    from paper_1710_09578_amd import capi

    assert capi.fm_version() == "0.1.0"


def st(lib, name, *args):
    return getattr(lib, name)(*args)


def test_invalid_arguments_return_status(lib):
    h = C.c_void_p()
    assert st(lib, "fm_op_create_fourier", None, 8, 1) == 1          # NULL out
    assert st(lib, "fm_op_create_fourier", C.byref(h), 8, 99) == 1   # bad dtype
    assert st(lib, "fm_op_create_fourier", C.byref(h), 8, 3) == 3    # integer Fourier
    assert st(lib, "fm_op_create_fourier", C.byref(h), (1 << 19) + 1, 1) == 5   # too long for Bluestein
    assert st(lib, "fm_op_create_lfsr_circulant", C.byref(h), 4, 0, 1, 1, None) == 1  # no taps
    assert st(lib, "fm_op_create_lfsr_circulant", C.byref(h), 4, 3, 0, 1, None) == 1  # zero state
    assert st(lib, "fm_op_create_lfsr_circulant", C.byref(h), 30, 3, 1, 1, None) == 5  # order too large
    assert st(lib, "fm_op_conj", None, None) == 1
    assert st(lib, "fm_op_calibrate", None, 16, None, None, None, None) == 1
    assert st(lib, "fm_op_set_path", C.c_void_p(0x1000), 0) == 9
    assert st(lib, "fm_op_gram", C.byref(h), C.c_void_p(0x1000)) == 9
    assert st(lib, "fm_op_inverse", C.byref(h), None) == 1
    assert st(lib, "fm_op_create_fourier", C.byref(h), 0, 1) == 5
    assert st(lib, "fm_op_create_circulant", C.byref(h), 8, None, 1, None) == 1
    assert st(lib, "fm_op_create_toeplitz", C.byref(h), 0, 4, None, None, 1, None) == 1
    assert st(lib, "fm_op_create_dense", C.byref(h), 4, 4, C.c_void_p(16), 3, 1, None) == 2  # lda < m
    assert st(lib, "fm_op_create_select_rows", C.byref(h), 4, 5, C.c_void_p(16), 1, None) == 2  # m > n
    assert st(lib, "fm_op_create_mltoeplitz", C.byref(h), 4, None, None, 1, None) == 5
    assert st(lib, "fm_op_compose", C.byref(h), 0, 0, None) == 1
    assert st(lib, "fm_op_create_blocks", C.byref(h), 0, 2, None) == 1    # empty grid
    assert st(lib, "fm_op_create_blocks", None, 1, 1, None) == 1          # NULL out
    assert st(lib, "fm_op_create_blocks", C.byref(h), 2, 2, (C.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)) == 9
    assert st(lib, "fm_op_release", None) == 1
    # a pointer that was never a handle
    bogus = C.c_void_p(0x1000)
    assert st(lib, "fm_op_release", bogus) == 9
    assert st(lib, "fm_op_shape", bogus, None, None, None) == 9
    assert st(lib, "fm_apply", None, 0, 1, None, 1, None, 1, None, 0, None) == 1
    size = C.c_size_t()
    assert st(lib, "fm_workspace_size", bogus, 0, 1, C.byref(size)) == 9
    msg = lib.fm_last_error().decode()
    assert "released" in msg
    # differentiation helpers
    assert st(lib, "fm_circulant_grad_generator", 16, 1, 0, None, 16, None, 16, None, 0, 3, None) == 3  # int dtype
    assert st(lib, "fm_circulant_grad_generator", 12, 1, 0, None, 12, None, 12, C.c_void_p(16), 0, 1, None) == 5
    assert st(lib, "fm_circulant_grad_generator", 16, 1, 7, None, 16, None, 16, None, 0, 1, None) == 1  # direction
    assert st(lib, "fm_fista_step", 8, 1, None, None, None, None, None, None, 4, None,
              C.c_double(1.0), 0, 1, 1, None) == 2  # ld < n
    assert st(lib, "fm_fista_step", 8, 1, None, None, None, None, None, None, 8, None,
              C.c_double(0.0), 0, 1, 1, None) == 1  # L <= 0
    assert st(lib, "fm_fista_step", 8, 1, None, None, None, None, None, None, 8, None,
              C.c_double(1.0), -1, 1, 1, None) == 1  # negative iteration index
    assert st(lib, "fm_fista_step_vjp", 8, 1, None, None, None, None, None, None, 8, None,
              C.c_double(1.0), 0, 1, 4, None) == 3  # integer dtype
    # momentum weights: the oracle's sequence (no GPU needed)
    from oracle import fista as ofista

    beta = C.c_double()
    _, ref = ofista.momentum_sequence(40)
    for k in (0, 1, 2, 7, 39):
        assert st(lib, "fm_fista_momentum", k, 1, C.byref(beta)) == 0 and abs(beta.value - ref[k]) <= 1e-15
    assert st(lib, "fm_fista_momentum", 5, 0, C.byref(beta)) == 0 and beta.value == 0.0
    assert st(lib, "fm_fista_momentum", -1, 1, C.byref(beta)) == 1
    assert st(lib, "fm_axpby", 8, 1, C.c_double(1.0), None, 4, C.c_double(1.0), None, 8, None, 8, 1, None) == 2
    assert st(lib, "fm_op_norm_bound", None, None, None) == 1
    assert st(lib, "fm_omp", None, 1, None, 8, 4, C.c_double(0.0), None, 8, None, None, None, 0, None) == 1
    assert st(lib, "fm_omp", bogus, 1, None, 8, 4, C.c_double(0.0), None, 8, None, None, None, 0, None) == 9
    assert st(lib, "fm_omp_workspace_size", None, 1, 4, C.byref(size)) == 1
    assert st(lib, "fm_op_norm_bound", bogus, None, None) == 9
    # batch schedule / tuner
    from paper_1710_09578_amd import capi

    sc = capi.fm_batch_schedule()
    assert st(lib, "fm_batch_get_schedule", None, C.byref(sc)) == 1
    assert st(lib, "fm_batch_get_schedule", bogus, C.byref(sc)) == 9
    assert st(lib, "fm_batch_set_schedule", bogus, C.byref(sc)) == 9
    assert st(lib, "fm_batch_tune", None, 0, None, None, None, None, 1, None, None) == 1
    assert st(lib, "fm_batch_apply", bogus, 0, None, None, None, None, None) == 9


def test_binding_raises(lib):
    from paper_1710_09578_amd import capi

    with pytest.raises(capi.FmError) as e:
        capi.fm_op_create_fourier(3 << 19, capi.FM_C64)
    assert e.value.code == "FM_E_UNSUPPORTED"
