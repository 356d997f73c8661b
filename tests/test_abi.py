"""The C ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastfca.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastfca_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["fastfca_init", "fastfca_em_step", "fastfca_loglik", "fastfca_mwf",
                     "fastfca_get_params", "fastfca_destroy", "fastfca_last_error",
                     "fastfca_init_batch", "fastfca_autotune"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2101_08563_amd import fastfca
    if not os.path.exists(fastfca.LIB_PATH):
        pytest.skip("libfastfca.so not built")
    lib = fastfca.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding describes exactly the declared entry points
    assert sorted(fastfca.SIGNATURES) == declared_functions()


def test_last_error_without_context_is_callable():
    from paper_2101_08563_amd import fastfca
    if not os.path.exists(fastfca.LIB_PATH):
        pytest.skip("libfastfca.so not built")
    lib = fastfca.load_library()
    assert isinstance(lib.fastfca_last_error(None), bytes)


def test_invalid_shapes_rejected_before_any_gpu_work():
    """Shape validation happens on the host before device allocation."""
    from paper_2101_08563_amd import fastfca
    if not os.path.exists(fastfca.LIB_PATH):
        pytest.skip("libfastfca.so not built")
    lib = fastfca.load_library()
    ctx = ctypes.c_void_p()
    for (F, T, M, N) in [(0, 10, 2, 3), (4, 10, 1, 3), (4, 10, 2, 1), (4, 1, 2, 3)]:
        rc = lib.fastfca_init(ctypes.byref(ctx), ctypes.c_void_p(16), F, T, M, N, None, None, None, 0, None)
        assert rc == fastfca.E_ARG
        assert ctx.value is None
    rc = lib.fastfca_init(ctypes.byref(ctx), ctypes.c_void_p(16), 4, 100, 9, 3, None, None, None, 0, None)
    assert rc == fastfca.E_UNSUPPORTED
    rc = lib.fastfca_init(ctypes.byref(ctx), None, 4, 100, 2, 3, None, None, None, 0, None)
    assert rc == fastfca.E_ARG
    assert b"NULL" in lib.fastfca_last_error(None)


def test_noalloc_entry_point_rejects_before_any_gpu_work():
    """fastfca_fit_noalloc validates its arguments and the size of its fixed
    device array on the host, before any HIP call."""
    from paper_2101_08563_amd import fastfca
    if not os.path.exists(fastfca.LIB_PATH):
        pytest.skip("libfastfca.so not built")
    lib = fastfca.load_library()
    p = ctypes.c_void_p(256)
    # missing status
    assert lib.fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 5, None, None, None) == fastfca.E_ARG
    # T < M, n_iter < 1
    assert lib.fastfca_fit_noalloc(p, 9, 1, 2, 3, p, p, p, 5, p, None, None) == fastfca.E_ARG
    assert lib.fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 0, p, None, None) == fastfca.E_ARG
    # no compiled kernel
    assert lib.fastfca_fit_noalloc(p, 9, 100, 9, 3, p, p, p, 5, p, None, None) == fastfca.E_UNSUPPORTED
    # the trace would not fit in the fixed array: 9 frequencies x 200000 doubles
    assert lib.fastfca_fit_noalloc(p, 9, 100, 2, 3, p, p, p, 200000, p, None, None) == fastfca.E_ARG
    assert b"scratch" in lib.fastfca_last_error(None)
