"""The C ABI: every function declared in include/gift.h is exported by the
built library, and the binding declares the same set (CPU only; no compute
call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gift.h")
LIB = os.path.join(ROOT, "paper_1604_01879_amd", "libgift.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"\b(gift_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libgift.so not built (run python -m paper_1604_01879_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_six_calls_of_the_problem_statement():
    names = declared_functions()
    for call in ("gift_build_codebook", "gift_build_fif", "gift_build_sif",
                 "gift_query_exhaustive", "gift_query_fif", "gift_rerank_sif"):
        assert call in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_function(lib):
    from paper_1604_01879_amd import _lib as L
    assert sorted(L.exported_symbols()) == declared_functions()


def test_version_and_error_strings(lib):
    lib.gift_version.restype = ctypes.c_char_p
    lib.gift_last_error.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gift_version()
    assert isinstance(lib.gift_last_error(), bytes)


def test_argument_errors_need_no_device(lib):
    # invalid arguments are rejected on the host before any device work
    lib.gift_rerank_sif.restype = ctypes.c_int32
    st = lib.gift_rerank_sif(ctypes.c_int64(0), None, None, None, None, 0, 0, None, None,
                             None, 0, None, None, None, None)
    assert st == -1
    lib.gift_last_error.restype = ctypes.c_char_p
    assert b"n_shapes" in lib.gift_last_error()


def test_copy_async_argument_errors_need_no_device(lib):
    # an empty copy does nothing, a null buffer is rejected on the host
    lib.gift_copy_async.restype = ctypes.c_int32
    lib.gift_copy_async.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]
    assert lib.gift_copy_async(None, None, 0, None) == 0
    assert lib.gift_copy_async(None, 1 << 20, 8, None) == -1
    assert lib.gift_copy_async(1 << 20, None, 8, None) == -1


def test_plan_serve_argument_errors_need_no_device(lib):
    # a null plan or host buffer is rejected on the host, before any copy
    P = ctypes.c_void_p
    lib.gift_fif_plan_serve.restype = ctypes.c_int32
    lib.gift_fif_plan_serve.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        P, P, P, P, P, ctypes.c_int32, P, P, P, P, P, P, P]
    tail = (0, None, None, None, None, None, 0, None, None, None)
    assert lib.gift_fif_plan_serve(None, 1 << 20, 1 << 20, 1, 8, *tail, 1 << 20, 1 << 20,
                                   None, None) == -1
    assert lib.gift_fif_plan_serve(1 << 20, None, 1 << 20, 1, 8, *tail, 1 << 20, 1 << 20,
                                   None, None) == -1
    assert lib.gift_fif_plan_serve(1 << 20, 1 << 20, 1 << 20, 1, 8, *tail, None, 1 << 20,
                                   None, None) == -1


def test_static_scratch_capacity_needs_no_device(lib):
    # gift_query_exhaustive_static sizes its batch against the 64 MiB static
    # scratch on the host: a batch too large for it fails with
    # GIFT_ECAPACITY before any device call (the pointers are never touched)
    from paper_1604_01879_amd import _lib as L
    fake = 1 << 20  # aligned, never dereferenced
    q = L.gift_queries(fake, fake, 1, 64, 64)
    sizes = {}
    for n in (200_000, 250_000, 260_000, 300_000):
        v = L.gift_views(fake, L.F32, 64, n, 4096, 0, None, fake)
        sizes[n] = L._lib.gift_query_exhaustive_static_bytes(ctypes.byref(v), ctypes.byref(q),
                                                             100, 200)
    # one 64-view query: 260 bytes per shape (match buffer + score row)
    assert sizes[250_000] <= L.STATIC_SCRATCH_BYTES < sizes[260_000]
    v = L.gift_views(fake, L.F32, 64, 300_000, 4096, 0, None, fake)
    st = L._lib.gift_query_exhaustive_static(ctypes.byref(v), ctypes.byref(q), 100, 200,
                                             None, None, None, None)
    assert st == L.ECAPACITY
    assert b"static scratch" in L._lib.gift_last_error()
