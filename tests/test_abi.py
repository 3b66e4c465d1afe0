"""CPU checks of the C ABI: the library loads, exports every function that
include/pgdto.h declares, and its struct layouts match the Python binding.
No compute calls are made here (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgdto.h")
LIB = os.path.join(ROOT, "paper_2511_13905_amd", "libpgdto.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(pgdto_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pgdto_project", "pgdto_project_async", "pgdto_pgd_step", "pgdto_batch_create",
                 "pgdto_batch_submit", "pgdto_batch_poll", "pgdto_batch_destroy", "pgdto_ctx_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libpgdto.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_binding():
    from paper_2511_13905_amd import _native as N
    L = N.lib()
    for i, S in enumerate(N.STRUCTS):
        assert L.pgdto_struct_size(i) == ctypes.sizeof(S), S.__name__
    assert L.pgdto_version() == 2
    assert N.status_string(N.ERR_ARG) == "invalid argument"


def test_null_arguments_are_rejected_without_a_device():
    from paper_2511_13905_amd import _native as N
    L = N.lib()
    r = N.Result()
    assert L.pgdto_project(None, None, None, ctypes.byref(r), None) == N.ERR_ARG
    assert L.pgdto_ctx_create(0, None) == N.ERR_ARG
    assert L.pgdto_batch_poll(None, 1, ctypes.byref(r)) == N.ERR_ARG
    p = N.Params()
    L.pgdto_params_default(ctypes.byref(p))
    assert p.tol_b == 1e-8 and p.max_newton == 50 and p.c1 == 1e-4 and p.c2 == 0.9
