"""CPU checks of the C ABI: the library loads, exports every function that
include/pgdto.h declares, and its struct layouts match the Python binding.
No compute calls are made here (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgdto.h")
LIB = os.environ.get("PGDTO_LIB") or os.path.join(ROOT, "paper_2511_13905_amd", "libpgdto.so")


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
    assert L.pgdto_version() == 8
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


def _problem(N, kind="single", m=1, n=1000, dtype=0, lda=None, b=None, offsets=None, C=float("inf"),
             lo=1e-3, hi=1.0, eq=0, y=0x100000, A=0x200000, x=0x300000, mask=None, lam0=None):
    """A problem struct with fake (never dereferenced) device addresses."""
    p = N.Problem()
    p.kind = N.KINDS[kind]
    p.dtype = dtype
    p.n = n
    p.m = m
    p.y, p.A, p.x = y, A, x
    p.lda = n if lda is None else lda
    keep = [(ctypes.c_double * m)(*(b if b is not None else [0.5] * m))]
    p.b = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_double))
    if offsets is not None:
        keep.append((ctypes.c_int64 * len(offsets))(*offsets))
        p.block_offsets = ctypes.cast(keep[-1], ctypes.POINTER(ctypes.c_int64))
    p.lo, p.hi, p.C = lo, hi, C
    p.free_mask = mask
    p.eq_mask = eq
    if lam0 is not None:
        keep.append((ctypes.c_double * m)(*lam0))
        p.lambda0 = ctypes.cast(keep[-1], ctypes.POINTER(ctypes.c_double))
    return p, keep


def test_host_validation_without_a_device():
    """pgdto_problem_check: the host-side argument rules, with no GPU."""
    from paper_2511_13905_amd import _native as N
    L = N.lib()
    chk = lambda **kw: L.pgdto_problem_check(ctypes.byref(_problem(N, **kw)[0]), None)
    assert chk() == N.OK
    assert chk(kind="coupled", m=3, lda=1000) == N.OK
    assert chk(kind="coupled", m=3, lda=1001) == N.ERR_ARG            # rows not 16-byte aligned
    assert chk(kind="coupled", m=3, lda=999) == N.ERR_ARG             # lda < n
    assert chk(kind="coupled", m=9, lda=1000) == N.OK                 # the wide coupled kernel
    assert chk(kind="coupled", m=64, lda=1000, b=[0.5] * 64) == N.OK
    assert chk(kind="coupled", m=65, lda=1000, b=[0.5] * 65) == N.ERR_ARG   # m > PGDTO_MAX_M
    assert chk(kind="coupled", m=9, lda=1000, dtype=N.F64) == N.ERR_ARG     # beyond 8 rows: float32 only
    assert chk(kind="coupled", m=8, lda=1000, dtype=N.F64) == N.OK
    assert chk(kind="coupled", m=64, lda=1000, b=[0.5] * 64, eq=1 << 63) == N.OK
    assert chk(kind="single", m=2) == N.ERR_ARG
    assert chk(n=0) == N.ERR_ARG
    assert chk(y=0x100004) == N.ERR_ARG                               # misaligned y
    assert chk(x=0x200000) == N.ERR_ARG                               # x aliases A
    assert chk(mask=0x400002) == N.ERR_ARG                            # misaligned mask
    assert chk(lo=1.0, hi=1.0) == N.ERR_ARG
    assert chk(lo=float("nan")) == N.ERR_ARG
    assert chk(b=[float("nan")]) == N.ERR_ARG and chk(b=[float("inf")]) == N.ERR_ARG   # b finite
    # C: > 0 or INFINITY; < 0 asks for the automatic penalty; 0, NaN, -INFINITY rejected
    assert chk(C=1e12) == N.OK and chk(C=-1e-6) == N.OK
    assert chk(C=0.0) == N.ERR_ARG and chk(C=float("nan")) == N.ERR_ARG and chk(C=float("-inf")) == N.ERR_ARG
    # equality rows: bits below m only
    assert chk(eq=1) == N.OK and chk(eq=2) == N.ERR_ARG
    assert chk(kind="coupled", m=3, lda=1000, eq=0b101) == N.OK
    assert chk(kind="coupled", m=3, lda=1000, eq=0b1000) == N.ERR_ARG
    # warm start: finite; >= 0 unless the row is an equality
    assert chk(lam0=[0.25]) == N.OK and chk(lam0=[0.0]) == N.OK
    assert chk(lam0=[-0.25]) == N.ERR_ARG and chk(lam0=[float("nan")]) == N.ERR_ARG
    assert chk(lam0=[float("inf")]) == N.ERR_ARG
    assert chk(lam0=[-0.25], eq=1) == N.OK
    assert chk(kind="coupled", m=3, lda=1000, lam0=[1.0, -2.0, 0.0], eq=0b010) == N.OK
    assert chk(kind="coupled", m=3, lda=1000, lam0=[1.0, -2.0, 0.0], eq=0b001) == N.ERR_ARG
    # independent blocks: offsets from 0 to n, strictly increasing
    assert chk(kind="independent", m=2, offsets=[0, 400, 1000]) == N.OK
    assert chk(kind="independent", m=2, offsets=[0, 400, 999]) == N.ERR_ARG
    assert chk(kind="independent", m=2, offsets=[0, 0, 1000]) == N.ERR_ARG
    assert chk(kind="independent", m=2, offsets=[1, 400, 1000]) == N.ERR_ARG
    # params
    p, keep = _problem(N)
    prm = N.Params()
    L.pgdto_params_default(ctypes.byref(prm))
    assert L.pgdto_problem_check(ctypes.byref(p), ctypes.byref(prm)) == N.OK
    prm.tol_n = 0.0
    assert L.pgdto_problem_check(ctypes.byref(p), ctypes.byref(prm)) == N.ERR_ARG


C_PROGRAM = r"""
#include <math.h>
#include <stdio.h>
#include "pgdto.h"
int main(void) {
  pgdto_ctx* ctx = NULL;
  if (pgdto_ctx_create(0, &ctx) != PGDTO_OK) return 1;
  const int64_t n = 1024;
  double b[1] = {0.5};
  pgdto_problem p = {PGDTO_SINGLE, PGDTO_F32, n, 1, (void*)0, (void*)0, n, NULL, b, 1e-3, 1.0, INFINITY,
                     (void*)0, NULL, 0};
  pgdto_params prm;
  pgdto_params_default(&prm);
  printf("%d\n", pgdto_problem_check(&p, &prm));
  pgdto_result res;
  int st = pgdto_project(ctx, &p, &prm, &res, NULL);
  pgdto_ctx_destroy(ctx);
  return st == PGDTO_OK ? 0 : 2;
}
"""


def test_c_program_builds_against_the_header(tmp_path):
    """A C program (not C++) includes the header and links the library: the
    boundary is plain C.  Compiled and linked only; nothing is run."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(C_PROGRAM)
    out = tmp_path / "use"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(out), "-L", os.path.dirname(LIB), "-lpgdto", "-lm",
                        "-Wl,--unresolved-symbols=ignore-in-shared-libs"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises ImportError: there is no
    CPU fallback behind the product path."""
    from paper_2511_13905_amd import _native as N
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "libpgdto.so"))
    with pytest.raises(ImportError):
        N.lib()


def test_product_package_does_not_import_the_oracle():
    """The package (binding and API) loads without touching oracle/, which is
    test infrastructure only."""
    import subprocess
    import sys
    code = ("import sys; import paper_2511_13905_amd, paper_2511_13905_amd.api, paper_2511_13905_amd._native; "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "assert not bad, bad")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def test_tune_shape_count_matches_header():
    """The binding sizes the autotuner's timing array from the header's
    PGDTO_TUNE_SHAPES."""
    from paper_2511_13905_amd import api
    m = re.search(r"#define\s+PGDTO_TUNE_SHAPES\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == api.TUNE_SHAPES == len(api.TUNE_SLOTS)
