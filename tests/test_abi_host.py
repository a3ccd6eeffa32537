"""The C ABI on a host without a GPU: the library loads, exports every symbol
include/caqr.h declares, and validates arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1303_5837_amd import caqr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "caqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:caqr_status_t|const char \*|int)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["tsqr_factor", "caqr_factor", "apply_q", "ls_solve", "caqr_create", "caqr_destroy",
                     "caqr_sync", "caqr_factors_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = caqr.library()
    names = declared_functions()
    assert names
    out = subprocess.run(["nm", "-D", "--defined-only", caqr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    for n in names:
        assert n in exported, n
        assert getattr(lib, n) is not None
    assert set(caqr.EXPORTS) <= set(names)


def _no_gpu():
    return caqr.device_count() == 0


def test_create_without_device():
    if not _no_gpu():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p(1)
    assert caqr.library().caqr_create(ctypes.byref(h), 0) == 3  # CAQR_ERR_DEVICE
    assert not h.value


def test_status_strings():
    lib = caqr.library()
    for code in range(8):
        assert lib.caqr_status_string(code)
    assert b"unknown" in lib.caqr_status_string(99)


def _tsqr(m, n, A, lda, opts=None, F=True, h=None):
    f = ctypes.c_void_p()
    return caqr.library().tsqr_factor(h, m, n, A, lda, opts, ctypes.byref(f) if F else None)


def test_argument_validation_without_device():
    lib = caqr.library()
    A = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
    assert _tsqr(10, 20, A, 10) == 4  # m < n: NOT_SUPPORTED
    assert _tsqr(-1, 2, A, 10) == 1
    assert _tsqr(10, 2, A, 9) == 1  # lda < m
    assert _tsqr(10, 2, None, 10) == 1  # A NULL with n > 0
    assert _tsqr(10, 2, A, 10, F=False) == 1
    assert _tsqr(10, 2, A, 10) == 1  # valid sizes, NULL handle
    bad = caqr.TreeOpts(100, 0, 0, 0)
    assert _tsqr(10, 2, A, 10, ctypes.byref(bad)) == 1
    bad = caqr.TreeOpts(256, 3, 0, 0)
    assert _tsqr(10, 2, A, 10, ctypes.byref(bad)) == 1
    f = ctypes.c_void_p()
    assert lib.caqr_factor(None, 100, 100, 0, A, 100, None, ctypes.byref(f)) == 1  # nb = 0
    assert lib.caqr_factor(None, 100, 100, 65, A, 100, None, ctypes.byref(f)) == 1  # nb > 64
    assert lib.caqr_factor(None, 10, 100, 64, A, 10, None, ctypes.byref(f)) == 4
    assert lib.apply_q(None, None, 2, 1, A, 10) == 1  # bad op
    assert lib.apply_q(None, None, 1, 1, A, 10) == 1  # NULL handle / factors
    assert lib.ls_solve(None, 5, 6, 1, A, 5, A, 5, None, None) == 4
    assert lib.ls_solve(None, 6, 5, -1, A, 6, A, 6, None, None) == 1
    assert lib.ls_solve(None, 6, 5, 1, A, 6, A, 5, None, None) == 1  # ldb < m
    assert lib.ls_solve(None, 6, 5, 1, A, 6, A, 6, None, None) == 1  # NULL handle
    assert lib.caqr_sync(None) == 1
    assert lib.caqr_destroy(None) == 1
    assert lib.caqr_factors_destroy(None) == 1


def test_batched_argument_validation_without_device():
    """tsqr_factor_batched checks every problem before the handle."""
    lib = caqr.library()
    A = ctypes.c_void_p(0x1000)

    def call(m, n, ld, ptrs=None, dt=caqr.F64, opts=None, batch=None, F=True):
        k = len(m) if batch is None else batch
        M = (ctypes.c_int64 * max(1, len(m)))(*m)
        N = (ctypes.c_int64 * max(1, len(n)))(*n)
        LD = (ctypes.c_int64 * max(1, len(ld)))(*ld)
        P = (ctypes.c_void_p * max(1, len(m)))(*(ptrs if ptrs is not None else [A.value] * len(m)))
        f = ctypes.c_void_p()
        return lib.tsqr_factor_batched(None, k, M, N, P, LD, dt, opts, ctypes.byref(f) if F else None)

    assert call([10, 20], [2, 3], [10, 20], batch=-1) == 1          # negative batch
    assert call([10], [2], [10], F=False) == 1                        # no output pointer
    assert call([10, 20], [2, 3], [9, 20]) == 1                       # lda < m
    assert call([10, 20], [2, 3], [10, 20], ptrs=[A.value, None]) == 1  # NULL A with n > 0
    assert call([10, 20], [2, 0], [10, 20], ptrs=[A.value, None]) == 1  # n = 0 may be NULL: only the handle fails
    assert call([10, 20], [2, 30], [10, 20]) == 4                     # m < n
    assert call([100], [65], [100]) == 4                              # n > 64
    assert call([100], [8], [100], dt=caqr.F32) == 1                  # FP32 valid: NULL handle
    assert call([100], [8], [100], dt=7) == 1                         # unknown dtype
    bad = caqr.TreeOpts(100, 0, 0, 0)
    assert call([100], [8], [100], opts=ctypes.byref(bad)) == 1       # leaf_rows not 64/128/256
    assert call([100, 300], [8, 64], [100, 300]) == 1                 # valid: NULL handle
    assert call([], [], [], batch=0) == 1                             # empty batch, NULL handle
    assert lib.caqr_batch_destroy(None) == 0
    assert lib.caqr_batch_get_plan(None, 0, None) == 1
    assert lib.caqr_batch_get_signs(None, 0, None) == 1
    assert lib.caqr_tune_batched(None, caqr.F64) == 1
    assert lib.caqr_batch_plan_for(None, 100, 8, caqr.F64, None) == 1


def test_server_argument_validation_without_device():
    """caqr_server_create / submit check their arguments before the device."""
    lib = caqr.library()
    S = ctypes.c_void_p()
    bad = [caqr.ServerOpts(0, 0, 1 << 20, 0), caqr.ServerOpts(0, 65, 1 << 20, 0),
           caqr.ServerOpts(0, 2, 100, 0), caqr.ServerOpts(0, 2, 1 << 20, 1)]
    for o in bad:
        assert lib.caqr_server_create(ctypes.byref(o), ctypes.byref(S)) == 1
    assert lib.caqr_server_create(None, ctypes.byref(S)) == 1
    assert lib.caqr_server_create(ctypes.byref(caqr.ServerOpts(0, 2, 1 << 20, 0)), None) == 1
    if caqr.device_count() == 0:
        assert lib.caqr_server_create(ctypes.byref(caqr.ServerOpts(0, 2, 1 << 20, 0)), ctypes.byref(S)) == 3
    p = ctypes.c_void_p(0x1000)
    t = ctypes.c_int64()
    sub = lib.caqr_server_submit
    st = ctypes.c_void_p(0)  # no ordering stream
    assert sub(None, 100, 10, 1, p, 100, p, 100, p, 10, st, ctypes.byref(t)) == 1   # valid request, NULL server
    assert sub(None, 100, 10, 1, p, 99, p, 100, p, 10, st, ctypes.byref(t)) == 1    # lda < m
    assert sub(None, 100, 10, 1, p, 100, p, 100, p, 9, st, ctypes.byref(t)) == 1    # ldx < n
    assert sub(None, 100, 10, 1, None, 100, p, 100, p, 10, st, ctypes.byref(t)) == 1  # NULL A
    assert sub(None, 10, 20, 1, p, 10, p, 10, p, 20, st, ctypes.byref(t)) == 4      # m < n
    assert sub(None, 100, 10, 1, p, 100, p, 100, p, 10, st, None) == 1              # NULL ticket
    assert lib.caqr_server_wait(None, 1, None, None) == 1
    assert lib.caqr_server_destroy(None) == 1


def test_batched_ls_argument_validation_without_device():
    """ls_solve_batched checks every problem before the handle."""
    lib = caqr.library()
    P = ctypes.c_void_p(0x1000)

    def call(m, n, r, lda=None, ldb=None, pa=True, pb=True, batch=None, info=True, opts=None):
        k = len(m) if batch is None else batch
        arr = lambda v: (ctypes.c_int64 * max(1, len(v)))(*v)
        ptrs = lambda ok: (ctypes.c_void_p * max(1, len(m)))(*([P.value if ok else None] * len(m)))
        inf = (caqr.LsInfo * max(1, len(m)))()
        return lib.ls_solve_batched(None, k, arr(m), arr(n), arr(r), ptrs(pa), arr(lda or m), ptrs(pb),
                                    arr(ldb or m), opts, inf if info else None)

    assert call([100], [10], [1], batch=-1) == 1                 # negative batch
    assert call([100], [10], [1], info=False) == 1                # no info array
    assert call([100], [10], [-1]) == 1                           # negative nrhs
    assert call([100], [10], [1], lda=[99]) == 1                  # lda < m
    assert call([100], [10], [1], ldb=[99]) == 1                  # ldb < m
    assert call([100], [10], [1], pa=False) == 1                  # NULL A
    assert call([100], [10], [1], pb=False) == 1                  # NULL B
    assert call([100], [65], [1]) == 4                            # n > 64
    assert call([10], [20], [1]) == 4                             # m < n
    bad = caqr.TreeOpts(100, 0, 0, 0)
    assert call([100], [10], [1], opts=ctypes.byref(bad)) == 1    # invalid plan
    assert call([100, 50], [10, 0], [1, 3]) == 1                  # valid: NULL handle


def test_inner_block_validation_without_device():
    """inner_block: 0, 16, 32 or 64 for the single factorizations; the batched
    calls accept only 0 (NOT_SUPPORTED otherwise, after every argument check)."""
    lib = caqr.library()
    A = ctypes.c_void_p(0x1000)
    for ib in (0, 16, 32, 64):  # valid: the NULL handle is what fails
        assert _tsqr(100, 40, A, 100, ctypes.byref(caqr.TreeOpts(0, 0, ib, 0))) == 1
        f = ctypes.c_void_p()
        o = caqr.TreeOpts(0, 0, ib, 0)
        assert lib.caqr_factor(None, 100, 100, 64, A, 100, ctypes.byref(o), ctypes.byref(f)) == 1
    for ib in (8, 24, 48, -16, 128, 1):
        assert _tsqr(100, 40, A, 100, ctypes.byref(caqr.TreeOpts(0, 0, ib, 0))) == 1
    assert _tsqr(10, 20, A, 10, ctypes.byref(caqr.TreeOpts(0, 0, 16, 0))) == 4  # m < n still NOT_SUPPORTED
    assert _tsqr(100, 40, A, 100, ctypes.byref(caqr.TreeOpts(0, 0, 16, 7))) == 1  # arity 7 is invalid
    assert _tsqr(100, 40, A, 100, ctypes.byref(caqr.TreeOpts(0, 0, 16, 4))) == 4  # inner blocks need arity 2
    assert _tsqr(100, 40, A, 100, ctypes.byref(caqr.TreeOpts(0, 0, 16, 2))) == 1  # valid: the NULL handle fails
    M = (ctypes.c_int64 * 1)(100)
    N = (ctypes.c_int64 * 1)(8)
    P = (ctypes.c_void_p * 1)(A.value)
    f = ctypes.c_void_p()
    o = caqr.TreeOpts(0, 0, 16, 0)
    assert lib.tsqr_factor_batched(None, 1, M, N, P, M, caqr.F64, ctypes.byref(o), ctypes.byref(f)) == 4
    o = caqr.TreeOpts(0, 0, 24, 0)
    assert lib.tsqr_factor_batched(None, 1, M, N, P, M, caqr.F64, ctypes.byref(o), ctypes.byref(f)) == 1
    R = (ctypes.c_int64 * 1)(1)
    inf = (caqr.LsInfo * 1)()
    o = caqr.TreeOpts(0, 0, 32, 0)
    assert lib.ls_solve_batched(None, 1, M, N, R, P, M, P, M, ctypes.byref(o), inf) == 4


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says why."""
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_arity_validation_without_device():
    """arity: 0 (default), 2 or 4; leaves_per_wg a power of the arity (2 selects
    the binary tree when arity is left open)."""
    A = ctypes.c_void_p(0x1000)
    for ar, lpw in ((0, 0), (2, 1), (2, 2), (2, 4), (4, 1), (4, 4), (0, 2), (0, 4)):
        assert _tsqr(1000, 40, A, 1000, ctypes.byref(caqr.TreeOpts(0, lpw, 0, ar))) == 1, (ar, lpw)  # NULL handle
    for ar, lpw in ((3, 0), (8, 0), (-2, 0), (1, 0), (4, 2)):
        assert _tsqr(1000, 40, A, 1000, ctypes.byref(caqr.TreeOpts(0, lpw, 0, ar))) == 1, (ar, lpw)
    lib = caqr.library()
    M = (ctypes.c_int64 * 1)(100)
    N = (ctypes.c_int64 * 1)(8)
    P = (ctypes.c_void_p * 1)(A.value)
    f = ctypes.c_void_p()
    assert lib.tsqr_factor_batched(None, 1, M, N, P, M, caqr.F64, ctypes.byref(caqr.TreeOpts(0, 4, 0, 4)),
                                   ctypes.byref(f)) == 1  # valid arity-4 plan: the NULL handle fails
    assert lib.tsqr_factor_batched(None, 1, M, N, P, M, caqr.F64, ctypes.byref(caqr.TreeOpts(0, 2, 0, 4)),
                                   ctypes.byref(f)) == 1  # two leaves per workgroup with arity 4: invalid


def test_ls_options_validation_without_device():
    """caqr_ls_opts_t: precision 0 or 1, max_iter >= 0, tol >= 0, no_fallback 0
    or 1, reserved 0 (checked before the sizes' NOT_SUPPORTED, so an m < n call
    separates a bad option, 1, from a good one, 4)."""
    lib = caqr.library()
    A = ctypes.c_void_p(0x1000)
    good = [caqr.LsOpts(0, 0, 0.0, 0, 0), caqr.LsOpts(1, 0, 0.0, 0, 0), caqr.LsOpts(1, 50, 1e-10, 1, 0)]
    bad = [caqr.LsOpts(2, 0, 0.0, 0, 0), caqr.LsOpts(1, -1, 0.0, 0, 0), caqr.LsOpts(1, 0, -1e-12, 0, 0),
           caqr.LsOpts(1, 0, float("nan"), 0, 0), caqr.LsOpts(1, 0, 0.0, 2, 0), caqr.LsOpts(1, 0, 0.0, 0, 3)]
    for o in good:
        assert lib.ls_solve(None, 5, 6, 1, A, 5, A, 5, ctypes.byref(o), None) == 4
    for o in bad:
        assert lib.ls_solve(None, 5, 6, 1, A, 5, A, 5, ctypes.byref(o), None) == 1
