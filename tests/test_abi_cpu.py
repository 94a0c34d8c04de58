"""C-ABI library checks that need no GPU: it loads, exports every entry point
declared in include/chanflow.h, and rejects bad arguments before touching the
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2104_08863_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "chanflow.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cf_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"{n} missing from the Python binding"
    assert set(L.SIGNATURES) == set(names)


def test_status_strings_and_defaults():
    lib = L.lib()
    for s in range(6):
        assert lib.cf_status_string(s)
    assert lib.cf_status_string(L.CF_ERR_NUMERIC) == b"non-finite values"
    # the status path of the numeric check: a failure reaches the Python caller
    # as an exception carrying CF_ERR_NUMERIC and the library's message
    with pytest.raises(L.ChanflowError) as e:
        L.check(L.CF_ERR_NUMERIC, "cf_plan_numeric_status")
    assert e.value.status == L.CF_ERR_NUMERIC and "non-finite" in str(e.value)
    opt = L.cf_options()
    lib.cf_options_default(C.byref(opt))
    assert opt.precision == L.CF_FP64 and opt.n_parts == 0 and opt.refine_passes == 1
    assert opt.fp64_kx == 4 and opt.fp64_kz == 4 and opt.drop_tol < 0


def _create(nx, ny, nz, yf, opt=None, lx=1.0, lz=1.0):
    lib = L.lib()
    h = C.c_void_p(1234)
    yp = yf.ctypes.data_as(C.POINTER(C.c_double)) if yf is not None else None
    st = lib.cf_plan_create(C.byref(h), nx, ny, nz, lx, lz, yp, C.byref(opt) if opt else None)
    return st, h


@pytest.mark.parametrize("nx,ny,nz,why,code", [
    (63, 8, 8, "odd nx", L.CF_ERR_ARG),
    (2, 8, 8, "nx too small", L.CF_ERR_ARG),
    (14, 8, 8, "nx/2 = 7", L.CF_ERR_UNSUPPORTED),
    (16, 8, 10, "nz = 10", L.CF_ERR_UNSUPPORTED),
    (16, 8, 18, "nz = 18 (two factors of 3)", L.CF_ERR_UNSUPPORTED),
    (8192, 8, 8, "nx/2 above 2048", L.CF_ERR_UNSUPPORTED),
    (16, 1, 8, "ny = 1", L.CF_ERR_ARG),
    (16, 1031, 8, "ny = 1031 needs more than 64 partitions of at most 16 rows (FP64)", L.CF_ERR_UNSUPPORTED),
])
def test_plan_rejects_bad_sizes(nx, ny, nz, why, code):
    yf = np.linspace(-1, 1, max(ny, 1) + 1)
    st, h = _create(nx, ny, nz, yf)
    assert st == code, why
    assert h.value is None
    assert L.lib().cf_last_error()


def test_plan_rejects_bad_grid_and_options():
    yf = np.linspace(-1, 1, 9)
    bad = yf.copy()
    bad[4] = bad[3]
    assert _create(16, 8, 8, bad)[0] == L.CF_ERR_ARG
    bad = yf.copy()
    bad[2] = np.nan
    assert _create(16, 8, 8, bad)[0] == L.CF_ERR_ARG
    assert _create(16, 8, 8, None)[0] == L.CF_ERR_ARG
    assert _create(16, 8, 8, yf, lx=-1.0)[0] == L.CF_ERR_ARG
    opt = L.cf_options()
    L.lib().cf_options_default(C.byref(opt))
    opt.precision = 7
    assert _create(16, 8, 8, yf, opt)[0] == L.CF_ERR_ARG
    L.lib().cf_options_default(C.byref(opt))
    opt.n_parts = 5  # 5 partitions of ceil(8/5) = 2 rows: the fifth would hold only padding
    assert _create(16, 8, 8, yf, opt)[0] == L.CF_ERR_UNSUPPORTED
    L.lib().cf_options_default(C.byref(opt))
    opt.precision = L.CF_MIXED
    opt.refine_passes = -1
    assert _create(16, 8, 8, yf, opt)[0] == L.CF_ERR_ARG
    assert L.lib().cf_plan_create(None, 16, 8, 8, 1.0, 1.0, yf.ctypes.data_as(C.POINTER(C.c_double)), None) == L.CF_ERR_ARG


def test_plan_rejects_unsupported_y_transform_solve():
    opt = L.cf_options()
    L.lib().cf_options_default(C.byref(opt))
    opt.flags = L.CF_PLAN_Y_DCT
    yf = np.linspace(-1, 1, 17)
    stretched = np.tanh(2.0 * np.linspace(-1, 1, 17)) / np.tanh(2.0)
    assert _create(16, 16, 8, stretched, opt)[0] == L.CF_ERR_ARG            # not uniform
    assert _create(16, 3, 8, np.linspace(-1, 1, 4), opt)[0] == L.CF_ERR_UNSUPPORTED   # odd ny
    assert _create(16, 20, 8, np.linspace(-1, 1, 21), opt)[0] == L.CF_ERR_UNSUPPORTED  # 20 not 2^a, 3*2^a
    opt.precision = L.CF_MIXED
    assert _create(16, 16, 8, yf, opt)[0] == L.CF_ERR_UNSUPPORTED           # FP64 only


def test_plan_rejects_bad_partition_options():
    yf = np.linspace(-1, 1, 65)
    opt = L.cf_options()
    L.lib().cf_options_default(C.byref(opt))
    assert opt.lines_per_block == 0
    opt.flags = L.CF_PLAN_TUNE_PARTS
    opt.n_parts = 4
    assert _create(16, 64, 8, yf, opt)[0] == L.CF_ERR_ARG               # tuning with a fixed count
    opt.n_parts, opt.lines_per_block = 0, 16
    assert _create(16, 64, 8, yf, opt)[0] == L.CF_ERR_ARG               # tuning with a fixed block
    opt.lines_per_block = 0
    opt.flags = L.CF_PLAN_TUNE_PARTS | L.CF_PLAN_Y_DCT
    assert _create(16, 64, 8, yf, opt)[0] == L.CF_ERR_ARG               # no partitions to tune
    L.lib().cf_options_default(C.byref(opt))
    opt.lines_per_block = -1
    assert _create(16, 64, 8, yf, opt)[0] == L.CF_ERR_ARG
    opt.n_parts, opt.lines_per_block = 8, 128                           # 1024 threads per block
    assert _create(16, 64, 8, yf, opt)[0] == L.CF_ERR_ARG


def test_calls_reject_null_plan_and_pointers():
    lib = L.lib()
    buf = (C.c_double * 8)()
    p = C.cast(buf, C.c_void_p)
    assert lib.cf_poisson_solve(None, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_solve_spectral(None, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_solve_spectral_slabs(None, 1, p, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_forward_spectral(None, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_inverse_spectral(None, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_divergence(None, p, p, p, p, 1.0, None) == L.CF_ERR_ARG
    assert lib.cf_rk2_predictor(None, p, p, p, p, p, p, 1e-3, 0.01, 0.0, None) == L.CF_ERR_ARG
    assert lib.cf_plane_stats(None, p, p, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_run_steps(None, p, p, p, p, p, p, 1, 1e-3, 0.01, 0.0, 0, None, None, 0, None) == L.CF_ERR_ARG
    assert lib.cf_plan_query(None, None) == L.CF_ERR_ARG
    assert lib.cf_solve_spectral_slabs_noalloc(None, 1, p, p, None) == L.CF_ERR_ARG
    assert lib.cf_plan_numeric_status(None, None) == L.CF_ERR_ARG
    n = C.c_int(-1)
    assert lib.cf_plan_tuning(None, 0, C.byref(n), None, None, None) == L.CF_ERR_ARG
    lib.cf_plan_destroy(None)
