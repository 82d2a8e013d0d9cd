"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/lobpcg.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_2109_00485_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lobpcg_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2109_00485_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_defaults(lib):
    for code in (L.OK, L.EINVAL, L.ENOMEM, L.EHIP, L.ENOTSPD, L.ENOCONV, L.ENONFINITE, L.EUNSUPPORTED):
        assert lib.lobpcg_strerror(code)
    o = L.default_opts()
    assert (o.dtype, o.gram, o.format, o.tile, o.kmax) == (L.F32, L.GRAM_AUTO, L.FORMAT_AUTO, 64, 16)
    assert o.tau_rel == 1e-3 and o.eps_rel == 1e-5


def test_create_rejects_bad_arguments_on_host(lib):
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(64)  # never dereferenced: the checks below fail first
    assert lib.lobpcg_create(None, 10, fake, fake, fake, None, None) == L.EINVAL
    assert lib.lobpcg_create(ctypes.byref(h), 0, fake, fake, fake, None, None) == L.EINVAL
    assert lib.lobpcg_create(ctypes.byref(h), 1 << 31, fake, fake, fake, None, None) == L.EINVAL
    assert lib.lobpcg_create(ctypes.byref(h), 10, None, fake, fake, None, None) == L.EINVAL
    for field, value, code in (("dtype", 3, L.EINVAL), ("kmax", 17, L.EINVAL), ("kmax", 0, L.EINVAL),
                               ("gram", 9, L.EINVAL), ("format", 5, L.EINVAL), ("tile", 32, L.EUNSUPPORTED),
                               ("tau_rel", 0.0, L.EINVAL), ("eps_rel", -1.0, L.EINVAL)):
        o = L.default_opts()
        setattr(o, field, value)
        assert lib.lobpcg_create(ctypes.byref(h), 10, fake, fake, fake, ctypes.byref(o), None) == code, field
    o = L.default_opts()
    o.dtype, o.gram = L.F64, L.GRAM_BF16X3
    assert lib.lobpcg_create(ctypes.byref(h), 10, fake, fake, fake, ctypes.byref(o), None) == L.EINVAL
    assert not h.value


def test_entry_points_reject_null_context(lib):
    fake = ctypes.c_void_p(64)
    assert lib.lobpcg_spmm_sym(None, fake, fake, 8, None) == L.EINVAL
    assert lib.lobpcg_precond_apply(None, fake, fake, fake, 8, 1, None) == L.EINVAL
    assert lib.lobpcg_gram(None, fake, 8, fake, 8, fake, 0, None) == L.EINVAL
    assert lib.lobpcg_solve(None, 8, 5, fake, fake, None, 1e-6, 10, 1, None, None) == L.EINVAL
    assert lib.lobpcg_query(None, None, None, None, None, None) == L.EINVAL
    assert lib.lobpcg_last_error(None) == b"null context"
    lib.lobpcg_destroy(None)
    assert lib.lobpcg_set_precond_offset(None, 1.0) == L.EINVAL
    assert lib.lobpcg_cholqr(None, fake, 8, 1, None, None) == L.EINVAL
    assert lib.lobpcg_orthonormalize(None, fake, fake, 8, None, None) == L.EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; asking for more exits with a message, before
    any device is touched."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_counter_summary_parses():
    """The FETCH/WRITE counter summary that bench.py turns into roofline.traffic
    is readable and gives a positive byte count per product (it is reported as
    null instead when the sparse-product source has changed since)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t, note = bench.counter_traffic("tiled_2m", 8)
    if t is None:
        assert note == "kernel sources changed since the counters were taken"
    else:
        assert 3.3e9 < t < 1e11 and note["fetch_scale"] > 0 and note["write_scale"] > 0
