"""The C-ABI library loads and exports every entry point include/dbfft.h
declares (no GPU needed; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbfft.h")
LIB = os.path.join(ROOT, "paper_1905_12725_amd", "libdbfft.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dbfft_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dbfft_setup", "dbfft_apply", "dbfft_solve", "dbfft_homogenize", "dbfft_adjoint",
                     "dbfft_destroy", "dbfft_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_binding_names_match_header():
    from paper_1905_12725_amd import _native
    assert sorted(_native.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_default_opts_and_error_string_without_gpu():
    from paper_1905_12725_amd import _native
    o = _native.default_opts()
    assert o.tol == 1e-8 and o.tol_load == 1e-10 and o.max_iter == 10000
    assert o.newton_tol == 1e-6
    lib = _native.lib()
    assert isinstance(lib.dbfft_last_error(), bytes)
    assert o.fused_cg == 1 and o.graph == 1 and o.checkpoint == 0


def test_opts_binding_has_the_header_layout():
    """dbfft_default_opts clears the whole C struct before filling it: the
    bytes it touches in a poisoned buffer give sizeof(dbfft_opts), which
    must equal the ctypes mirror's size (a shorter mirror would be
    overwritten past its end)."""
    from paper_1905_12725_amd import _native
    buf = (ctypes.c_ubyte * 512)(*([0xAB] * 512))
    _native.lib().dbfft_default_opts(ctypes.cast(buf, ctypes.POINTER(_native.Opts)))
    touched = max(i for i in range(512) if buf[i] != 0xAB) + 1
    size = ctypes.sizeof(_native.Opts)
    assert size - 8 < touched <= size
    assert bytes(buf[size:]) == bytes([0xAB] * (512 - size))


# -- argument validation: every case below is rejected before any HIP call,
#    so it runs without a GPU (the header's stated error behaviour)

def _setup(n, kin=0, prec=0, mat=0, field=1, params=(1.0, 0.3), out=True):
    from paper_1905_12725_amd import _native
    lib = _native.lib()
    h = ctypes.c_void_p()
    nn = (ctypes.c_int64 * 3)(*n)
    pp = (ctypes.c_double * max(len(params), 1))(*params)
    st = lib.dbfft_setup(ctypes.byref(h) if out else None, nn, kin, prec, mat,
                         ctypes.c_void_p(field) if field else None, pp if params else None, len(params), None)
    return st, lib.dbfft_last_error().decode()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
@pytest.mark.parametrize("kwargs,needle", [
    (dict(n=(11, 8, 8)), "2^a 3^b 5^c 7^d"),
    (dict(n=(8, 0, 8)), "2^a 3^b 5^c 7^d"),
    (dict(n=(8, 8, 8), kin=1, mat=0), "FINITE"),
    (dict(n=(8, 8, 8), kin=0, mat=5), "FINITE"),
    (dict(n=(8, 8, 8), kin=0, mat=4), "FINITE"),
    (dict(n=(8, 8, 8), mat=9), "unknown material"),
    (dict(n=(8, 8, 8), kin=2), "kinematics"),
    (dict(n=(8, 8, 8), prec=7), "precision"),
    (dict(n=(8, 8, 8), field=0), "null material field"),
    (dict(n=(8, 8, 8), params=()), "parameters"),
    (dict(n=(8, 8, 8), out=False), "null output"),
])
def test_setup_rejects_invalid_arguments(kwargs, needle):
    st, msg = _setup(**kwargs)
    assert st == 1, (st, msg)  # DBFFT_EINVAL
    assert needle in msg, msg


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
@pytest.mark.parametrize("kwargs,needle", [
    (dict(n=(1372, 4, 4)), "n1 and n2"),          # 2^2 7^3, one past the longest x line
    (dict(n=(4, 1372, 4)), "n1 and n2"),
    (dict(n=(4, 4, 750)), "n3 too large"),        # 2 3 5^3: M = 375 > 372
    (dict(n=(4, 4, 600), kin=1, mat=4, params=(1.0, 3.0)), "n3 too large"),  # finite: M = 300 > 292
])
def test_setup_rejects_lines_beyond_the_maximum(kwargs, needle):
    st, msg = _setup(**kwargs)
    assert st == 6, (st, msg)  # DBFFT_EUNSUPPORTED
    assert needle in msg, msg


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_null_handles_are_rejected():
    from paper_1905_12725_amd import _native
    lib = _native.lib()
    load = (ctypes.c_double * 9)()
    mask = (ctypes.c_uint8 * 9)()
    info = _native.Info()
    assert lib.dbfft_solve(None, load, mask, 1, 1.0, None, ctypes.byref(info)) == 1
    assert lib.dbfft_batch_create(None, None, 0, 1) == 1
    assert lib.dbfft_batch_solve(None, load, mask, 1, 1.0, None, ctypes.byref(info)) == 1
    assert lib.dbfft_set_lengths(None, (ctypes.c_double * 3)(1.0, 1.0, 1.0)) == 1
    assert lib.dbfft_solve_many(None, 1, load, mask, None, ctypes.byref(info), 2) == 1
    assert lib.dbfft_residuals(None, None, None, None, None, (ctypes.c_double * 4)()) == 1
    lib.dbfft_destroy(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_apply_noalloc_rejects_null_arguments_without_gpu():
    """The allocation-free apply checks its arguments before any GPU call."""
    from paper_1905_12725_amd import _native
    lib = _native.lib()
    n = (ctypes.c_int64 * 3)(8, 8, 8)
    params = (ctypes.c_double * 2)(1.0, 0.3)
    assert lib.dbfft_apply_noalloc(n, 0, None, params, 2, None, None, None) == 1
    assert lib.dbfft_apply_noalloc(None, 0, None, params, 2, None, None, None) == 1
    assert "null" in lib.dbfft_last_error().decode()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbfft.so not built")
def test_binding_maps_one_hip_runtime():
    """Loading the binding before torch must not bring a second HIP runtime
    into the process (torch and the library name it differently)."""
    import subprocess
    import sys
    code = ("from paper_1905_12725_amd import _native\n"
            "_native.lib()\n"
            "import torch\n"
            "paths = set()\n"
            "for line in open('/proc/self/maps'):\n"
            "    f = line.split()[-1]\n"
            "    if 'libamdhip64' in f:\n"
            "        paths.add(f)\n"
            "print(len(paths))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
