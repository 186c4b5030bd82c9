"""The C-ABI library on a host without a GPU: it loads, exports every call
include/vg.h declares, names every status code, and rejects bad arguments
before touching a device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vg_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def vgmod():
    import paper_1604_03155_amd as vg
    return vg


def test_library_exports_every_declared_call(vgmod):
    lib = ctypes.CDLL(vgmod.LIBRARY_PATH)
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(vgmod.EXPORTED)


def test_status_strings(vgmod):
    for code, name in enumerate(["VG_OK", "VG_ERR_INVALID_ARG", "VG_ERR_UNSUPPORTED_SIZE", "VG_ERR_OUT_OF_MEMORY",
                                 "VG_ERR_NO_DEVICE", "VG_ERR_DEVICE", "VG_ERR_NOT_CAPTURABLE", "VG_ERR_INTERNAL"]):
        assert vgmod.status_string(code) == name
    assert vgmod.status_string(99) == "VG_ERR_UNKNOWN"


BAD = [
    (dict(d=4, N=8), 1),                 # dimension
    (dict(d=3, N=7), 1),                 # odd N
    (dict(d=3, N=2), 1),                 # too small
    (dict(d=3, N=8, kernel=1, k=0.0), 1),     # Helmholtz needs k > 0
    (dict(d=3, N=8, kernel=1, k=float("nan")), 1),
    (dict(d=3, N=8, kernel=7), 1),       # unknown kernel
    (dict(d=3, N=8, kernel=5), 1),
    (dict(d=3, N=8, kernel=4), 1),       # convection needs h with |h| > 0
    (dict(d=2, N=8, kernel=4, h=(0.0, 0.0)), 1),
    (dict(d=3, N=8, kernel=4, h=(1.0, float("inf"), 0.0)), 1),
    (dict(d=3, N=8, kernel=4, h=(float("nan"), 1.0, 0.0)), 1),
    (dict(d=3, N=320, kernel=4, h=(1.0, 0.0, 0.0)), 2),   # 3D convection limited to N <= 256
    (dict(d=2, N=16384, kernel=4, h=(1.0, 0.0)), 2),      # (2N)^2 complex64 table above 4 GiB
    (dict(d=2, N=8, kernel=3, k=0.0), 1),     # Delta(Delta + k^2) needs k > 0
    (dict(d=2, N=8, kernel=3, k=-2.0), 1),
    (dict(d=3, N=8, L=1.5), 1),          # L below sqrt(3)
    (dict(d=2, N=8, L=1.2), 1),          # L below sqrt(2)
    (dict(d=3, N=8, P=2), 1),            # P not above 1 + L
    (dict(d=3, N=8, precision=5), 1),
    (dict(d=3, N=22), 2),                # 2N = 44 has the factor 11
    (dict(d=3, N=26), 2),                # 2N = 52 has the factor 13
]


@pytest.mark.parametrize("args,code", BAD)
def test_invalid_arguments_rejected_without_device(vgmod, args, code):
    lib = ctypes.CDLL(vgmod.LIBRARY_PATH)
    hv = list(args.get("h", ())) + [0.0] * (3 - len(args.get("h", ())))
    opts = vgmod._Opts(args.get("precision", 0), args.get("L", 0.0), args.get("P", 0), 0, 0, None,
                       (ctypes.c_double * 3)(*hv))
    h = ctypes.c_void_p(123)
    st = lib.vg_plan_create_ex(args["d"], args["N"], args.get("kernel", 0), ctypes.c_double(args.get("k", 0.0)),
                               ctypes.byref(opts), ctypes.byref(h))
    assert st == code
    assert h.value is None  # *out cleared on error
    assert lib.vg_last_error()  # a message is set


def test_null_arguments(vgmod):
    lib = vgmod._lib
    assert lib.vg_plan_create(3, 8, 0, 0.0, None) == 1
    assert lib.vg_apply(None, None, None, None, None) == 1
    assert lib.vg_gradient(None, None, None, None, None, None) == 1
    assert lib.vg_workspace_size(None) == 0
    assert lib.vg_plan_get_info(None, None) == 1
    arr = (ctypes.c_void_p * 1)()
    assert lib.vg_apply_batched(0, arr, arr, arr, None, None) == 1
    lib.vg_plan_destroy(None)  # no-op
    assert lib.vg_profiler_enable(3) == 1 and lib.vg_profiler_enable(-1) == 1
    assert lib.vg_profiler_enable(0) == 0


def test_no_device_reported_on_cpu_host(vgmod):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = vgmod._lib.vg_plan_create(3, 8, 0, 0.0, ctypes.byref(h))
    assert st == 4  # VG_ERR_NO_DEVICE


def test_header_is_plain_c_and_cpp():
    """include/vg.h is the boundary for C callers too: it must compile as C99
    and as C++17 on its own."""
    import shutil
    import subprocess
    for cc, args in (("gcc", ["-x", "c", "-std=c99"]), ("g++", ["-x", "c++", "-std=c++17"])):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not installed")
        r = subprocess.run([cc, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", *args, HEADER],
                           capture_output=True, text=True)
        assert r.returncode == 0, (cc, r.stderr)
