"""CPU tests of the C-ABI boundary (include/sht.h, libsht.so): the library
loads, exports every declared symbol, and rejects bad arguments on the host
before any HIP call.  No transform is computed here."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from _util import ROOT, ensure_built

HEADER = os.path.join(ROOT, "include", "sht.h")


@pytest.fixture(scope="module")
def lib():
    return ensure_built()


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:sht_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_call_list():
    names = _declared_functions()
    for n in ("sht_plan", "sht_plan_destroy", "sht_forward", "isht_forward", "sht_backward", "isht_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2507_12144_amd", "libsht.so")],
                         capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for name in _declared_functions():
        assert name in exported, name


def test_binding_lists_every_symbol():
    from paper_2507_12144_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared_functions()


def _plan(lib, descs, prec=0):
    from paper_2507_12144_amd import _lib
    arr = (_lib.ShtDesc * max(len(descs), 1))(*[_lib.ShtDesc(*d) for d in descs])
    h = ctypes.c_void_p()
    rc = lib.sht_plan(ctypes.byref(h), arr if descs else None, len(descs), prec, None)
    return rc, h, lib.sht_last_error().decode()


GOOD = (33, 64, 17, 17, 0, 1, 2)


@pytest.mark.parametrize("desc,code", [
    ((1, 64, 17, 17, 0, 1, 2), 1),        # nlat < 2
    ((33, 1, 1, 1, 0, 1, 2), 1),          # nlon < 2
    ((33, 64, 0, 0, 0, 1, 2), 1),         # lmax < 1
    ((33, 64, 17, 0, 0, 1, 2), 1),        # mmax < 1
    ((33, 64, 17, 18, 0, 1, 2), 1),       # mmax > lmax
    ((33, 64, 40, 33, 0, 1, 2), 1),       # mmax > nlon/2
    ((33, 64, 17, 17, 0, 0, 2), 1),       # batch < 1
    ((33, 64, 17, 17, 0, 1, 0), 1),       # channels < 1
    ((33, 64, 17, 17, 3, 1, 2), 1),       # unknown grid
    ((33, 64, 17, 17, -1, 1, 2), 1),      # unknown grid
    ((33, 70, 17, 17, 0, 1, 2), 2),       # prime factor 7
    ((33, 1442, 17, 17, 0, 1, 2), 2),     # prime factor 7 and 103
    ((33, 8192, 17, 17, 0, 1, 2), 2),     # beyond the longest ring
])
def test_invalid_descs(lib, desc, code):
    rc, h, msg = _plan(lib, [desc])
    assert rc == code, msg
    assert h.value is None
    assert msg


def test_invalid_plan_arguments(lib):
    from paper_2507_12144_amd import _lib
    arr = (_lib.ShtDesc * 1)(_lib.ShtDesc(*GOOD))
    h = ctypes.c_void_p()
    assert lib.sht_plan(None, arr, 1, 0, None) == 1
    assert lib.sht_plan(ctypes.byref(h), None, 1, 0, None) == 1
    assert lib.sht_plan(ctypes.byref(h), arr, 0, 0, None) == 1
    assert lib.sht_plan(ctypes.byref(h), arr, 1, 7, None) == 1     # unknown precision
    # a bad second descriptor is reported with its index
    arr2 = (_lib.ShtDesc * 2)(_lib.ShtDesc(*GOOD), _lib.ShtDesc(33, 64, 17, 18, 0, 1, 2))
    assert lib.sht_plan(ctypes.byref(h), arr2, 2, 0, None) == 1
    assert "desc 1" in lib.sht_last_error().decode()


def test_null_plan_calls(lib):
    for fn in (lib.sht_forward, lib.isht_forward, lib.sht_backward, lib.isht_backward):
        assert fn(None, None, None, None) == 1
    assert lib.sht_plan_destroy(None) == 0
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sht_plan_segment(None, 0, ctypes.byref(a), ctypes.byref(b)) == 1
    assert lib.sht_plan_sizes(None, ctypes.byref(a), ctypes.byref(b)) == 1
    assert lib.sht_channel_mix(None, None, None, None, 0, None) == 1
    assert lib.sht_channel_mix_weight_grad(None, None, None, None, None) == 1
    g = ctypes.c_void_p(1)
    assert lib.sht_graph_create(None, 1, None, None, None, ctypes.byref(g)) == 1
    assert g.value is None  # cleared before the argument checks fail
    assert lib.sht_graph_create(None, 1, None, None, None, None) == 1
    assert lib.sht_graph_launch(None, None) == 1
    assert lib.sht_graph_destroy(None) == 0
    assert lib.sht_plan_tune(None, None, None, None) == 1


def test_status_strings(lib):
    names = {0: b"SHT_OK", 1: b"SHT_ERR_INVALID_ARG", 2: b"SHT_ERR_UNSUPPORTED", 3: b"SHT_ERR_OUT_OF_MEMORY",
             4: b"SHT_ERR_HIP", 5: b"SHT_ERR_INTERNAL"}
    for k, v in names.items():
        assert lib.sht_status_string(k) == v
    assert lib.sht_status_string(99) == b"unknown sht_status"


def test_valid_plan_without_gpu_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the GPU tests")
    rc, h, msg = _plan(lib, [GOOD])
    assert rc == 4 and h.value is None
    assert "hip" in msg.lower()


def test_binding_fails_loudly_without_library(tmp_path):
    code = ("import paper_2507_12144_amd._lib as L; L.LIB_PATH = '/nonexistent/libsht.so'; L._lib = None\n"
            "try:\n    L.load()\nexcept ImportError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "raised" in r.stdout, r.stderr


def test_product_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2507_12144_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
