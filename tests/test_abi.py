"""The C ABI library loads and exports every entry point include/conv.h declares; argument checks
that make no HIP call reject bad input (no compute calls here: this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_1711_00289_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if not n.isupper()))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libconv.so not built")
    lib = C.CDLL(binding.LIB_PATH)
    decl = declared_functions()
    assert len(decl) >= 9
    for name in decl:
        assert hasattr(lib, name), name
    assert set(binding.EXPORTS) <= set(decl)


def test_argument_checks_without_gpu():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libconv.so not built")
    L = binding.lib()
    h = C.c_void_p()
    p = binding.make_params()
    assert L.conv_create(10, 30, None, C.c_void_p(256), 1 << 20, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_create(-1, 30, C.byref(p), C.c_void_p(256), 1 << 20, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_create(10, 1, C.byref(p), C.c_void_p(256), 1 << 20, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_create(10, 30, C.byref(p), C.c_void_p(257), 1 << 20, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_create(10, 30, C.byref(p), None, 1 << 20, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_deep_forward(None, None, None, None) == binding.CONV_EINVAL
    assert L.conv_step(None, None, None, None, None) == binding.CONV_EINVAL
    assert L.conv_set_params(None, C.byref(p)) == binding.CONV_EINVAL
    assert L.conv_strerror(binding.CONV_EINVAL) == b"invalid argument"
