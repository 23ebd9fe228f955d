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


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the C compiler's sizes and offsets for every struct the
    header declares (compiled here with gcc against include/conv.h)."""
    import shutil
    import subprocess

    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    checks = [("conv_params_t", binding.Params, [f for f, _ in binding.Params._fields_]),
              ("conv_state_t", binding.State, [f for f, _ in binding.State._fields_]),
              ("conv_deep_out_t", binding.DeepOut, [f for f, _ in binding.DeepOut._fields_]),
              ("conv_shallow_out_t", binding.ShallowOut, [f for f, _ in binding.ShallowOut._fields_]),
              ("conv_deep_cot_t", binding.DeepCot, [f for f, _ in binding.DeepCot._fields_]),
              ("conv_deep_grad_t", binding.DeepGrad, [f for f, _ in binding.DeepGrad._fields_]),
              ("conv_member_t", binding.Member, [f for f, _ in binding.Member._fields_])]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "conv.h"', "int main(void) {"]
    for cname, _, fields in checks:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = iter(int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                              text=True).stdout.split())
    for cname, cls, fields in checks:
        assert next(got) == C.sizeof(cls), cname
        for f in fields:
            assert next(got) == getattr(cls, f).offset, (cname, f)


def test_ensemble_argument_checks_without_gpu():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libconv.so not built")
    L = binding.lib()
    h = C.c_void_p()
    m = (binding.Member * 2)()
    m[0].ncol, m[0].nlev = 10, 30  # null arrays
    m[1].ncol, m[1].nlev = 0, 30
    assert L.conv_ensemble_workspace_bytes(2, m) == 0
    assert L.conv_ensemble_create(2, m, C.c_void_p(256), 1 << 30, C.byref(h)) == binding.CONV_EINVAL
    assert L.conv_ensemble_create(0, m, C.c_void_p(256), 1 << 30, C.byref(h)) == binding.CONV_EINVAL
    m[0].ncol = 0
    m[0].nlev = 1
    assert L.conv_ensemble_workspace_bytes(2, m) == 0
    assert L.conv_ensemble_step(None, None) == binding.CONV_EINVAL
    assert L.conv_ensemble_replay(None, None) == binding.CONV_EINVAL
    assert L.conv_ensemble_capture(None, None) == binding.CONV_EINVAL
    assert L.conv_ensemble_set_launch(None, 1, 1) == binding.CONV_EINVAL
    assert L.conv_autotune(None, None, None, None, None, 1, 0, None, None, None) == binding.CONV_EINVAL


def test_mlp_training_batch_limit_sizes():
    """A smaller training limit shrinks the MLP workspace; the plain call is the limit = max_batch
    case; a limit above max_batch or below 1 is rejected."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libconv.so not built")
    L = binding.lib()
    w = [96, 512, 512, 512, 512, 64]
    wa = (C.c_int32 * len(w))(*w)
    n = len(w) - 1
    full = L.mlp_workspace_bytes(wa, n, 884736)
    assert full > 0 and L.mlp_workspace_bytes_ex(wa, n, 884736, 884736) == full
    small = L.mlp_workspace_bytes_ex(wa, n, 884736, 16384)
    assert 0 < small < full / 3
    assert L.mlp_workspace_bytes_ex(wa, n, 1000, 1001) == 0
    assert L.mlp_workspace_bytes_ex(wa, n, 1000, 0) == 0
    h = C.c_void_p()
    assert L.mlp_create_ex(wa, n, 1000, 1001, C.c_void_p(256), 1 << 30, C.byref(h)) == -1


def test_static_step_rejects_sizes_beyond_its_scratch_without_gpu():
    """conv_step_static checks its arguments and the size of the workspace its static device array
    must hold before any HIP call that launches or allocates: bad arguments give CONV_EINVAL,
    sizes beyond the array CONV_ERANGE (on 256 compute units the bound for 72 levels is 385,344
    columns), nothing is enqueued."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libconv.so not built")
    L = binding.lib()
    p = binding.make_params()
    d = binding.DeepOut(*([256] * 10))
    s = binding.ShallowOut(*([256] * 8))
    st = binding.State(*([256] * 8), 3_000_000, 1800.0)  # never dereferenced
    assert L.conv_step_static(2_000_000, 30, C.byref(p), C.byref(st), C.byref(d), C.byref(s),
                              None) == binding.CONV_ERANGE
    assert L.conv_step_static(2_000_000, 30, None, C.byref(st), C.byref(d), C.byref(s),
                              None) == binding.CONV_EINVAL
    assert L.conv_step_static(10, 1, C.byref(p), C.byref(st), C.byref(d), C.byref(s),
                              None) == binding.CONV_EINVAL
    assert L.conv_step_static(0, 30, C.byref(p), C.byref(st), C.byref(d), C.byref(s),
                              None) == binding.CONV_OK
    st.ld = 10  # ld < ncol
    assert L.conv_step_static(200, 30, C.byref(p), C.byref(st), C.byref(d), C.byref(s),
                              None) == binding.CONV_EINVAL
    assert L.conv_strerror(binding.CONV_ERANGE).startswith(b"size beyond")
