"""CPU-side checks of the C ABI: the library loads, exports every function
include/md.h declares, and its host-only entry points agree with the oracle's
constants.  No device work is launched here."""
import ctypes

import numpy as np
import pytest

import oracle as orc
from paper_2606_08039_amd import md


def test_library_exports_every_declared_symbol():
    L = md.lib()
    names = md.header_symbols()
    assert "md_step" in names and "md_create" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in md.md_version()


def test_default_params_match_oracle_constants():
    p = md.md_default_params_cf2x()
    P = orc.cf2x()
    for name, _ in md.md_params._fields_:
        a, b = getattr(p, name), getattr(P, name)
        if isinstance(a, float):
            assert a == b, name
        else:
            assert list(a) == list(b), name


def test_derived_constants_match_oracle():
    p = md.md_default_params_cf2x()
    d = md.md_derive(p)
    D = orc.derive(orc.cf2x())
    for k in ("hover_rpm", "max_rpm", "max_thrust", "h_clip"):
        assert getattr(d, k) == pytest.approx(getattr(D, k), rel=1e-15), k


def test_create_rejects_bad_arguments_before_touching_a_device():
    p = md.md_default_params_cf2x()
    L = md.lib()
    out = ctypes.c_void_p()
    assert L.md_create(None, 1 / 240, 0, 0, 1, ctypes.byref(out)) == md.MD_E_INVALID_ARG
    assert L.md_create(ctypes.byref(p), 0.0, 0, 0, 1, ctypes.byref(out)) == md.MD_E_INVALID_ARG
    assert L.md_create(ctypes.byref(p), 1 / 240, 0, 7, 1, ctypes.byref(out)) == md.MD_E_INVALID_ARG
    assert L.md_create(ctypes.byref(p), 1 / 240, 0, 0, 0, ctypes.byref(out)) == md.MD_E_INVALID_ARG
    assert L.md_create(ctypes.byref(p), 1 / 240, 8 | 4, 0, 1, ctypes.byref(out)) == md.MD_E_INVALID_ARG
    assert out.value is None
    assert "SURROGATE" in md.md_last_error(None)
    assert L.md_step(None, None, None, 0, None, 0, 1, 0, None) == md.MD_E_INVALID_ARG


STRUCTS = ("md_params", "md_derived", "md_state", "md_dr", "md_wind", "md_launch_config", "md_judge")


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every public struct of include/md.h has the size and field offsets the
    Python binding declares (a C program built with gcc against the header
    prints them)."""
    import os
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include <stdio.h>', '#include "md.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (s, s))
        for f, _ in getattr(md, s)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (s, f, s, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-std=c11", "-I", inc, str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for s in STRUCTS:
        cls = getattr(md, s)
        assert got[(s, "size")] == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)
