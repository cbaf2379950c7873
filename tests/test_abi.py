"""The C-ABI library loads and exports every symbol include/stdecomp.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stdecomp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stdecomp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("stdecomp_init", "stdecomp_epoch", "stdecomp_predict", "stdecomp_loss", "stdecomp_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2012_03550_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2012_03550_amd import binding
    assert sorted(binding.SIGNATURES) == declared_functions()


def test_strerror_without_gpu():
    from paper_2012_03550_amd import binding
    L = binding.load()
    assert L.stdecomp_strerror(0) == b"ok"
    assert L.stdecomp_strerror(-1) == b"invalid argument"
    assert L.stdecomp_strerror(-5).startswith(b"diverged")


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the sizes and field offsets the
    C compiler gives the header's structs."""
    import subprocess
    from paper_2012_03550_amd import binding
    structs = {"stdecomp_problem": binding.Problem, "stdecomp_options": binding.Options,
               "stdecomp_epoch_stats": binding.EpochStats, "stdecomp_loss_out": binding.LossOut,
               "stdecomp_info_out": binding.InfoOut}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "stdecomp.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_null_arguments_are_rejected_without_gpu():
    from paper_2012_03550_amd import binding
    L = binding.load()
    assert L.stdecomp_init(None, None, None) == binding.STD_E_INVAL
    assert L.stdecomp_free(None) == binding.STD_OK
    assert L.stdecomp_epoch(None, 1, None) == binding.STD_E_STATE


def test_bad_placement_is_rejected_without_gpu():
    """options.placement outside STD_PLACE_AUTO..STD_PLACE_ONE_XCC is refused
    before any device call."""
    import numpy as np
    from paper_2012_03550_amd import binding
    L = binding.load()
    dims = np.array([4, 5, 6], np.int64)
    ranks = np.array([2, 2, 2], np.int32)
    idx = np.zeros((3, 8), np.int32)
    vals = np.ones(8, np.float32)
    p = binding.Problem(3, dims.ctypes.data_as(binding._i64p), ranks.ctypes.data_as(binding._i32p), 8,
                        ctypes.c_void_p(idx.ctypes.data), ctypes.c_void_p(vals.ctypes.data))
    for bad in (-1, 3):
        o = binding.Options()
        assert L.stdecomp_default_options(ctypes.byref(o)) == binding.STD_OK
        assert o.placement == 0  # STD_PLACE_AUTO by default
        o.placement = bad
        h = ctypes.c_void_p()
        assert L.stdecomp_init(ctypes.byref(p), ctypes.byref(o), ctypes.byref(h)) == binding.STD_E_INVAL
        assert not h.value
