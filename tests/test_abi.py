"""The C-ABI library loads and exports every function include/dsbcg.h declares."""
import ctypes
import os
import subprocess

import pytest

from paper_1205_0359_amd import _lib


def test_header_declares_the_boundary():
    names = _lib.header_functions()
    for want in ("dsbcg_create", "dsbcg_destroy", "dsbcg_neighbors", "dsbcg_apply_A",
                 "dsbcg_apply_D", "dsbcg_solve", "dsbcg_link_grad", "dsbcg_last_error",
                 "dsbcg_default_opts"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _lib.header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _lib.header_functions():
        assert name in exported, name


def test_default_opts_and_argument_errors_without_a_device():
    o = _lib.default_opts()
    assert o.precision == 0 and o.max_iters == 10000 and o.ru_interval == 50
    assert o.refine == 1 and o.freeze == 1
    lib = _lib.load()
    h = ctypes.c_void_p()
    bad = (ctypes.c_int32 * 4)(4, 4, 1, 4)
    assert lib.dsbcg_create(bad, ctypes.byref(h)) == _lib.DSBCG_ERR_ARG
    assert b"extent" in lib.dsbcg_last_error()
    assert lib.dsbcg_create(None, ctypes.byref(h)) == _lib.DSBCG_ERR_ARG


def test_opts_struct_matches_header_layout(tmp_path):
    """The ctypes mirrors of dsbcg_opts and dsbcg_stats have the size and field
    offsets that a C compiler gives the header's structs."""
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dsbcg.h"', "int main(void) {"]
    for cls in (_lib.dsbcg_opts, _lib.dsbcg_stats):
        name = cls.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.dirname(_lib.HEADER_PATH)
    subprocess.run(["gcc", "-I", include, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cls in (_lib.dsbcg_opts, _lib.dsbcg_stats):
        name = cls.__name__
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_single_hip_runtime_in_process():
    # the library must bind to the HIP runtime PyTorch already loaded: two
    # runtimes in one process cannot both open the device
    _lib.load()
    maps = open("/proc/self/maps").read().splitlines()
    hip = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    hsa = {ln.split()[-1] for ln in maps if "libhsa-runtime64" in ln}
    assert len(hip) == 1 and len(hsa) <= 1, (hip, hsa)
