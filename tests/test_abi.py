"""The C-ABI library loads and exports every function include/fire2.h
declares; host-only helpers follow the paper's Table 1.  No GPU needed (no
compute call is made)."""
import ctypes
import json
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fire2.h")
LIB = os.path.join(ROOT, "paper_1908_02038_amd", "libfire2.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fire_\w+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("fire_init", "fire_minimize", "fire_energy_forces", "fire_hvp", "fire_minimize_batched",
              "fire_energy_forces_dev", "fire_hvp_dev", "fire_minimize_dev", "fire_lowest_curvature"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1908_02038_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in declared():
        getattr(lib, n)
    from paper_1908_02038_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


def test_params_default_is_table1():
    from paper_1908_02038_amd import api
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_defaults.json")))
    p = api.fire_params_default()
    assert p.integrator == 0 and p.halfstepback == ref["halfstepback"] and p.initialdelay == ref["initialdelay"]
    for k in ("tmax", "tmin", "dtgrow", "dtshrink", "alpha0", "alphashrink"):
        assert getattr(p, k) == ref[k], k
    assert p.delaystep == ref["delaystep"] and p.vdfmax == ref["vdfmax"]


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors must match the C layout (sizes and offsets from gcc)."""
    from paper_1908_02038_amd import _lib
    structs = {"fire_box": _lib.fire_box, "fire_potential": _lib.fire_potential,
               "fire_params": _lib.fire_params, "fire_result": _lib.fire_result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fire2.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_stop_names():
    from paper_1908_02038_amd import _lib
    lib = _lib.load()
    assert lib.fire_stop_name(3) == b"maxvdotf" and lib.fire_stop_name(1) == b"converged"
