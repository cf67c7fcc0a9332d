"""CPU-only checks of the C ABI: the built library loads, exports every
entry point declared in include/bsm.h, and the binding's struct layouts
match the header (sizes and offsets printed by a gcc-compiled probe)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bsm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2003_03868_amd import bsm
    lib = bsm.load()
    declared = _declared()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(bsm.EXPORTED) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", bsm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted(set(re.findall(r" T (bsm_[a-z0-9_]+)$", out, flags=re.M)))
    assert exported == declared


def test_host_only_calls():
    from paper_2003_03868_amd import bsm
    assert "gfx950" in bsm.bsm_version()
    o = bsm.bsm_sign_opts_default()
    assert o.tol == 1e-6 and o.max_iter == 100 and o.prec == bsm.FP64
    assert isinstance(bsm.bsm_last_error(), str)


def test_struct_layouts_match_header(tmp_path):
    import ctypes as C
    from paper_2003_03868_amd import bsm
    structs = {
        "bsm_info": bsm.bsm_info, "bsm_mult_stats": bsm.bsm_mult_stats,
        "bsm_sign_opts": bsm.bsm_sign_opts, "bsm_sign_stats": bsm.bsm_sign_stats,
        "bsm_mu_stats": bsm.bsm_mu_stats, "bsm_tc2_stats": bsm.bsm_tc2_stats,
        "bsm_smm_params": bsm.bsm_smm_params, "bsm_sub_stats": bsm.bsm_sub_stats,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bsm.h"', 'int main(void){']
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for sname, cls in structs.items():
        assert got[(sname, "size")] == C.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert got[(sname, fname)] == getattr(cls, fname).offset, (sname, fname)
