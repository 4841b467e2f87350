"""CPU checks of the boundary: the C ABI library loads and exports every
function declared in include/mgar.h; the binding's struct layouts agree with
the header; no GPU is touched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgar.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s+\*?(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_parses():
    names = declared_functions()
    assert "mgar_setup" in names and "mgcg_solve" in names and "sens_filter" in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_2210_00947_amd import mgar as M
    L = M.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(M.EXPORTS) == declared_functions()


def test_struct_layout_matches_header(tmp_path):
    """Compile a probe against the header with the host C compiler and compare
    every field offset with the ctypes mirror used by the binding."""
    import subprocess
    from paper_2210_00947_amd import mgar as M
    fields = {"mgar_params": [f for f, _ in M.mgar_params._fields_],
              "mgar_stats": [f for f, _ in M.mgar_stats._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgar.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                    check=True).stdout.splitlines())
    for st, cls in (("mgar_params", M.mgar_params), ("mgar_stats", M.mgar_stats)):
        assert int(out[st]) == ctypes.sizeof(cls)
        for f, _ in cls._fields_:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_default_params_and_strerror():
    from paper_2210_00947_amd import mgar as M
    p = M.mgar_params()
    M.lib().mgar_default_params(ctypes.byref(p))
    assert p.k0 == 1.0 and p.kmin == 1e-3 and p.penal == 3.0 and p.omega == 0.8
    assert p.n_basis == 2 and p.cg_max == 200 and p.precision == 0
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert M.strerror(code) != "unknown error"


def test_params_for_config():
    import workloads as W
    from paper_2210_00947_amd import mgar as M
    p = M.params_for(W.C3)
    assert (p.dim, p.nelx, p.nely, p.nelz, p.levels) == (3, 128, 128, 128, 6)
    assert list(p.fix_lo) == [52, 52, 0] and list(p.fix_hi) == [76, 76, 0]
