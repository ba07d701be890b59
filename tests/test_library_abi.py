"""The C-ABI library loads and exports every function include/ms.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_13386_amd", "libms.so")


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:ms_status|void|double|const char\s*\*)\s+(ms_\w+)\s*\(", txt, flags=re.M))
    return sorted(names)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_defaults_are_sane():
    from paper_2508_13386_amd import ms
    p = ms.solver_defaults()
    assert p.max_newton > 0 and 0 < p.newton_tol < 1e-6 and p.refine_iters in (0, 20, 40)
    assert p.subspace_rtol == 1e-4 and p.paper_eps == 1e-3
    b = ms.basis_defaults()
    assert b.prune_ratio == 1.75 and b.prune_every == 10 and b.prune_n == 5


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2508_13386_amd import ms
    monkeypatch.setattr(ms, "LIB_PATH", "/nonexistent/libms.so")
    monkeypatch.setattr(ms, "_lib", None)
    with pytest.raises(RuntimeError):
        ms.lib()


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the parameter and statistics structs have the
    C layout of include/ms.h (size and offset of every field)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2508_13386_amd import ms
    structs = [ms.ms_solver_params, ms.ms_step_stats, ms.ms_basis_params]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ms.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'  printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{st.__name__}.{f} %zu\\n", offsetof({st.__name__}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for st in structs:
        assert int(got[st.__name__]) == ctypes.sizeof(st), st.__name__
        for f, _ in st._fields_:
            assert int(got[f"{st.__name__}.{f}"]) == getattr(st, f).offset, (st.__name__, f)
