"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no compute call is made)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\w[\w \*]*?\b(sde_\w+)\s*\(", txt, re.M)
    return names


def test_header_declares_entry_points():
    names = _declared()
    for n in ("sde_jj_integrate", "sde_kuramoto_integrate", "sde_observables", "sde_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_0903_3852_amd as sde
    L = sde.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(sde.EXPORTS) <= set(_declared())


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the binding's ctypes mirrors
    equals what a C compiler makes of include/sde.h."""
    import ctypes
    import shutil
    import subprocess
    import paper_0903_3852_amd as sde
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [sde.sde_jj_point, sde.sde_run, sde.sde_kuramoto_desc, sde.sde_stats,
               sde.sde_surrogate_scaling, sde.sde_train_opts, sde.sde_scan_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sde.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append(f'printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for st in structs:
        n = st.__name__
        assert int(got[n]) == ctypes.sizeof(st), n
        for f, _ in st._fields_:
            assert int(got[f"{n}.{f}"]) == getattr(st, f).offset, (n, f)
    assert sde.JJ_POINT_DTYPE.itemsize == ctypes.sizeof(sde.sde_jj_point)
    for f, _ in sde.sde_jj_point._fields_:
        assert sde.JJ_POINT_DTYPE.fields[f][1] == getattr(sde.sde_jj_point, f).offset, f


def test_status_strings():
    import paper_0903_3852_amd as sde
    assert sde.sde_strerror(sde.SDE_ERR_INVALID) == "invalid argument"
    assert sde.sde_strerror(sde.SDE_ERR_NUMERIC).startswith("state became")


def test_create_without_gpu_fails_cleanly():
    import torch
    import paper_0903_3852_amd as sde
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sde.SDEError):
        sde.sde_create(0)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_0903_3852_amd as sde
    monkeypatch.setattr(sde, "_lib", None)
    monkeypatch.setattr(sde, "LIBPATH", str(tmp_path / "libsde.so"))
    with pytest.raises(ImportError):
        sde.lib()
