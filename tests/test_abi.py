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


def test_struct_layouts_match_header():
    import ctypes
    import paper_0903_3852_amd as sde
    assert ctypes.sizeof(sde.sde_jj_point) == 6 * 8 + 2 * 4 + 2 * 8
    assert ctypes.sizeof(sde.sde_run) == 8 + 8 + 4 * 4
    assert ctypes.sizeof(sde.sde_kuramoto_desc) == 4 + 4 + 3 * 8 + 8 + 4 + 4


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
