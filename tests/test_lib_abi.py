"""The C-ABI library loads and exports every symbol the public headers
declare (no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(pd_\w+)\s*\(", txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_headers_declare_the_boundary():
    names = _declared()
    for n in ["pd_plan_create", "pd_plan_destroy", "pd_force", "pd_force_adjoint", "pd_verlet_step",
              "pd_static_solve", "pd_damage_index", "pd_verlet_adjoint", "pd_status_str"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2105_06055_amd.build import LIB
    if not os.path.exists(LIB):
        pytest.skip("libpdfcbm.so not built")
    lib = ctypes.CDLL(LIB)
    for n in sorted(_declared()):
        assert hasattr(lib, n), n
    lib.pd_status_str.restype = ctypes.c_char_p
    assert lib.pd_status_str(1) == b"invalid argument"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2105_06055_amd import binding
    monkeypatch.setattr(binding, "LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.lib()
