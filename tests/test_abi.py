"""The C-ABI library loads and exports every function include/dgmi.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1609_00098_amd", "libdgmi.so")


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s\*]+([A-Za-z_][A-Za-z0-9_]*)\s*\(", txt,
                             flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.append(name)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("dg_rhs", "dg_step", "con2prim", "dgmi_create", "dgmi_destroy", "dgmi_prim2cons",
                     "mlp_train_step", "mlp_forward", "mlp_grad"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libdgmi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_1609_00098_amd import dgmi
    x = torch.zeros((5, 4), dtype=torch.float64)
    with pytest.raises(TypeError):
        dgmi._ptr(x)
