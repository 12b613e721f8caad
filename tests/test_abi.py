"""The C ABI library loads without a GPU and exports every entry point declared in
include/*.h; argument validation that needs no device is checked here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(hipipm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("hipipm_create", "hipipm_solve", "hipipm_destroy", "hipipm_kkt_factor_solve",
                 "hipipm_state_import", "hipipm_state_export", "hipipm_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_26341_amd import hipipm
    L = hipipm.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    from paper_2606_26341_amd import mlp
    assert set(hipipm.EXPORTS) | set(mlp.EXPORTS) == set(declared_functions())


def test_struct_sizes_match_header_layout():
    from paper_2606_26341_amd import hipipm
    # the ctypes mirrors follow the header's field order: doubles are 8-byte aligned
    assert C.sizeof(hipipm.ProblemDesc) == 4 * 4 + 11 * 8
    o = hipipm.default_options()
    assert o.tol == 1e-8 and o.max_iter == 1000 and o.warm_gate == 1 and o.poll_every >= 1


def test_create_rejects_bad_arguments_without_touching_the_device():
    from paper_2606_26341_amd import hipipm, workloads as W
    L = hipipm.load()
    d = hipipm.desc_from(W.get("C1"))
    o = hipipm.default_options()
    h = C.c_void_p()
    assert L.hipipm_create(C.byref(d), C.byref(o), 0, C.byref(h)) == -1          # no slots
    bad = hipipm.desc_from(W.get("C1"))
    bad.N = 0
    assert L.hipipm_create(C.byref(bad), C.byref(o), 4, C.byref(h)) == -1
    bad = hipipm.desc_from(W.get("C1"))
    bad.n_agents = 4
    assert L.hipipm_create(C.byref(bad), C.byref(o), 4, C.byref(h)) == -3        # unsupported family size
    o2 = hipipm.default_options(max_iter=-1)
    assert L.hipipm_create(C.byref(d), C.byref(o2), 4, C.byref(h)) == -1
    assert L.hipipm_create(None, C.byref(o), 4, C.byref(h)) == -1
