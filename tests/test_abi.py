"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/helm.h declares, fills descriptor defaults, and rejects invalid
arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2404_02493_amd import lib

    return lib()


def test_header_symbols_are_exported():
    from paper_2404_02493_amd._abi import EXPORTS

    hdr = open(os.path.join(ROOT, "include", "helm.h")).read()
    declared = set(re.findall(r"\b(helm_[a-z_]+)\s*\(", hdr))
    assert declared == set(EXPORTS), declared ^ set(EXPORTS)
    L = _lib()
    for name in declared:
        assert hasattr(L, name), name


def test_desc_defaults():
    from paper_2404_02493_amd import default_desc

    d = default_desc(4096, 2100.0)
    assert (d.n, d.levels, d.damping_cells, d.sign, d.adr_steps) == (4096, 7, 16, 1, 8)
    assert (d.cheb_pre, d.cheb_post, d.cheb_coarse, d.gmres_m, d.gmres_coarse_m, d.restart) == (5, 5, 10, 3, 3, 20)
    assert (d.adr_levels, d.gmres_arnoldi, d.use_graphs, d.tail_n, d.wave_tail_n) == (3, 0, 1, 64, 32)
    assert d.damping_strength == 0.5 and d.k == 2100.0
    assert default_desc(128, 80.0).levels == 4


@pytest.mark.parametrize("field,value", [("n", 100), ("n", 8), ("levels", 1), ("levels", 7), ("k", -1.0),
                                         ("damping_cells", 0), ("sign", 0), ("cycle_prec", 5),
                                         ("gmres_m", 0), ("gmres_m", 25), ("restart", 30), ("cheb_pre", 0),
                                         ("adr_levels", -1), ("use_graphs", 2), ("gmres_arnoldi", 3),
                                         ("tail_n", -5), ("wave_tail_n", -1)])
def test_setup_rejects_invalid_descriptors(field, value):
    from paper_2404_02493_amd import default_desc

    L = _lib()
    d = default_desc(64, 30.0)
    setattr(d, field, value)
    ctx = ctypes.c_void_p()
    st = L.helm_setup(ctypes.byref(d), ctypes.c_void_p(1), ctypes.byref(ctx), None)
    assert st == 1, (field, value, st)
    assert ctx.value is None
    assert len(L.helm_last_error()) > 0


def test_null_arguments_are_rejected():
    from paper_2404_02493_amd import default_desc

    L = _lib()
    d = default_desc(64, 30.0)
    ctx = ctypes.c_void_p()
    assert L.helm_setup(ctypes.byref(d), None, ctypes.byref(ctx), None) == 1
    assert L.helm_setup(None, None, ctypes.byref(ctx), None) == 1
    assert L.helm_cycle(None, None, None, None) == 1
    assert L.helm_solve(None, None, None, 1e-6, 10, 0, None, None, None, None) == 1
    assert L.helm_cycle_backward(None, 1, None, None, None, None, None, None, None) == 1
    assert L.helm_loss(None, None, None, None, None, None) == 1
    assert L.helm_destroy(None) == 0


def test_status_strings():
    L = _lib()
    for s in range(7):
        assert L.helm_status_string(s).startswith(b"HELM_")
    assert L.helm_status_string(99) == b"unknown status"
    assert b"gfx950" in L.helm_version()
