"""The C-ABI library loads and exports every entry point include/rkhsba.h
declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from helpers import ROOT

HEADER = os.path.join(ROOT, "include", "rkhsba.h")
LIB = os.path.join(ROOT, "paper_2403_01254_amd", "_lib", "librkhsba.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(rkhsba_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2403_01254_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_abi():
    names = declared_functions()
    for required in ("rkhsba_build_neighbors", "rkhsba_eval_loss", "rkhsba_accumulate_normal_eqs", "rkhsba_gn_step"):
        assert required in names
    assert len(names) >= 10


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} missing from {LIB}"


def test_default_options_and_create_without_device(lib):
    from paper_2403_01254_amd import rkhsba
    o = rkhsba.default_options()
    assert o.ell == 0.1 and o.cutoff_factor == 3.0 and o.sigma == 1.0 and o.cell_subdiv == 0 and o.pass_points == 0
    h = ctypes.c_void_p()
    bad = rkhsba.default_options()
    bad.ell = -1.0
    assert rkhsba.lib().rkhsba_create(ctypes.byref(h), ctypes.byref(bad)) == rkhsba.EINVAL
    bad = rkhsba.default_options()
    bad.pass_points = 48
    assert rkhsba.lib().rkhsba_create(ctypes.byref(h), ctypes.byref(bad)) == rkhsba.EINVAL
    rc = rkhsba.lib().rkhsba_create(ctypes.byref(h), ctypes.byref(o))
    if rc == rkhsba.OK:  # a machine with a GPU
        rkhsba.lib().rkhsba_destroy(h)
    else:
        assert rc == rkhsba.EDEVICE and not h.value


def test_server_default_options_and_validation_without_device(lib):
    """The server's defaults as documented in the header, and argument checks that come before any device
    call (lane count, work limit, split threshold, lane weight, lane-1 order)."""
    from paper_2403_01254_amd import rkhsba
    o = rkhsba.ServerOptions()
    rkhsba.lib().rkhsba_server_default_options(ctypes.byref(o))
    assert (o.max_active, o.hbm_budget_bytes, o.pass_points, o.use_graphs, o.lanes) == (64, 0, 0, 1, 1)
    assert o.lane_split_entries == 2_000_000 and o.lane_work_entries == 0
    assert o.lane1_max_active == 1 and o.lane_split_work == 5e8 and o.lane0_weight == 0.25
    assert o.lane1_order == 1
    h = ctypes.c_void_p()
    for field, value in (("lanes", 0), ("lanes", 3), ("lane_work_entries", -1), ("lane_split_entries", -1),
                         ("max_active", 0), ("lane0_weight", 0.0), ("lane0_weight", -1.0),
                         ("lane0_weight", float("nan")), ("lane1_order", 2), ("lane1_order", -1)):
        bad = rkhsba.ServerOptions()
        rkhsba.lib().rkhsba_server_default_options(ctypes.byref(bad))
        setattr(bad, field, value)
        assert rkhsba.lib().rkhsba_server_create(ctypes.byref(h), ctypes.byref(bad)) == rkhsba.EINVAL, field
        assert not h.value


def test_product_code_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2403_01254_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f"{f} references the oracle"
