"""The C-ABI library loads on a machine without a GPU and exports every
function that include/pms.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1708_04710_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(pms_\w+)\s*\(", txt, flags=re.M))
    return names


def test_header_declares_entry_points():
    d = _declared()
    assert {"pms_create", "pms_destroy", "pms_reduce", "pms_last_error"} <= d
    assert d == set(_binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libpms.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_binding.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_layout_and_defaults():
    lib = _binding.load()
    o = lib.pms_default_options()
    assert (o.variant, o.compression, o.max_rounds, o.chain, o.validate, o.arena_entries) == (0, 1, 0, 1, 1, 0)
    assert ctypes.sizeof(_binding.PmsOptions) == 64
    assert (o.debug_invariants, o.c8, o.sweep, o.priority, o.round_budget, o.reserved) == (0, 0, 0, 0, 0, 0)
    assert ctypes.sizeof(_binding.PmsBoundary) == 48
    assert lib.pms_version().decode().startswith("pms-gfx950")
    # no context: the error text is static, and a null handle is rejected
    assert lib.pms_last_error(None) == b"no context"
    assert lib.pms_reduce(None, None, None, None) == _binding.PMS_ERR_INVALID_ARG
    assert o.diagnostics == 0 and ctypes.sizeof(_binding.PmsRoundStats) == 56
    assert lib.pms_round_stats_read(None, 0, None, None) == _binding.PMS_ERR_INVALID_ARG
    assert lib.pms_essential_estimate(None, 0, None) == _binding.PMS_ERR_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with status 2 and says
    so, before it touches torch or the device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout
