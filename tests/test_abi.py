"""The C-ABI library loads and exports every entry point its header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibfsi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ib_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2103_06415_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2103_06415_amd import build
        build.build()
    return binding.load()


def test_header_declares_the_step_api():
    syms = declared_symbols()
    for name in ("ib_create", "ib_add_rigid", "ib_add_torsional", "ib_add_deformable",
                 "ib_set_subdomain", "ib_set_vorticity", "ib_prepare", "ib_step", "ib_sync",
                 "ib_read_stresses", "ib_read_deflection", "ib_read_vorticity", "ib_destroy",
                 "ib_status_str", "ib_op_solve"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2103_06415_amd", "lib", "libibfsi.so"))
    missing = [s for s in declared_symbols() if not hasattr(raw, s)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.ib_status_str(0) == b"ok"
    assert b"sub-domain" in lib.ib_status_str(-6)
    assert lib.ib_status_str(-100) == b"unknown status"


def test_create_rejects_bad_configs_without_a_gpu(lib):
    from paper_2103_06415_amd import binding
    out = ctypes.c_void_p()
    for n, levels, h in ((100, 1, 0.1), (32, 0, 0.1), (32, 1, -1.0), (30, 1, 0.1)):
        cfg = binding.IbConfig(n=n, levels=levels, h=h, re=100.0, dt=0.01)
        assert lib.ib_create(ctypes.byref(cfg), None, None, ctypes.byref(out)) == -1
    assert lib.ib_create(None, None, None, ctypes.byref(out)) == -1


def test_null_handles_are_rejected(lib):
    assert lib.ib_prepare(None) == -1
    assert lib.ib_step(None, 1) == -1
    assert lib.ib_destroy(None) == -1
