"""The C-ABI library loads and exports every symbol include/qtp.h declares."""

import ctypes
import os
import re

from paper_1808_02558_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "qtp.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(qtp_[a-z0-9_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
        assert n in binding.SIGNATURES, n


def test_default_config():
    c = binding.default_config()
    assert c.precision == 0 and c.solve_tol == 1e-8 and c.fgmres_restart == 30
    c2 = binding.default_config(precision="bf16", qtt_rmax=64)
    assert c2.precision == 2 and c2.qtt_rmax == 64
    assert ctypes.sizeof(binding.Config) >= 80
