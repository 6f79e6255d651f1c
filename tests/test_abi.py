"""The C-ABI library loads and exports every function include/glecsim.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ge_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_are_exported():
    lib_path = os.path.join(ROOT, "paper_2506_11320_amd", "libglecsim.so")
    if not os.path.exists(lib_path):
        pytest.fail("libglecsim.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(lib_path)
    names = declared("glecsim.h")
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2506_11320_amd.glecsim import EXPORTS
    assert set(declared("glecsim.h")) <= set(EXPORTS) | {"ge_create"}


def test_binding_refuses_without_gpu(monkeypatch):
    import torch
    from paper_2506_11320_amd import Simulation
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        Simulation(1, (8, 1, 1), (0.5, 1, 1), theta=0.5, dt=0.5)
