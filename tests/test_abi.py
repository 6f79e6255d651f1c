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


def test_binding_refuses_host_tensors():
    """Pointers handed to the library must be device tensors; the check is a
    ValueError (it stays under python -O)."""
    import torch
    from paper_2506_11320_amd.glecsim import _ptr
    with pytest.raises(ValueError):
        _ptr(torch.zeros(3, dtype=torch.float64))


def test_host_validation_refuses_before_any_device_call():
    """ge_create checks its arguments on the host first: refused grids never
    reach the device (so this runs without a GPU): a bad dimension, and a
    grid of 2^31 cells or more."""
    from paper_2506_11320_amd.glecsim import GEGrid, GEParams, load_library
    L = load_library()
    hdr = open(os.path.join(ROOT, "include", "glecsim.h")).read()
    err_arg = int(re.search(r"GE_ERR_ARG\s*=\s*(-?\d+)", hdr).group(1))
    fp64 = int(re.search(r"GE_FP64\s*=\s*(\d+)", hdr).group(1))

    def create(dim, n, precision):
        g = GEGrid()
        g.dim = dim
        for d in range(3):
            g.n[d] = n[d]
            g.dx[d] = 0.5
        p = GEParams(0.5, 1.0, 0.5, 1, 1, 1.0, 1, 1.0, 1, 5, 0.5, precision, 0, 0, 0.8, 0.1, 0)
        h = ctypes.c_void_p()
        rc = L.ge_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h))
        return rc, h.value

    assert create(4, (8, 8, 8), fp64) == (err_arg, None)
    assert L.ge_last_error(None).decode() == "ge_create: dim"
    assert create(3, (2048, 1024, 1024), fp64) == (err_arg, None)


@pytest.mark.parametrize("field,value", [("theta", 0.4), ("theta", 1.5), ("dt", 0.0), ("c", -1.0), ("precision", 7),
                                         ("n_smooth_u", -1), ("beta_lim", -0.5), ("ns_j", -1), ("ch_frac", -0.1),
                                         ("dedner_damp", -1.0), ("ns_e", -2)])
def test_host_validation_of_each_parameter(field, value):
    """Each out-of-range parameter is refused by ge_create before any device
    call (so this runs without a GPU)."""
    from paper_2506_11320_amd.glecsim import GEGrid, GEParams, load_library
    L = load_library()
    g = GEGrid()
    g.dim = 1
    g.n[0], g.n[1], g.n[2] = 8, 1, 1
    g.dx[0] = g.dx[1] = g.dx[2] = 0.5
    p = GEParams(0.5, 1.0, 0.5, 1, 1, 1.0, 1, 1.0, 1, 5, 0.5, 0, 0, 0, 0.8, 0.1, 0)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    assert L.ge_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1 and h.value is None


@pytest.mark.parametrize("dim,n", [(1, (2, 1, 1)), (2, (8, 1, 1)), (2, (8, 8, 2)), (3, (8, 8, 2))])
def test_host_validation_of_grid_shapes(dim, n):
    """Active axes need at least 3 cells, inactive ones exactly 1."""
    from paper_2506_11320_amd.glecsim import GEGrid, GEParams, load_library
    L = load_library()
    g = GEGrid()
    g.dim = dim
    for d in range(3):
        g.n[d] = n[d]
        g.dx[d] = 0.5
    p = GEParams(0.5, 1.0, 0.5, 1, 1, 1.0, 1, 1.0, 1, 5, 0.5, 1, 0, 0, 0.8, 0.1, 0)
    h = ctypes.c_void_p()
    assert L.ge_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1 and h.value is None
