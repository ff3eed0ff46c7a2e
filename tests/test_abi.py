"""Host-side checks of the C ABI: the library loads without a GPU, exports every
symbol the public headers declare, and its host-computed element stiffness agrees
with the oracle's quadrature."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(topo_\w+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2004_05756_amd import binding
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2004_05756_amd import binding
    declared = _declared_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared <= set(binding.EXPORTED) | set(getattr(binding, "SERVE_EXPORTED", ()))


@pytest.mark.parametrize("nel,h,nu,plane", [((4, 3), (1, 1), 0.3, 0), ((4, 3), (0.5, 2.0), 0.25, 0),
                                            ((4, 3), (1, 1), 0.3, 1), ((2, 2, 2), (1, 1, 1), 0.3, 0),
                                            ((2, 2, 2), (1.0, 0.5, 2.0), 0.2, 0)])
def test_library_element_stiffness_matches_oracle(nel, h, nu, plane):
    from paper_2004_05756_amd import binding
    m = W.Mesh(nel, h=h, nu=nu)
    mm = binding.make_mesh(m)
    mm.plane = plane
    ne = mm.dim * 2 ** mm.dim
    out = (C.c_double * (ne * ne))()
    assert binding.load().topo_element_stiffness(C.byref(mm), out) == 0
    K = np.frombuffer(out, dtype=np.float64).reshape(ne, ne)
    Ko = O.element_stiffness(len(nel), h, 1.0, nu, plane_stress=(plane == 0))
    assert np.abs(K - Ko).max() < 1e-14 * np.abs(Ko).max()


def test_invalid_mesh_rejected_on_host(lib):
    from paper_2004_05756_amd import binding
    out = (C.c_double * 64)()
    bad = binding.make_mesh(W.Mesh((4, 3)))
    bad.nu = 0.5
    assert lib.topo_element_stiffness(C.byref(bad), out) == binding.TOPO_EINVAL
    bad = binding.make_mesh(W.Mesh((4, 3)))
    bad.nel[0] = 0
    assert lib.topo_element_stiffness(C.byref(bad), out) == binding.TOPO_EINVAL
    bad = binding.make_mesh(W.Mesh((4, 3)))
    bad.dim = 4
    assert lib.topo_element_stiffness(C.byref(bad), out) == binding.TOPO_EINVAL
    assert lib.topo_strerror(-4) == b"TOPO_ENOTSPD"


def test_null_context_is_einval(lib):
    from paper_2004_05756_amd import binding
    m = binding.make_mesh(W.Mesh((4, 3)))
    assert lib.topo_hdm_gradient(None, C.byref(m), None, None, None, None) == binding.TOPO_EINVAL
    assert lib.topo_rom_solve(None, 4, 1, None, None, None, None, None, None) == binding.TOPO_EINVAL
