"""Host-side argument checks of the Python binding: every array handed to the C ABI is
checked against the mesh, the batch and the basis size before any library call, so a
mis-shaped tensor raises ValueError instead of letting a kernel read or write outside
it.  Runs without a GPU: a correctly shaped CPU tensor gets past the size checks and is
refused by the device-pointer check (TypeError) instead."""
import pytest
import torch

import workloads as W
from paper_2004_05756_amd import binding


@pytest.fixture(scope="module")
def ctx():
    c = object.__new__(binding.Context)  # no device: only the checks run
    c.lib = binding.load()
    c.h = None
    return c


def _mesh2():
    return W.Mesh((6, 4))  # 24 elements, 35 nodes, 70 DOFs


def _mesh3():
    return W.Mesh((3, 2, 2))  # 12 elements, 36 nodes, 108 DOFs


def f64(*shape):
    return torch.zeros(shape, dtype=torch.float64)


def u8(n):
    return torch.zeros(n, dtype=torch.uint8)


def test_mesh_sizes():
    assert binding.mesh_sizes(binding.make_mesh(_mesh2())) == (24, 35, 70)
    assert binding.mesh_sizes(binding.make_mesh(_mesh3())) == (12, 36, 108)


def test_apply_shapes(ctx):
    m = _mesh2()
    with pytest.raises(ValueError, match="rho"):
        ctx.apply(m, f64(2, 23), u8(70), f64(2, 70), f64(2, 70))
    with pytest.raises(ValueError, match="x"):
        ctx.apply(m, f64(2, 24), u8(70), f64(1, 70), f64(1, 70))
    with pytest.raises(ValueError, match="mask"):
        ctx.apply(m, f64(2, 24), u8(69), f64(2, 70), f64(2, 70))
    with pytest.raises(TypeError):
        ctx.apply(m, f64(2, 24), u8(70), f64(2, 70), f64(2, 70))


def test_hdm_shapes(ctx):
    m = _mesh3()
    with pytest.raises(ValueError, match="f"):
        ctx.hdm_solve(m, f64(12), u8(108), f64(107))
    with pytest.raises(ValueError, match="u"):
        ctx.hdm_solve(m, f64(12), u8(108), f64(108), u=f64(100))
    with pytest.raises(TypeError):
        ctx.hdm_solve(m, f64(12), u8(108), f64(108))
    with pytest.raises(ValueError, match="dc"):
        ctx.hdm_gradient(m, f64(12), f64(108), dc=f64(11))
    with pytest.raises(ValueError, match="u"):
        ctx.hdm_gradient(m, f64(12), f64(36))


def test_rom_shapes(ctx):
    m = _mesh2()
    phi = torch.zeros((70, 8), dtype=torch.float32)
    with pytest.raises(ValueError, match="phi"):
        ctx.rom_build(m, torch.zeros((69, 8)), 4, u8(70), f64(70), f64(3, 24))
    with pytest.raises(ValueError, match="k="):
        ctx.rom_build(m, phi, 9, u8(70), f64(70), f64(3, 24))
    with pytest.raises(ValueError, match="Khat"):
        ctx.rom_build(m, phi, 4, u8(70), f64(70), f64(3, 24), Khat=f64(2, 4, 4))
    with pytest.raises(TypeError):
        ctx.rom_build(m, phi, 4, u8(70), f64(70), f64(3, 24))
    with pytest.raises(ValueError, match="fhat"):
        ctx.rom_solve(f64(3, 4, 4), f64(5))
    with pytest.raises(ValueError, match="Khat"):
        ctx.rom_solve(f64(3, 4, 5), f64(4))
    with pytest.raises(ValueError, match="status"):
        ctx.rom_solve(f64(3, 4, 4), f64(4), status=torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError, match="yhat"):
        ctx.rom_solve_noalloc(f64(3, 4, 4), f64(4), torch.zeros(3, dtype=torch.int32), f64(3, 3), f64(3))
    with pytest.raises(ValueError, match="yhat"):
        ctx.rom_estimate(m, phi, 4, u8(70), f64(70), f64(3, 24), f64(3, 4, 4), f64(2, 4))
    with pytest.raises(ValueError, match="dJ"):
        ctx.rom_estimate(m, phi, 4, u8(70), f64(70), f64(3, 24), f64(3, 4, 4), f64(3, 4), dJ=f64(3, 23))
    with pytest.raises(TypeError):
        ctx.rom_estimate(m, phi, 4, u8(70), f64(70), f64(3, 24), f64(3, 4, 4), f64(3, 4))
    with pytest.raises(ValueError, match="yhat"):
        ctx.rom_gradient(m, phi, 4, u8(70), f64(3, 24), f64(3, 5))


def test_filter_and_basis_shapes(ctx):
    m = _mesh3()
    with pytest.raises(ValueError, match="nodal"):
        ctx.filter_forward(m, 1.0, f64(2, 12), phi=f64(2, 35))
    with pytest.raises(ValueError, match="output"):
        ctx.filter_adjoint(m, 1.0, f64(2, 12), g=f64(1, 12))
    with pytest.raises(TypeError):
        ctx.filter_forward(m, 1.0, f64(2, 12), phi=f64(2, 36))
    with pytest.raises(ValueError, match="G"):
        ctx.pod_push(f64(4, 50), f64(4, 3), [0, 0], f64(50))
    with pytest.raises(ValueError, match="u"):
        ctx.pod_push(f64(4, 50), f64(4, 4), [0, 0], f64(49))
    with pytest.raises(ValueError, match="phi"):
        ctx.pod_basis(f64(4, 50), f64(4, 4), 2, f64(50), 2, f64(49, 3))
