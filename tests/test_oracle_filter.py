"""Pins of the oracle's Helmholtz filter (Sec. 2.2) and of the gradient through it
(Sec. 2.4): closed-form element matrices, constants and volume preserved exactly, the
reduction of x-only data to the 1D problem, the adjoint against the forward map, and
finite differences of J(psi) = c(rho*(psi))."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle import filter as F
import workloads as W


def test_element_matrices_closed_form():
    """Bilinear square element: Laplacian (1/6)[4 -1 -1 -2 ...], mass (h^2/36)[4 2 2 1 ...]
    in local order (0,0),(1,0),(0,1),(1,1); load h^2/4 per node.  Trilinear cube: the
    tensor products of the 1D matrices K1 = [1 -1; -1 1]/h, M1 = h [2 1; 1 2]/6."""
    r, h = 1.7, 2.0
    H, b = F.helmholtz_element(2, (h, h), r)
    KL = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    M = h * h / 36.0 * np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]])
    assert np.allclose(H, r * r * KL + M, rtol=1e-14, atol=1e-14)
    assert np.allclose(b, h * h / 4.0)
    hx, hy, hz = 1.0, 2.0, 0.5
    K1 = lambda a: np.array([[1, -1], [-1, 1]]) / a
    M1 = lambda a: a * np.array([[2, 1], [1, 2]]) / 6.0
    # local order x fastest: index = ix + 2 iy + 4 iz  ->  kron(z, y, x)
    KL3 = (np.kron(M1(hz), np.kron(M1(hy), K1(hx))) + np.kron(M1(hz), np.kron(K1(hy), M1(hx)))
           + np.kron(K1(hz), np.kron(M1(hy), M1(hx))))
    M3 = np.kron(M1(hz), np.kron(M1(hy), M1(hx)))
    H3, b3 = F.helmholtz_element(3, (hx, hy, hz), r)
    assert np.allclose(H3, r * r * KL3 + M3, rtol=1e-14, atol=1e-14)
    assert np.allclose(b3, hx * hy * hz / 8.0)


@pytest.mark.parametrize("mk", [lambda: W.mbb2d(14, 6).mesh, lambda: W.cantilever3d(5, 4, 3).mesh])
def test_constants_and_volume_are_preserved(mk):
    m = mk()
    r = F.filter_radius(1.3)
    rho, phi = F.filter_forward(m, r, np.full(m.n_elems, 0.37))
    assert np.abs(rho - 0.37).max() < 1e-13 and np.abs(phi - 0.37).max() < 1e-13
    psi = np.random.default_rng(4).uniform(0, 1, m.n_elems)
    rho, _ = F.filter_forward(m, r, psi)
    assert abs(rho.sum() - psi.sum()) < 1e-12 * psi.sum()  # equal element sizes


def test_x_only_data_reduces_to_the_1d_problem():
    """With psi depending on the column only, phi = phi_x (x) 1 where
    (r^2 K1 + M1) phi_x = b_x(psi) is the assembled 1D problem (tridiagonal)."""
    nx, ny, h = 16, 5, 1.0
    m = W.mbb2d(nx, ny).mesh
    r = 2.3
    col = np.random.default_rng(2).uniform(0, 1, nx)
    psi = np.tile(col, ny)
    _, phi = F.filter_forward(m, r, psi)
    A = np.zeros((nx + 1, nx + 1))
    bx = np.zeros(nx + 1)
    for e in range(nx):
        A[e:e + 2, e:e + 2] += r * r * np.array([[1, -1], [-1, 1]]) / h + h * np.array([[2, 1], [1, 2]]) / 6.0
        bx[e:e + 2] += col[e] * h / 2.0
    # banded solve of the tridiagonal system
    ab = np.zeros((3, nx + 1))
    ab[0, 1:] = np.diag(A, 1)
    ab[1] = np.diag(A)
    ab[2, :-1] = np.diag(A, -1)
    phix = sla.solve_banded((1, 1), ab, bx)
    assert np.abs(phi.reshape(ny + 1, nx + 1) - phix[None, :]).max() < 1e-13


@pytest.mark.parametrize("mk", [lambda: W.mbb2d(9, 4).mesh, lambda: W.cantilever3d(4, 3, 3).mesh])
def test_adjoint_is_the_transpose_of_the_forward_map(mk):
    m = mk()
    r = F.filter_radius(0.9)
    rng = np.random.default_rng(8)
    for _ in range(3):
        w = rng.standard_normal(m.n_elems)
        v = rng.standard_normal(m.n_elems)
        Aw, _ = F.filter_forward(m, r, w)
        ATv, _ = F.filter_adjoint(m, r, v)
        assert abs(v @ Aw - ATv @ w) < 1e-13 * np.abs(v).sum() * np.abs(Aw).max() * 10


@pytest.mark.parametrize("mk", [lambda: W.mbb2d(10, 4), lambda: W.cantilever3d(4, 3, 2)])
def test_gradient_through_the_filter_matches_finite_differences(mk):
    """dJ/dpsi = (d rho*/d psi)^T dc/drho (Sec. 2.4), J(psi) = f^T u(rho*(psi))."""
    p = mk()
    m = p.mesh
    r = F.filter_radius(1.1)
    psi = np.random.default_rng(5).uniform(0.3, 0.8, m.n_elems)

    def J(ps):
        rho, _ = F.filter_forward(m, r, ps)
        return O.compliance(p.f, O.solve_direct(m, rho, p.f, p.mask))

    rho, _ = F.filter_forward(m, r, psi)
    u = O.solve_direct(m, rho, p.f, p.mask)
    g, _ = F.filter_adjoint(m, r, O.sensitivity(m, rho, u))
    for e in (0, m.n_elems // 3, m.n_elems - 1):
        d = 1e-5
        pp, pm = psi.copy(), psi.copy()
        pp[e] += d
        pm[e] -= d
        fd = (J(pp) - J(pm)) / (2 * d)
        assert abs(fd - g[e]) <= 1e-6 * abs(g).max(), (e, fd, g[e])


def test_large_radius_gives_the_volume_mean():
    m = W.mbb2d(8, 4).mesh
    psi = np.random.default_rng(1).uniform(0, 1, m.n_elems)
    rho, _ = F.filter_forward(m, 1e4, psi)
    assert np.abs(rho - psi.mean()).max() < 1e-6


def test_cited_length_matches_the_conic_filter_second_moment():
    """Which relation between r and R the two readings give, pinned on the oracle's own
    filter: in 1D the Helmholtz kernel exp(-|x|/r)/(2r) has second moment 2 r^2 and the
    conic filter of radius R (weights R - |x|) has R^2 / 6, so r = R / (2 sqrt(3))
    gives a filter as wide as the conic one of radius R.  On a strip of unit elements,
    a one-element impulse filtered with r = filter_radius_cited(R) spreads with that
    variance (up to the O(h^2) of the element averages); with the printed r = 2 sqrt(3) R
    it spreads 144 times wider."""
    R = 24.0
    m = W.Mesh((401, 1))
    psi = np.zeros(m.n_elems)
    psi[200] = 1.0
    x = np.arange(m.n_elems) - 200.0
    var = {}
    for name, r in (("cited", F.filter_radius_cited(R)), ("printed", F.filter_radius(R))):
        rho, _ = F.filter_forward(m, r, psi)
        rho = rho[0] if rho.ndim == 2 else rho
        var[name] = float(np.sum(x * x * rho) / np.sum(rho))
    assert abs(var["cited"] / (R * R / 6.0) - 1.0) < 0.02, var
    assert var["printed"] > 50 * R * R / 6.0 or var["printed"] > 0.5 * (400 ** 2 / 12), var
