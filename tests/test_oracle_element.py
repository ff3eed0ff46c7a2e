"""Pins of the oracle's element stiffness (Sec. 2.1) against closed forms that do not
go through its quadrature code."""
import itertools

import numpy as np
import pytest

import oracle as O


def _1d(h):
    """Exact 1D integrals of linear shape functions f0 = 1 - x/h, f1 = x/h on [0, h]:
    mass M, stiffness S and the mixed form G[a][b] = int f_a' f_b."""
    M = np.array([[h / 3, h / 6], [h / 6, h / 3]])
    S = np.array([[1 / h, -1 / h], [-1 / h, 1 / h]])
    s = np.array([-1.0, 1.0])
    G = np.array([[s[a] / 2 for b in range(2)] for a in range(2)])
    return M, S, G


def _closed_form_q4(hx, hy, D):
    """Q4 stiffness as a sum of tensor products of 1D integrals (independent of any
    quadrature): K_ab^{mn} = sum_{ij} D-weighted int d_i N_a d_j N_b."""
    Mx, Sx, Gx = _1d(hx)
    My, Sy, Gy = _1d(hy)
    K = np.zeros((8, 8))
    for a, b in itertools.product(range(4), range(4)):
        ax, ay, bx, by = a & 1, a >> 1, b & 1, b >> 1
        dxdx = Sx[ax, bx] * My[ay, by]
        dydy = Mx[ax, bx] * Sy[ay, by]
        dxdy = Gx[ax, bx] * Gy[by, ay]   # int dNa/dx * dNb/dy
        dydx = Gx[bx, ax] * Gy[ay, by]   # int dNa/dy * dNb/dx
        K[2 * a, 2 * b] = D[0, 0] * dxdx + D[2, 2] * dydy
        K[2 * a + 1, 2 * b + 1] = D[1, 1] * dydy + D[2, 2] * dxdx
        K[2 * a, 2 * b + 1] = D[0, 1] * dxdy + D[2, 2] * dydx
        K[2 * a + 1, 2 * b] = D[1, 0] * dydx + D[2, 2] * dxdy
    return K


def _closed_form_h8(h, E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    one = [_1d(hh) for hh in h]

    def integral(a, b, da, db):
        """int (d_da N_a)(d_db N_b) over the box; da/db = axis index or -1 (no deriv)."""
        val = 1.0
        for ax in range(3):
            M, S, G = one[ax]
            ia, ib = (a >> ax) & 1, (b >> ax) & 1
            if da == ax and db == ax:
                val *= S[ia, ib]
            elif da == ax:
                val *= G[ia, ib]
            elif db == ax:
                val *= G[ib, ia]
            else:
                val *= M[ia, ib]
        return val

    K = np.zeros((24, 24))
    for a, b in itertools.product(range(8), range(8)):
        for m, n in itertools.product(range(3), range(3)):
            if m == n:
                v = (lam + 2 * mu) * integral(a, b, m, m)
                v += mu * sum(integral(a, b, k, k) for k in range(3) if k != m)
            else:
                v = lam * integral(a, b, m, n) + mu * integral(a, b, n, m)
            K[3 * a + m, 3 * b + n] = v
    return K


@pytest.mark.parametrize("h,nu,ps", [((1, 1), 0.3, True), ((0.5, 2.0), 0.25, True),
                                     ((1, 1), 0.3, False), ((3 / 180, 1 / 60), 0.3, True)])
def test_q4_matches_tensor_closed_form(h, nu, ps):
    K = O.element_stiffness(2, h, 1.0, nu, ps)
    D = O.constitutive(2, 1.0, nu, ps)
    assert np.allclose(K, _closed_form_q4(h[0], h[1], D), rtol=0, atol=1e-14)


@pytest.mark.parametrize("h,nu", [((1, 1, 1), 0.3), ((1.0, 0.5, 2.0), 0.2), ((2, 2, 2), 0.45)])
def test_h8_matches_tensor_closed_form(h, nu):
    K = O.element_stiffness(3, h, 1.0, nu)
    assert np.allclose(K, _closed_form_h8(h, 1.0, nu), rtol=0, atol=1e-14)


def test_q4_textbook_plane_stress_matrix():
    """The well-known closed form of the unit-square Q4 plane-stress element used by
    the compact SIMP codes the paper follows (nodes counter-clockwise from the lower
    left corner, DOFs interleaved)."""
    nu = 0.3
    k = np.array([1 / 2 - nu / 6, 1 / 8 + nu / 8, -1 / 4 - nu / 12, -1 / 8 + 3 * nu / 8,
                  -1 / 4 + nu / 12, -1 / 8 - nu / 8, nu / 6, 1 / 8 - 3 * nu / 8])
    pattern = [[1, 2, 3, 4, 5, 6, 7, 8], [2, 1, 8, 7, 6, 5, 4, 3], [3, 8, 1, 6, 7, 4, 5, 2],
               [4, 7, 6, 1, 8, 3, 2, 5], [5, 6, 7, 8, 1, 2, 3, 4], [6, 5, 4, 3, 2, 1, 8, 7],
               [7, 4, 5, 2, 3, 8, 1, 6], [8, 3, 2, 5, 4, 7, 6, 1]]
    KE = k[np.array(pattern) - 1] / (1 - nu ** 2)
    K = O.element_stiffness(2, (1, 1), 1.0, nu)
    ccw = [0, 1, 3, 2]  # tensor-order index of the counter-clockwise nodes
    dofs = [2 * a + c for a in ccw for c in range(2)]
    assert np.abs(K[np.ix_(dofs, dofs)] - KE).max() < 1e-15
    assert abs(K[0, 0] - (0.5 - nu / 6) / (1 - nu ** 2)) < 1e-15


def test_h8_diagonal_closed_form():
    nu = 0.3
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    K = O.element_stiffness(3, (1, 1, 1), 1.0, nu)
    assert np.allclose(np.diag(K), (lam + 4 * mu) / 9, atol=1e-15)
    assert abs(K[0, 0] - 0.2350427350427350) < 1e-15


def _rigid_modes(dim):
    nodes = [tuple((a >> d) & 1 for d in range(dim)) for a in range(2 ** dim)]
    X = np.array(nodes, float)
    modes = []
    for c in range(dim):
        v = np.zeros((2 ** dim, dim))
        v[:, c] = 1
        modes.append(v.ravel())
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in pairs:
        v = np.zeros((2 ** dim, dim))
        v[:, i] = -X[:, j]
        v[:, j] = X[:, i]
        modes.append(v.ravel())
    return np.array(modes)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_invariants(dim):
    K = O.element_stiffness(dim, (1.0,) * dim)
    assert np.abs(K - K.T).max() < 1e-15
    ev = np.linalg.eigvalsh(K)
    nrigid = 3 if dim == 2 else 6
    assert np.all(ev[:nrigid] > -1e-14) and np.all(np.abs(ev[:nrigid]) < 1e-14)
    assert ev[nrigid] > 1e-3
    for v in _rigid_modes(dim):
        assert np.abs(K @ v).max() < 1e-14
    # rows sum to zero (translations); all diagonal entries equal on square / cube
    assert np.abs(K.sum(axis=1)).max() < 1e-14
    assert np.ptp(np.diag(K)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_two_point_gauss_is_exact(dim):
    h = (1.0, 0.7, 1.3)[:dim]
    assert np.allclose(O.element_stiffness(dim, h, ngauss=2),
                       O.element_stiffness(dim, h, ngauss=4), atol=1e-14)


def test_h8_scales_linearly_with_h_and_q4_is_scale_free():
    assert np.allclose(O.element_stiffness(3, (2, 2, 2)), 2 * O.element_stiffness(3, (1, 1, 1)), atol=1e-14)
    assert np.allclose(O.element_stiffness(2, (0.1, 0.1)), O.element_stiffness(2, (1, 1)), atol=1e-14)


@pytest.mark.parametrize("nu", [0.0, 0.25, 0.3, 0.45])
def test_plane_strain_is_3d_law_with_zero_out_of_plane_strain(nu):
    """Plane strain pinned independently of its own branch: (a) it is the isotropic 3D
    law (pinned through the H8 closed forms above) restricted to exx, eyy, gxy with
    ezz = gyz = gxz = 0; (b) it equals plane stress with E' = E / (1 - nu^2) and
    nu' = nu / (1 - nu), the textbook correspondence between the two states."""
    E = 1.7
    D3 = O.constitutive(3, E, nu)
    keep = [0, 1, 5]  # exx, eyy, gxy in the 3D Voigt order [exx, eyy, ezz, gyz, gxz, gxy]
    Dpe = O.constitutive(2, E, nu, plane_stress=False)
    assert np.allclose(Dpe, D3[np.ix_(keep, keep)], rtol=1e-15, atol=0)
    Dps = O.constitutive(2, E / (1 - nu ** 2), nu / (1 - nu), plane_stress=True)
    assert np.allclose(Dpe, Dps, rtol=1e-14, atol=0)


def test_plane_strain_element_from_plane_stress_correspondence():
    """The plane-strain Q4 element equals the plane-stress element of the corresponding
    material (E / (1 - nu^2), nu / (1 - nu)), whose quadrature and closed forms are
    pinned above."""
    nu, h = 0.3, (0.5, 2.0)
    Kpe = O.element_stiffness(2, h, 1.0, nu, plane_stress=False)
    Kps = O.element_stiffness(2, h, 1.0 / (1 - nu ** 2), nu / (1 - nu), plane_stress=True)
    assert np.abs(Kpe - Kps).max() <= 1e-14 * np.abs(Kps).max()
