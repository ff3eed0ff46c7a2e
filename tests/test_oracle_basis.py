"""Pins of the oracle's basis construction (Sec. 4.2): POD of the snapshot window, the
Gram-Schmidt step of the new snapshot, the limited-memory window, and the property the
construction exists for: the ROM is exact at the trust-region centre."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W


def _window(N=300, m=6, seed=0, decay=0.3):
    """Snapshots with a spread of singular values: a common smooth field plus
    perturbations of geometrically decreasing size."""
    rng = np.random.default_rng(seed)
    x = np.linspace(0, 1, N)
    base = np.sin(np.pi * x) + 0.2 * x
    cols = [base]
    for i in range(1, m):
        cols.append(base + decay ** i * rng.standard_normal(N))
    return np.stack(cols, axis=1)


def test_pod_brute_force_small_cases():
    U = np.array([[3.0, 0.0], [0.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    Phi, s = O.pod(U, 1)
    assert np.allclose(s, [3.0, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(np.abs(Phi[:, 0]), [1, 0, 0, 0], atol=1e-15)
    # rank one: U = a b^T has the single direction a / |a| and sigma_1 = |a| |b|
    a = np.array([1.0, -2.0, 2.0]); b = np.array([3.0, 4.0])
    Phi, s = O.pod(np.outer(a, b), 1)
    assert abs(s[0] - 15.0) < 1e-13 and abs(s[1]) < 1e-13
    assert np.allclose(np.abs(Phi[:, 0]), np.abs(a) / 3.0, atol=1e-15)
    assert np.sign(Phi[0, 0] * Phi[1, 0]) == np.sign(a[0] * a[1])


def test_pod_is_the_optimal_subspace():
    """Eckart-Young-Schmidt: the n leading left singular vectors capture the largest
    snapshot energy of any n-dimensional subspace, and the energy they miss is the sum
    of the trailing squared singular values (the squared singular values being the
    eigenvalues of the snapshot Gram matrix, computed here by a symmetric eigensolver)."""
    U = _window(N=200, m=7, seed=4)
    lam = np.sort(sla.eigh(U.T @ U, eigvals_only=True))[::-1]
    rng = np.random.default_rng(9)
    for n in (1, 3, 5):
        Phi, s = O.pod(U, n)
        assert np.allclose(s ** 2, lam, rtol=1e-10, atol=1e-12 * lam[0])
        miss = np.linalg.norm(U - Phi @ (Phi.T @ U)) ** 2
        assert abs(miss - np.sum(s[n:] ** 2)) <= 1e-10 * np.sum(s ** 2)
        best = np.linalg.norm(Phi.T @ U) ** 2
        for _ in range(50):
            Q, _ = np.linalg.qr(rng.standard_normal((U.shape[0], n)))
            assert np.linalg.norm(Q.T @ U) ** 2 <= best * (1 + 1e-12)
        # the trailing directions are worse whenever the spectrum has a gap
        Wt, _ = O.pod(U, U.shape[1])
        assert np.linalg.norm(Wt[:, -n:].T @ U) ** 2 < best


def test_pod_ignores_window_order_and_sign():
    U = _window(N=150, m=5, seed=2)
    P1, s1 = O.pod(U, 3)
    P2, s2 = O.pod(U[:, [3, 0, 4, 2, 1]] * np.array([1, -1, 1, -1, 1]), 3)
    assert np.allclose(s1, s2, rtol=1e-13)
    assert np.allclose(P1 @ P1.T, P2 @ P2.T, atol=1e-12)


def test_gram_schmidt_step_brute_force_and_properties():
    Phi = np.array([[1.0], [0.0], [0.0]])
    q, nv, c = O.gram_schmidt_step(Phi, np.array([1.0, 2.0, 0.0]))
    assert np.allclose(q, [0, 1, 0]) and nv == 2.0 and np.allclose(c, [1.0])
    rng = np.random.default_rng(3)
    Phi, _ = np.linalg.qr(rng.standard_normal((80, 6)))
    u = rng.standard_normal(80)
    q, nv, c = O.gram_schmidt_step(Phi, u)
    assert np.abs(Phi.T @ q).max() < 1e-14
    assert abs(np.linalg.norm(q) - 1) < 1e-14
    assert np.allclose(Phi @ c + nv * q, u, atol=1e-13)
    # against no columns the step only normalises
    q, nv, c = O.gram_schmidt_step(np.zeros((80, 0)), u)
    assert np.allclose(q * nv, u) and c.shape == (0,)


def test_basis_update_orthonormal_nested_and_contains_new_snapshot():
    U = _window(N=240, m=6, seed=5)
    u = _window(N=240, m=8, seed=6)[:, -1]
    for n_max in (1, 4, 6, 10):
        Phi, n, keep, s = O.basis_update(U, u, n_max)
        assert n == min(6, n_max) and keep and Phi.shape[1] == n + 1
        assert np.abs(Phi[:, :n].T @ Phi[:, :n] - np.eye(n)).max() < 1e-13
        # one classical step leaves the new column orthogonal to O(eps |u| / |v|)
        _, nv, _ = O.gram_schmidt_step(Phi[:, :n], u)
        assert np.abs(Phi[:, :n].T @ Phi[:, n]).max() < 20 * np.finfo(float).eps * np.linalg.norm(u) / nv
        assert abs(np.linalg.norm(Phi[:, n]) - 1) < 1e-14
        co = np.linalg.lstsq(Phi, u, rcond=None)[0]
        assert np.linalg.norm(u - Phi @ co) < 1e-13 * np.linalg.norm(u)
        Pn, _ = O.pod(U, n)
        assert np.allclose(Phi[:, :n] @ Phi[:, :n].T, Pn @ Pn.T, atol=1e-12)
    # first centre: empty window, the basis is the normalised snapshot
    Phi, n, keep, s = O.basis_update(np.zeros((240, 0)), u, 5)
    assert n == 0 and keep and np.allclose(Phi[:, 0], u / np.linalg.norm(u))


def test_basis_update_drops_what_the_data_do_not_determine():
    U = _window(N=100, m=4, seed=7)
    Ud = np.concatenate([U, U[:, :2] + U[:, 2:3]], axis=1)  # rank 4, six columns
    Phi, n, keep, s = O.basis_update(Ud, None, 6, rtol=1e-9)
    assert n == 4 and Phi.shape[1] == 4 and s[4] < 1e-12 * s[0]
    # a new snapshot inside the span adds nothing
    Phi, n, keep, s = O.basis_update(Ud, U @ np.array([1.0, -2.0, 0.5, 3.0]), 6, rtol=1e-9)
    assert n == 4 and not keep and Phi.shape[1] == 4


def test_window_keeps_the_last_L_oldest_first():
    w = O.SnapshotWindow(4)
    for i in range(7):
        w.push(np.full(3, float(i)))
        assert len(w) == min(i + 1, 4)
    assert np.array_equal(w.matrix()[0], [3.0, 4.0, 5.0, 6.0])


@pytest.mark.parametrize("n_max", [1, 3])
def test_rom_is_exact_at_the_trust_region_centre(n_max):
    """Sec. 4.2: the basis holds the HDM solution at the centre whatever n_k is, so the
    ROM compliance equals the HDM compliance there and the ROM residual vanishes."""
    p = W.mbb2d(24, 8)
    m = p.mesh
    win = O.SnapshotWindow(3)
    for i in range(5):
        win.push(O.solve_direct(m, W.rho_smoothed(m, 40 + i), p.f, p.mask))
    rho_c = W.rho_smoothed(m, 77)
    u_c = O.solve_direct(m, rho_c, p.f, p.mask)
    Phi, n, keep, _ = O.basis_update(win.matrix(), u_c, n_max)
    assert keep and n == min(3, n_max)
    ev = O.rom_eval(m, rho_c, Phi, p.mask, p.f)
    J = O.compliance(p.f, u_c)
    # bounds: the direct solve's own residual here is about 5e-11 |f|
    assert abs(ev["Jk"] - J) <= 1e-10 * J
    assert ev["resnorm"] <= 1e-9 * np.linalg.norm(p.f)
    # away from the centre the ROM is not exact and its compliance is a lower bound
    rho_o = W.rho_smoothed(m, 91)
    eo = O.rom_eval(m, rho_o, Phi, p.mask, p.f)
    Jo = O.compliance(p.f, O.solve_direct(m, rho_o, p.f, p.mask))
    assert eo["Jk"] < Jo and eo["resnorm"] > 1e-6 * np.linalg.norm(p.f)


def test_tall_orthonormalisation_spans_the_columns():
    """The benchmark's Cholesky-QR orthonormalisation of tall bases: orthonormal to
    rounding, zero on Dirichlet rows, and the same span as the Householder QR."""
    p = W.cantilever3d(12, 6, 6)
    rng = np.random.default_rng(3)
    cols = np.hstack([rng.standard_normal((p.mesh.n_dofs, 5)), W.cosine_basis(p.mesh, p.mask, 40, 9, np.float64)])
    q = W.orthonormalize_tall(cols, p.mask)
    h = W.orthonormalize(cols, p.mask)
    assert np.abs(q.T @ q - np.eye(q.shape[1])).max() < 1e-13
    assert np.all(q[p.mask == 1] == 0)
    assert np.abs(q @ q.T - h @ h.T).max() < 1e-12
