"""Pins of the oracle's ROM side (Sec. 3): reduced operator, reduced solve, ROM
compliance and the residual-norm indicator, against the remarks and theorems of
Sec. 3 and brute force."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _setup(nx=30, ny=10, k=6, seed=3):
    p = W.mbb2d(nx, ny)
    rho = W.rho_jitter(p.mesh, seed)
    phi = W.cosine_basis(p.mesh, p.mask, k, seed, np.float64)
    return p, rho, phi


def _alpha(rho, m):
    return m.Emin + (m.E0 - m.Emin) * rho ** m.penal


def test_operator_equals_elementwise_contraction():
    """Brute force of the element-sum form of the reduced stiffness (Sec. 3.1):
    sum_e alpha_e (P_e^T Phi)^T K_e (P_e^T Phi), written with explicit loops."""
    for p in (W.mbb2d(5, 3), W.cantilever3d(3, 2, 2)):
        m = p.mesh
        rho = np.random.default_rng(1).uniform(0.1, 1, m.n_elems)
        phi = W.cosine_basis(m, p.mask, 5, 2, np.float64)
        K0 = O.element_stiffness(m.dim, m.h)
        edofs = O.element_dofs(m)
        Kh = np.zeros((5, 5))
        phim = phi.copy()
        phim[p.mask == 1] = 0
        for e in range(m.n_elems):
            Pe = phim[edofs[e]]
            Kh += _alpha(rho[e], m) * Pe.T @ K0 @ Pe
        assert np.allclose(O.rom_operator(m, rho, phi, p.mask), Kh, rtol=1e-13, atol=1e-15)
        fh = np.zeros(5)
        for i in range(m.n_dofs):
            if p.mask[i] == 0:
                fh += phi[i] * p.f[i]
        assert np.allclose(O.rom_load(phi, p.mask, p.f), fh, rtol=1e-14, atol=1e-16)


def test_reduced_operator_spd_and_symmetric():
    p, rho, phi = _setup()
    Kh = O.rom_operator(p.mesh, rho, phi, p.mask)
    assert np.abs(Kh - Kh.T).max() < 1e-13 * np.abs(Kh).max()
    assert np.linalg.eigvalsh(Kh).min() > 0


def test_rank_deficient_basis_is_not_spd():
    p, rho, phi = _setup()
    phi[:, -1] = phi[:, 0]
    Kh = O.rom_operator(p.mesh, rho, phi, p.mask)
    ev = np.linalg.eigvalsh(Kh)
    assert abs(ev[0]) < 1e-13 * ev[-1]


def test_exactness_when_solution_in_span():
    """Remark (exactness): u* in span(Phi) => u_k = u*, J_k = J, ||r|| ~ 0."""
    p, rho, phi = _setup()
    u = O.solve_direct(p.mesh, rho, p.f, p.mask)
    basis = np.column_stack([phi, u])
    ev = O.rom_eval(p.mesh, rho, basis, p.mask, p.f)
    J = O.compliance(p.f, u)
    assert abs(ev["Jk"] / J - 1) < 1e-12
    assert ev["resnorm"] / np.linalg.norm(p.f) < 1e-10
    _, _, uk = O.rom_residual(p.mesh, rho, basis, p.mask, p.f, ev["yhat"])
    assert np.abs(uk - u).max() / np.abs(u).max() < 1e-10


def test_complete_basis_zero_estimate():
    """k = N_free (identity basis on the free DOFs): the error indicator vanishes."""
    p = W.mbb2d(6, 3)
    rho = W.rho_jitter(p.mesh, 9)
    free = O.free_dofs(p.mask)
    phi = np.zeros((p.mesh.n_dofs, len(free)))
    phi[free, np.arange(len(free))] = 1.0
    # mix the columns so the basis is not trivially the identity
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((len(free), len(free))))
    ev = O.rom_eval(p.mesh, rho, phi @ Q, p.mask, p.f)
    assert ev["resnorm"] / np.linalg.norm(p.f) < 1e-12
    J = O.compliance(p.f, O.solve_direct(p.mesh, rho, p.f, p.mask))
    assert abs(ev["Jk"] / J - 1) < 1e-12


def test_compliance_error_identity_and_bound():
    """For compliance: J - J_k = r^T K^{-1} r = ||u* - u_k||_K^2 >= 0, and
    |J - J_k| <= ||r||^2 / sigma_min(K) (Sec. 3.3, compliance remark)."""
    p, rho, phi = _setup(20, 8, 5)
    m = p.mesh
    u = O.solve_direct(m, rho, p.f, p.mask)
    J = O.compliance(p.f, u)
    ev = O.rom_eval(m, rho, phi, p.mask, p.f)
    r, rn, uk = O.rom_residual(m, rho, phi, p.mask, p.f, ev["yhat"])
    e = O.solve_direct(m, rho, r, p.mask)  # K^{-1} r
    K = O.assemble(m, rho)
    assert J - ev["Jk"] > 0
    assert abs((J - ev["Jk"]) / (r @ e) - 1) < 1e-9
    du = u - uk
    assert abs((J - ev["Jk"]) / (du @ (K @ du)) - 1) < 1e-9
    free = O.free_dofs(p.mask)
    smin = np.linalg.eigvalsh(K.toarray()[np.ix_(free, free)]).min()
    assert J - ev["Jk"] <= rn ** 2 / smin * (1 + 1e-12)


def test_primal_energy_error_bound():
    """Theorem (primal error): ||u* - u_k||_K <= sigma_min(K)^{-1/2} ||r||."""
    p, rho, phi = _setup(20, 8, 4, seed=5)
    m = p.mesh
    u = O.solve_direct(m, rho, p.f, p.mask)
    ev = O.rom_eval(m, rho, phi, p.mask, p.f)
    r, rn, uk = O.rom_residual(m, rho, phi, p.mask, p.f, ev["yhat"])
    K = O.assemble(m, rho)
    free = O.free_dofs(p.mask)
    smin = np.linalg.eigvalsh(K.toarray()[np.ix_(free, free)]).min()
    du = u - uk
    assert np.sqrt(du @ (K @ du)) <= smin ** -0.5 * rn * (1 + 1e-12)


def test_invariance_under_change_of_basis():
    """The Galerkin solution depends only on span(Phi) (Sec. 3.1, optimality remark)."""
    p, rho, phi = _setup()
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((phi.shape[1],) * 2))
    a = O.rom_eval(p.mesh, rho, phi, p.mask, p.f)
    b = O.rom_eval(p.mesh, rho, phi @ Q, p.mask, p.f)
    assert abs(a["Jk"] / b["Jk"] - 1) < 1e-12
    assert abs(a["resnorm"] / b["resnorm"] - 1) < 1e-10
    assert np.allclose(Q @ b["yhat"], a["yhat"], rtol=1e-9, atol=1e-12 * np.abs(a["yhat"]).max())


def test_monotone_enrichment():
    """Remark (refinement): adding columns never increases the energy error, so J_k is
    non-decreasing towards J."""
    p, rho, phi = _setup(30, 10, 10)
    m = p.mesh
    u = O.solve_direct(m, rho, p.f, p.mask)
    J = O.compliance(p.f, u)
    K = O.assemble(m, rho)
    prevJ, preve = -np.inf, np.inf
    for k in range(1, 11):
        ev = O.rom_eval(m, rho, phi[:, :k], p.mask, p.f)
        _, _, uk = O.rom_residual(m, rho, phi[:, :k], p.mask, p.f, ev["yhat"])
        err = (u - uk) @ (K @ (u - uk))
        assert ev["Jk"] >= prevJ - 1e-12 * J and ev["Jk"] <= J * (1 + 1e-12)
        assert err <= preve + 1e-12 * J
        prevJ, preve = ev["Jk"], err


def test_zero_coefficients_residual_is_load_norm():
    """||r(0; rho)|| = ||f|| over the free DOFs (the paper's initial trust-region radius)."""
    p, rho, phi = _setup()
    _, rn, _ = O.rom_residual(p.mesh, rho, phi, p.mask, p.f, np.zeros(phi.shape[1]))
    assert rn == pytest.approx(np.linalg.norm(p.f[p.mask == 0]), rel=1e-15)


def test_masked_rows_are_ignored():
    p, rho, phi = _setup()
    noisy = phi.copy()
    noisy[p.mask == 1] = 123.0
    a = O.rom_eval(p.mesh, rho, phi, p.mask, p.f)
    b = O.rom_eval(p.mesh, rho, noisy, p.mask, p.f)
    assert np.array_equal(a["Khat"], b["Khat"]) and a["Jk"] == b["Jk"]


def test_rom_gradient_matches_finite_differences():
    """dJ_k/drho_e by central differences of the ROM compliance itself (each J_k from
    K_hat, f_hat and the reduced Cholesky solve, no sensitivity formula), 2D and 3D."""
    for p, k in ((W.mbb2d(12, 5), 6), (W.cantilever3d(4, 3, 2), 7)):
        m = p.mesh
        rho = np.random.default_rng(4).uniform(0.2, 1.0, m.n_elems)
        phi = W.cosine_basis(m, p.mask, k, 5, np.float64)
        g, J = O.rom_gradient(m, rho, phi, p.mask, p.f)
        for e in (0, m.n_elems // 3, m.n_elems - 1):
            h = 1e-6 * rho[e]
            rp, rm = rho.copy(), rho.copy()
            rp[e] += h
            rm[e] -= h
            fd = (O.rom_eval(m, rp, phi, p.mask, p.f)["Jk"] - O.rom_eval(m, rm, phi, p.mask, p.f)["Jk"]) / (2 * h)
            assert abs(g[e] - fd) <= 1e-6 * abs(fd) + 1e-12 * abs(J)
        assert np.all(g <= 0)


def test_rom_gradient_homogeneity():
    """With Emin = 0 the reduced stiffness scales as t^p under rho -> t rho, so J_k is
    homogeneous of degree -p and sum_e rho_e dJ_k/drho_e = -p J_k (Euler)."""
    import dataclasses
    p = W.mbb2d(16, 6)
    m = dataclasses.replace(p.mesh, Emin=0.0)
    rho = np.random.default_rng(8).uniform(0.1, 1.0, m.n_elems)
    phi = W.cosine_basis(m, p.mask, 8, 3, np.float64)
    g, J = O.rom_gradient(m, rho, phi, p.mask, p.f)
    assert abs(np.dot(rho, g) / (-m.penal * J) - 1) < 1e-12


def test_rom_gradient_exact_when_solution_in_span():
    """u*(rho) in span(Phi): the ROM state is the HDM state, so the ROM sensitivity is
    the HDM one (Sec. 3.3 sensitivity error with a zero residual)."""
    p = W.mbb2d(20, 8)
    rho = W.rho_jitter(p.mesh, 6)
    u = O.solve_direct(p.mesh, rho, p.f, p.mask)
    phi = np.column_stack([W.cosine_basis(p.mesh, p.mask, 4, 2, np.float64), u])
    g, _ = O.rom_gradient(p.mesh, rho, phi, p.mask, p.f)
    g0 = O.sensitivity(p.mesh, rho, u)
    assert np.abs(g - g0).max() <= 1e-9 * np.abs(g0).max()
