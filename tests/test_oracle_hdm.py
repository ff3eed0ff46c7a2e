"""Pins of the oracle's full-order side: assembled K(rho), direct solve, compliance and
element sensitivity (Sec. 2.1-2.4), against mechanics, brute force and the paper."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _alpha(rho, m):
    return m.Emin + (m.E0 - m.Emin) * rho ** m.penal


def test_assembled_matrix_symmetric_and_spd_after_bcs():
    p = W.mbb2d(12, 4)
    rho = W.rho_jitter(p.mesh, 1)
    K = O.assemble(p.mesh, rho).toarray()
    assert np.abs(K - K.T).max() < 1e-14
    free = O.free_dofs(p.mask)
    Kff = K[np.ix_(free, free)]
    np.linalg.cholesky(Kff)  # raises if not SPD
    assert np.linalg.eigvalsh(Kff).min() > 0
    # without supports the matrix keeps its rigid modes
    assert np.sort(np.abs(np.linalg.eigvalsh(K)))[2] < 1e-12


def test_brute_force_two_element_assembly():
    """Hand assembly of a 2x1 Q4 mesh with the DOF map written out explicitly."""
    m = W.Mesh((2, 1))
    rho = np.array([0.7, 0.3])
    K0 = O.element_stiffness(2, (1, 1))
    n_nodes = 6  # nodes (i, j): i + 3 j
    # element 0 nodes (tensor order): (0,0),(1,0),(0,1),(1,1) -> 0,1,3,4
    # element 1 nodes: (1,0),(2,0),(1,1),(2,1) -> 1,2,4,5
    elems = [[0, 1, 3, 4], [1, 2, 4, 5]]
    K = np.zeros((12, 12))
    for e, nodes in enumerate(elems):
        dofs = [c * n_nodes + nd for nd in nodes for c in range(2)]
        K[np.ix_(dofs, dofs)] += _alpha(rho[e], m) * K0
    assert np.abs(O.assemble(m, rho).toarray() - K).max() < 1e-15


def test_brute_force_single_h8():
    m = W.Mesh((1, 1, 1))
    rho = np.array([0.6])
    K0 = O.element_stiffness(3, (1, 1, 1))
    dofs = [c * 8 + a for a in range(8) for c in range(3)]
    K = np.zeros((24, 24))
    K[np.ix_(dofs, dofs)] = _alpha(rho[0], m) * K0
    assert np.abs(O.assemble(m, rho).toarray() - K).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_linear_field(dim):
    """Uniform density, boundary DOFs prescribed from a linear displacement field:
    the interior reproduces the linear field to round-off."""
    nel = (6, 5) if dim == 2 else (4, 3, 3)
    m = W.Mesh(nel, h=(0.7, 1.3, 1.1)[:dim])
    rho = np.full(m.n_elems, 0.8)
    X = m.node_coords() * np.array(m.h)[:, None]
    A = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [0.2, 0.1, 0.25]])[:dim, :dim]
    b = np.array([0.1, -0.2, 0.3])[:dim]
    ulin = np.concatenate([A[c] @ X + b[c] for c in range(dim)])
    boundary = np.zeros(m.n_nodes, bool)
    for d in range(dim):
        boundary |= (m.node_coords()[d] == 0) | (m.node_coords()[d] == nel[d])
    mask = np.tile(boundary, dim).astype(np.uint8)
    K = O.assemble(m, rho)
    g = np.where(mask == 1, ulin, 0.0)
    u = O.solve_direct(m, rho, -(K @ g), mask) + g
    assert np.abs(u - ulin).max() < 1e-12
    # equivalently: interior rows of K u_lin vanish
    assert np.abs((K @ ulin)[mask == 0]).max() < 1e-12


def _tip_deflection_2d(nx, ny, L, H):
    m = W.Mesh((nx, ny), h=(L / nx, H / ny), Emin=0.0)
    mask = np.zeros(m.n_dofs, np.uint8)
    for j in range(ny + 1):
        mask[m.dof(0, m.node(0, j))] = mask[m.dof(1, m.node(0, j))] = 1
    f = np.zeros(m.n_dofs)
    tip = [m.node(nx, j) for j in range(ny + 1)]
    w = np.ones(ny + 1)
    w[0] = w[-1] = 0.5
    f[m.dof(1, np.array(tip))] = -w / ny  # unit total shear on the tip
    u = O.solve_direct(m, np.ones(m.n_elems), f, mask)
    return -np.mean(u[m.dof(1, np.array(tip))])


def test_slender_cantilever_2d_beam_theory():
    """Uniform-density slender cantilever (L/H = 20, plane stress, unit thickness,
    unit tip shear): tip deflection approaches the Timoshenko value
    P L^3/(3 E I) + P L/(kappa G A) from below (bilinear elements are too stiff in
    bending) and the gap shrinks under refinement."""
    L, H, E, nu = 20.0, 1.0, 1.0, 0.3
    I = H ** 3 / 12
    G = E / (2 * (1 + nu))
    ref = L ** 3 / (3 * E * I) + L / (5 / 6 * G * H)
    coarse = _tip_deflection_2d(160, 8, L, H) / ref
    fine = _tip_deflection_2d(320, 16, L, H) / ref
    assert 0.95 < coarse < fine < 1.005
    # Euler-Bernoulli alone within 1% as well
    assert abs(_tip_deflection_2d(320, 16, L, H) / (L ** 3 / (3 * E * I)) - 1) < 0.01


def test_slender_cantilever_3d_beam_theory():
    """Same check with trilinear H8 elements on a square-section cantilever (L/H = 10):
    below the Timoshenko value and converging towards it."""
    L, H, E, nu = 10.0, 1.0, 1.0, 0.3
    I = H ** 4 / 12
    G = E / (2 * (1 + nu))
    ref = L ** 3 / (3 * E * I) + L / (5 / 6 * G * H * H)

    def tip(nx, n):
        m = W.Mesh((nx, n, n), h=(L / nx, H / n, H / n), Emin=0.0)
        mask = np.zeros(m.n_dofs, np.uint8)
        for j in range(n + 1):
            for k in range(n + 1):
                for c in range(3):
                    mask[m.dof(c, m.node(0, j, k))] = 1
        f = np.zeros(m.n_dofs)
        w1 = np.ones(n + 1)
        w1[0] = w1[-1] = 0.5
        wf = np.outer(w1, w1) / n ** 2
        nodes = np.array([[m.node(nx, j, k) for k in range(n + 1)] for j in range(n + 1)])
        f[m.dof(2, nodes.ravel())] = -wf.ravel()
        u = O.solve_direct(m, np.ones(m.n_elems), f, mask)
        return -np.mean(u[m.dof(2, nodes.ravel())])

    coarse, fine = tip(20, 2) / ref, tip(40, 4) / ref
    assert 0.7 < coarse < fine < 1.005
    assert fine > 0.93


def test_uniform_density_scaling():
    """Uniform rho: K = alpha(rho) K_solid, so c(rho) = c_solid / alpha(rho) exactly."""
    p = W.cantilever2d(30, 10)
    m = p.mesh
    c1 = O.compliance(p.f, O.solve_direct(m, np.ones(m.n_elems), p.f, p.mask))
    for r in (0.5, 0.2):
        c = O.compliance(p.f, O.solve_direct(m, np.full(m.n_elems, r), p.f, p.mask))
        assert abs(c * _alpha(r, m) / c1 - 1) < 1e-12


def test_energy_identity_and_solution_residual():
    p = W.mbb2d(30, 10)
    rho = W.rho_jitter(p.mesh, 7)
    u = O.solve_direct(p.mesh, rho, p.f, p.mask)
    K = O.assemble(p.mesh, rho)
    free = p.mask == 0
    r = (p.f - K @ u)[free]
    # normwise backward error of a stable direct solve
    assert np.linalg.norm(r) / (abs(K).sum(axis=1).max() * np.linalg.norm(u)) < 1e-14
    c = O.compliance(p.f, u)
    assert abs(c - u @ (K @ u)) / c < 1e-12
    assert np.all(u[p.mask == 1] == 0)


def test_cg_agrees_with_direct():
    p = W.cantilever3d(8, 4, 4)
    rho = W.rho_smoothed(p.mesh, 3)
    ud = O.solve_direct(p.mesh, rho, p.f, p.mask)
    # the FP64 floor of the true residual on this mesh is ~5e-13 (direct solve too)
    uc, res = O.solve_cg(p.mesh, rho, p.f, p.mask, rtol=1e-12)
    assert res < 2e-12
    assert np.abs(uc - ud).max() / np.abs(ud).max() < 1e-9


def test_apply_rows_matches_assembled_apply():
    for p in (W.mbb2d(7, 3), W.bridge3d(4, 3, 2)):
        m = p.mesh
        rng = np.random.default_rng(0)
        rho = rng.uniform(0.1, 1, m.n_elems)
        x = rng.standard_normal(m.n_dofs)
        y = O.apply_masked(m, rho, p.mask, x)
        nodes = np.arange(m.n_nodes)
        yr = O.apply_rows(m, rho, p.mask, x, nodes)
        assert np.abs(yr.ravel() - y).max() < 1e-13
        assert np.all(y[p.mask == 1] == 0)


def test_apply_ebe_matches_assembled_apply_and_counts_cg_iterations():
    """The element-by-element product (no assembly; chunked) equals the assembled one;
    solve_cg reports its iteration count without changing its result."""
    for p in (W.mbb2d(9, 5), W.bridge3d(5, 3, 4), W.cantilever3d(3, 2, 2)):
        m = p.mesh
        rng = np.random.default_rng(1)
        rho = rng.uniform(0.1, 1, m.n_elems)
        x = rng.standard_normal(m.n_dofs)
        y = O.apply_masked(m, rho, p.mask, x)
        for chunk in (1 << 18, 7):
            ye = O.apply_ebe(m, rho, p.mask, x, chunk=chunk)
            assert np.abs(ye - y).max() <= 1e-14 * np.abs(y).max()
    p = W.cantilever3d(6, 3, 3)
    rho = W.rho_smoothed(p.mesh, 5)
    info = {}
    u1, r1 = O.solve_cg(p.mesh, rho, p.f, p.mask, rtol=1e-10, info=info)
    u2, r2 = O.solve_cg(p.mesh, rho, p.f, p.mask, rtol=1e-10)
    assert np.array_equal(u1, u2) and r1 == r2
    assert 10 < info["iters"] < 10 * p.mesh.n_dofs


def _fd_check(p, rho, elems, step=2e-4):
    """Central differences of the compliance in rho_e, Richardson-extrapolated from
    steps h and h/2 (truncation O(h^4)), for the listed elements."""
    m = p.mesh
    u = O.solve_direct(m, rho, p.f, p.mask)
    g = O.sensitivity(m, rho, u)

    def central(e, hs):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += hs
        rm[e] -= hs
        cp = O.compliance(p.f, O.solve_direct(m, rp, p.f, p.mask))
        cm = O.compliance(p.f, O.solve_direct(m, rm, p.f, p.mask))
        return (cp - cm) / (2 * hs)

    fd = []
    for e in elems:
        hs = step * rho[e]
        fd.append((4 * central(e, hs / 2) - central(e, hs)) / 3)
    return g, np.array(fd)


def test_sensitivity_finite_difference_2d():
    p = W.mbb2d(60, 20)
    rho = W.rho_jitter(p.mesh, 1000)
    rng = np.random.default_rng(5)
    elems = rng.choice(p.mesh.n_elems, 12, replace=False)
    elems = np.concatenate([elems, [0, p.mesh.n_elems - 1]])
    g, fd = _fd_check(p, rho, elems)
    scale = np.abs(g).max()
    assert np.abs(g[elems] - fd).max() / scale < 1e-7
    big = np.abs(g[elems]) > 1e-2 * scale
    assert np.all(np.abs(g[elems][big] - fd[big]) / np.abs(fd[big]) < 1e-6)


def test_sensitivity_finite_difference_3d():
    p = W.cantilever3d(6, 3, 3)
    rho = W.rho_smoothed(p.mesh, 11)
    elems = np.arange(0, p.mesh.n_elems, 7)
    g, fd = _fd_check(p, rho, elems)
    assert np.abs(g[elems] - fd).max() / np.abs(g).max() < 1e-6


def test_sensitivity_homogeneity_and_sign():
    """With Emin = 0 the compliance is homogeneous of degree -p in rho, so Euler's
    identity gives sum_e rho_e dc/drho_e = -p c; every sensitivity is <= 0."""
    for p in (W.mbb2d(30, 10, Emin=0.0), W.cantilever3d(6, 3, 3, Emin=0.0)):
        rho = W.rho_smoothed(p.mesh, 2) if p.mesh.dim == 3 else W.rho_jitter(p.mesh, 2)
        u = O.solve_direct(p.mesh, rho, p.f, p.mask)
        c = O.compliance(p.f, u)
        g = O.sensitivity(p.mesh, rho, u)
        assert abs(np.dot(rho, g) / (-p.mesh.penal * c) - 1) < 1e-11
        assert np.all(g <= 0)


def _paper(name):
    with open(os.path.join(GOLDEN, "paper_soft_pins.json")) as fh:
        return json.load(fh)["problems"][name]


@pytest.mark.parametrize("name,builder", [("mbb", W.paper_mbb), ("ssbeam", W.paper_ssbeam)])
def test_paper_initial_design_compliance(name, builder):
    """Soft pin: compliance of the paper's constant initial design, J(psi0) =
    J* (1 + e0) from the printed J* and the plotted initial relative error.  The
    tolerance covers the rounding of J* to its printed digits."""
    d = _paper(name)
    p = builder()
    rho = np.full(p.mesh.n_elems, d["psi0"])
    c = O.compliance(p.f, O.solve_direct(p.mesh, rho, p.f, p.mask))
    target = d["Jstar"] * (1 + d["e0"])
    tol = 0.5 * 10.0 ** (np.floor(np.log10(d["Jstar"])) - d["Jstar_digits"] + 1) / d["Jstar"]
    assert abs(c / target - 1) < 1.5 * tol


def test_fp64_definition_limit_of_the_600x200_workload(monkeypatch):
    """How tightly float64 defines the 600x200 cantilever's compliance and sensitivity:
    changing the oracle's element matrix by one rounding (its projection onto exact
    translation invariance, 1.1e-16 of its largest entry) moves the compliance by
    ~1e-9 and the sensitivity by ~1.4e-10 (max-norm), so no float64 evaluation of this
    operator (a different element-matrix rounding or summation order) can meet 1e-10 on
    them; the GPU parity gates on this workload are 2x these moves (2e-9, 3e-10).  On
    the 60x20 MBB workload the same change stays below 1e-10 (its gates are 1e-10)."""
    import oracle.fem as F
    out = {}
    for name in ("cantilever2d_600x200", "mbb2d_60x20"):
        cfg = W.config(name)
        p, m = cfg.problem, cfg.problem.mesh
        rho = cfg.rho(0)
        u0 = O.solve_direct(m, rho, p.f, p.mask)
        c0, g0 = O.compliance(p.f, u0), O.sensitivity(m, rho, u0)
        K0 = F._K0(m)
        Kp = K0.copy()
        for c in range(2):
            Kp[:, c::2] -= K0[:, c::2].sum(axis=1)[:, None] / 4
        Kp = 0.5 * (Kp + Kp.T)
        assert np.abs(Kp - K0).max() <= 2e-16 * np.abs(K0).max()
        with monkeypatch.context() as mp:
            mp.setattr(F, "_K0", lambda mesh, plane_stress=True: Kp)
            u1 = O.solve_direct(m, rho, p.f, p.mask)
            c1, g1 = O.compliance(p.f, u1), O.sensitivity(m, rho, u1)
        out[name] = (abs(c1 / c0 - 1), np.abs(g1 - g0).max() / np.abs(g0).max())
    dc, dg = out["cantilever2d_600x200"]
    assert 5e-10 < dc < 2e-9 and 5e-11 < dg < 3e-10, out
    dc, dg = out["mbb2d_60x20"]
    assert dc < 1e-10 and dg < 1e-10, out
