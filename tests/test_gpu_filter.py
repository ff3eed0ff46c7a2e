"""GPU parity of the Helmholtz density filter (Sec. 2.2) and of the gradient through it
(Sec. 2.4) against the oracle's direct solves, through the C ABI.

The device solves H phi = b by float64 Jacobi-PCG to |b - H phi| <= rtol |b|, so its
filtered densities differ from the direct solve by at most about kappa(H) rtol
(relative); each case's tolerance is 10 kappa(H) rtol with kappa(H) from the oracle's
assembled matrix."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import filter as F
import workloads as W
from gpu_util import ctx, dev, host, torch_cuda

pytestmark = pytest.mark.gpu

RTOL = 1e-13


def _kappa(m, r):
    H, _ = F.helmholtz_assemble(m, r)
    if H.shape[0] <= 64:
        ev = np.linalg.eigvalsh(H.toarray())
        return ev[-1] / ev[0]
    lmax = spla.eigsh(H, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(H, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return lmax / lmin


CASES = [  # (mesh, filter radius R); the last two have non-square elements
    (W.mbb2d(13, 7).mesh, 1.2), (W.mbb2d(60, 20).mesh, 2.0), (W.mbb2d(60, 20).mesh, 0.0),
    (W.cantilever2d(37, 11).mesh, 3.5), (W.cantilever3d(7, 5, 3).mesh, 1.0),
    (W.bridge3d(6, 4, 5).mesh, 2.5), (W.mbb2d(1, 1).mesh, 1.0),
    (W.Mesh(nel=(17, 9), h=(0.5, 2.0)), 1.5), (W.Mesh(nel=(6, 5, 7), h=(0.7, 1.3, 0.4)), 0.8),
]


@pytest.mark.parametrize("m,R", CASES, ids=lambda v: str(getattr(v, "nel", v)))
def test_filter_forward_and_adjoint_match_oracle(m, R):
    torch = torch_cuda()
    r = F.filter_radius(R)
    rng = np.random.default_rng(3)
    B = 3
    psi = rng.uniform(0, 1, (B, m.n_elems))
    v = rng.standard_normal((B, m.n_elems))
    tol = 10 * _kappa(m, r) * RTOL
    c = ctx()
    phi = torch.empty((B, m.n_nodes), dtype=torch.float64, device="cuda")
    rho, its = c.filter_forward(m, r, dev(psi, torch.float64), phi=phi, rtol=RTOL)
    g, its2 = c.filter_adjoint(m, r, dev(v, torch.float64), rtol=RTOL)
    rho, g, phi = host(rho), host(g), host(phi)
    for b in range(B):
        ro, pho = F.filter_forward(m, r, psi[b])
        go, _ = F.filter_adjoint(m, r, v[b])
        assert np.abs(rho[b] - ro).max() <= tol * np.abs(ro).max()
        assert np.abs(phi[b] - pho).max() <= tol * np.abs(pho).max()
        assert np.abs(g[b] - go).max() <= tol * np.abs(go).max()
    assert its >= 1 and its2 >= 1


def test_filter_batch_invariance_and_dot_product():
    torch = torch_cuda()
    m = W.cantilever2d(37, 11).mesh
    r = F.filter_radius(2.0)
    rng = np.random.default_rng(6)
    w = rng.uniform(0, 1, (4, m.n_elems))
    c = ctx()
    all4, _ = c.filter_forward(m, r, dev(w, torch.float64), rtol=1e-12)
    one, _ = c.filter_forward(m, r, dev(w[2:3], torch.float64), rtol=1e-12)
    assert torch.equal(all4[2:3], one)
    v = rng.standard_normal((1, m.n_elems))
    Aw, _ = c.filter_forward(m, r, dev(w[:1], torch.float64), rtol=RTOL)
    ATv, _ = c.filter_adjoint(m, r, dev(v, torch.float64), rtol=RTOL)
    lhs = float(v[0] @ host(Aw)[0])
    rhs = float(host(ATv)[0] @ w[0])
    assert abs(lhs - rhs) <= 10 * _kappa(m, r) * RTOL * np.abs(v).sum()


def test_gradient_through_filter_on_device_matches_oracle():
    """dJ/dpsi = (d rho*/d psi)^T dc/drho at rho = rho*(psi), every step on the device
    (filter, HDM solve, HDM sensitivity, adjoint filter)."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64
    p = W.mbb2d(60, 20)
    m = p.mesh
    r = F.filter_radius(2.0)
    psi = np.random.default_rng(12).uniform(0.2, 0.9, m.n_elems)
    c = ctx()
    rho_d, _ = c.filter_forward(m, r, dev(psi[None], torch.float64), rtol=RTOL)
    u_d, inf = c.hdm_solve(m, rho_d[0], dev(p.mask, torch.uint8), dev(p.f, torch.float64), rtol=1e-12,
                           prec=FP64)
    dc_d = c.hdm_gradient(m, rho_d[0], u_d)
    g_d, _ = c.filter_adjoint(m, r, dc_d.reshape(1, -1), rtol=RTOL)
    rho_o, _ = F.filter_forward(m, r, psi)
    u_o = O.solve_direct(m, rho_o, p.f, p.mask)
    g_o, _ = F.filter_adjoint(m, r, O.sensitivity(m, rho_o, u_o))
    # the elasticity solve to 1e-12 leaves about cond(K) 1e-12 in u and dc/drho
    assert np.abs(host(g_d)[0] - g_o).max() <= 1e-6 * np.abs(g_o).max()


def test_filter_full_size_2d_against_oracle():
    """The 600 x 200 mesh (120,801 nodes), the oracle's direct solve element by element."""
    torch = torch_cuda()
    m = W.cantilever2d(600, 200).mesh
    r = F.filter_radius(3.0)
    psi = W.rho_smoothed(m, 2001)
    rho, its = ctx().filter_forward(m, r, dev(psi[None], torch.float64), rtol=1e-12)
    ro, _ = F.filter_forward(m, r, psi)
    assert np.abs(host(rho)[0] - ro).max() <= 1e-8 * np.abs(ro).max()


def test_filter_full_size_3d_properties():
    """96 x 48 x 48 (232,897 nodes): constants are kept and volume is preserved; the
    volume changes by at most 1^T (b - H phi) <= sqrt(N_n) rtol |b|."""
    torch = torch_cuda()
    m = W.cantilever3d(96, 48, 48).mesh
    r = F.filter_radius(1.5)
    c = ctx()
    rho, _ = c.filter_forward(m, r, torch.full((1, m.n_elems), 0.4, dtype=torch.float64, device="cuda"),
                              rtol=1e-12)
    assert float((rho - 0.4).abs().max()) <= 1e-12
    psi = W.rho_smoothed(m, 3001)
    rho, _ = c.filter_forward(m, r, dev(psi[None], torch.float64), rtol=1e-12)
    bnorm = np.linalg.norm(F.filter_load(m, r, psi))
    assert abs(float(rho.sum()) - psi.sum()) <= np.sqrt(m.n_nodes) * 1e-12 * bnorm  # unit elements


def test_filter_argument_errors():
    torch = torch_cuda()
    from paper_2004_05756_amd import binding
    m = W.mbb2d(4, 3).mesh
    c = ctx()
    x = torch.zeros((1, m.n_elems), dtype=torch.float64, device="cuda")
    for kw in ({"rtol": 0.0}, {"rtol": 1.5}, {"maxit": 0}):
        with pytest.raises(binding.TopoError):
            c.filter_forward(m, 1.0, x, **kw)
    with pytest.raises(binding.TopoError):
        c.filter_forward(m, -1.0, x)
    # a field that cannot converge within the iteration cap reports TOPO_ENOCONV
    with pytest.raises(binding.TopoError) as e:
        c.filter_forward(m, 5.0, torch.rand((1, m.n_elems), dtype=torch.float64, device="cuda"),
                         rtol=1e-14, maxit=1)
    assert e.value.code == binding.TOPO_ENOCONV
    # psi = 0 is converged at once
    rho, its = c.filter_forward(m, 1.0, x)
    assert float(rho.abs().max()) == 0.0


def test_filter_warm_start():
    """With TOPO_FILTER_WARM the nodal array is the initial guess: the field's own solution
    takes no iteration and gives the same output; a nearby design's solution converges in
    fewer iterations to the same tolerance."""
    torch = torch_cuda()
    m = W.cantilever2d(37, 11).mesh
    r = F.filter_radius(2.0)
    rng = np.random.default_rng(21)
    psi = rng.uniform(0, 1, (1, m.n_elems))
    psi2 = np.clip(psi + 0.01 * rng.standard_normal(psi.shape), 0, 1)
    c = ctx()
    phi = torch.empty((1, m.n_nodes), dtype=torch.float64, device="cuda")
    rho, its = c.filter_forward(m, r, dev(psi, torch.float64), phi=phi, rtol=RTOL)
    again, its0 = c.filter_forward(m, r, dev(psi, torch.float64), phi=phi.clone(), rtol=RTOL, warm=True)
    assert its0 == 0 and torch.equal(again, rho)
    _, its_cold = c.filter_forward(m, r, dev(psi2, torch.float64), rtol=RTOL)
    rho2, its_warm = c.filter_forward(m, r, dev(psi2, torch.float64), phi=phi.clone(), rtol=RTOL, warm=True)
    assert its_warm < its_cold
    ro, _ = F.filter_forward(m, r, psi2[0])
    assert np.abs(host(rho2)[0] - ro).max() <= 10 * _kappa(m, r) * RTOL * np.abs(ro).max()
    v = -rng.uniform(0, 1, (1, m.n_elems))
    mu = torch.empty((1, m.n_nodes), dtype=torch.float64, device="cuda")
    g, _ = c.filter_adjoint(m, r, dev(v, torch.float64), mu=mu, rtol=RTOL)
    g2, its_a = c.filter_adjoint(m, r, dev(v * 1.001, torch.float64), mu=mu, rtol=RTOL, warm=True)
    go, _ = F.filter_adjoint(m, r, v[0] * 1.001)
    assert np.abs(host(g2)[0] - go).max() <= 10 * _kappa(m, r) * RTOL * np.abs(go).max()
