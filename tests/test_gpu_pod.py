"""GPU parity of the reduced-basis construction at a trust-region centre (Sec. 4.2):
snapshot window with its Gram matrix (topo_pod_push), POD of the window plus one
Gram-Schmidt step of the new snapshot (topo_pod_basis), against the oracle's SVD-based
definition, through the C ABI.

Tolerances follow from the arithmetic of the method of snapshots: the Gram matrix and
its Jacobi eigen-decomposition carry an absolute error of order m eps sigma_0^2 in the
squared singular values, so sigma_i is good to about m eps sigma_0^2 / sigma_i, POD
column j to about that error over sigma_j times the gaps to the other singular values,
and the Gram-Schmidt column to the error of the projector times |u| / |v|.  A POD
direction is only determined up to its sign, so columns are compared up to sign."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, dev, host, torch_cuda

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _snapshots(p, count, seed, decay):
    return W.snapshot_fields(p.mesh, p.mask, count, seed, decay)


def _new_snapshot(p, U, seed):
    """Mostly inside the window's span: half the sum of two snapshots plus 5 % of an
    unrelated field."""
    other = W.snapshot_fields(p.mesh, p.mask, 1, seed + 100, 0.5)[0]
    u = 0.5 * (U[0] + U[min(1, len(U) - 1)])
    return u + 0.05 * other * np.linalg.norm(u) / np.linalg.norm(other)


def _window(L, snaps):
    torch = torch_cuda()
    from paper_2004_05756_amd import binding
    sw = binding.SnapshotWindow(ctx(), snaps.shape[1], L)
    ow = O.SnapshotWindow(L)
    for x in snaps:
        sw.push(dev(x, torch.float64))
        ow.push(x)
    return sw, ow


def _col_tol(s, j, m):
    """Bound on the error of POD column j (max norm, columns of unit 2-norm)."""
    dl = 64 * m * EPS * s[0] ** 2
    gaps = [abs(s[j] - s[k]) for k in range(len(s)) if k != j]
    return sum(dl / (s[j] * g) for g in gaps) + dl / s[j] ** 2 + 1e-14


def _match_up_to_sign(a, b):
    return min(np.abs(a - b).max(), np.abs(a + b).max())


@pytest.mark.parametrize("L,pushes", [(1, 1), (1, 3), (4, 2), (5, 5), (5, 8), (48, 50)])
def test_window_push_gram_and_state(L, pushes):
    """The window holds the last L snapshots, oldest at `next` once full, and G is
    their Gram matrix (against the definition U^T U in slot order)."""
    p = W.mbb2d(13, 7)
    snaps = _snapshots(p, pushes, 21, 0.7)
    sw, ow = _window(L, snaps)
    count = min(pushes, L)
    assert sw.state[0] == count
    assert sw.state[1] == (pushes - L) % L if pushes > L else sw.state[1] == 0
    S = host(sw.S)[:count]
    # slot i holds push number i + L * k for the largest k that is still <= pushes - 1
    for i in range(count):
        last = max(q for q in range(pushes) if q % L == i)
        assert np.array_equal(S[i], snaps[last])
    G = host(sw.G)[:count, :count]
    ref = S @ S.T
    nrm = np.linalg.norm(S, axis=1)
    assert np.all(np.abs(G - ref) <= 2 * S.shape[1] * EPS * np.outer(nrm, nrm))
    assert np.array_equal(G, G.T)
    # the window's content (in age order) is the oracle's
    age = [(sw.state[1] + a) % L for a in range(count)] if pushes >= L else list(range(count))
    assert np.array_equal(S[age], ow.matrix().T)


CASES = [  # (problem, L, snapshots pushed, nmax, decay)
    (W.mbb2d(60, 20), 1, 1, 1, 0.5),
    (W.mbb2d(60, 20), 3, 3, 3, 0.5),
    (W.mbb2d(60, 20), 5, 8, 4, 0.5),
    (W.cantilever2d(37, 11), 7, 7, 7, 0.5),
    (W.cantilever3d(7, 5, 3), 6, 9, 2, 0.6),
    (W.bridge3d(6, 4, 5), 20, 20, 19, 0.8),
    (W.cantilever2d(600, 200), 20, 23, 19, 0.8),
    (W.mbb2d(60, 20), 48, 50, 47, 0.9),  # the largest window and basis
]


@pytest.mark.parametrize("p,L,pushes,nmax,decay", CASES, ids=lambda v: getattr(v, "name", str(v)))
@pytest.mark.parametrize("phi_dtype", ["f64", "f32"])
def test_pod_basis_matches_oracle(p, L, pushes, nmax, decay, phi_dtype):
    torch = torch_cuda()
    snaps = _snapshots(p, pushes, 5, decay)
    sw, ow = _window(L, snaps)
    U = ow.matrix()
    u = _new_snapshot(p, snaps[-min(L, pushes):], 9)
    m = U.shape[1]
    rtol = 1e-7
    Phi_o, n_o, keep_o, s_o = O.basis_update(U, u, nmax, rtol)
    dt = torch.float32 if phi_dtype == "f32" else torch.float64
    N = p.mesh.n_dofs
    ld = min(m, nmax) + 3  # wider than the basis: the extra columns must stay untouched
    phi = torch.full((N, ld), 7.0, dtype=dt, device="cuda")
    sig = torch.zeros(m, dtype=torch.float64, device="cuda")
    ncols, npod = sw.basis(dev(u, torch.float64), nmax, phi, rtol, sig)
    assert (npod, ncols) == (n_o, n_o + int(keep_o))
    P = host(phi).astype(np.float64)
    assert np.all(P[:, ncols:] == 7.0)
    s = host(sig)
    for i in range(m):
        assert abs(s[i] - s_o[i]) <= 64 * m * EPS * s_o[0] ** 2 / max(s_o[i], 1e-300) + 1e-15 * s_o[0]
    rnd = 2.0 ** -23 if phi_dtype == "f32" else 0.0
    for j in range(n_o):
        tol = _col_tol(s_o[:m], j, m) + rnd
        assert _match_up_to_sign(P[:, j], Phi_o[:, j]) <= tol, (j, tol)
    # the POD part is orthonormal to the accuracy of its directions
    Q = P[:, :n_o]
    orth = 64 * m * EPS * (s_o[0] / s_o[n_o - 1]) ** 2 + 2 * rnd if n_o else 0
    assert np.abs(Q.T @ Q - np.eye(n_o)).max() <= orth + 1e-13
    if keep_o:
        q = P[:, n_o]
        _, nv, _ = O.gram_schmidt_step(Phi_o[:, :n_o], u)
        lam = s_o[:m] ** 2
        theta = 64 * m * EPS * lam[0] / lam[n_o - 1] if n_o else 0.0
        if 0 < n_o < m:
            theta += 64 * m * EPS * lam[0] / (lam[n_o - 1] - lam[n_o])
        tol_q = 10 * (np.linalg.norm(u) / nv) * (theta + 1e-13) + rnd
        assert np.abs(q - Phi_o[:, n_o]).max() <= tol_q * np.abs(Phi_o[:, n_o]).max()
        assert abs(np.linalg.norm(q) - 1.0) <= 1e-12 + rnd
        # u lies in the span of the basis (the point of the construction)
        co = np.linalg.lstsq(P[:, :ncols], u, rcond=None)[0]
        span_tol = 1e-11 if phi_dtype == "f64" else 4 * rnd * np.sqrt(ncols)
        assert np.linalg.norm(u - P[:, :ncols] @ co) <= span_tol * np.linalg.norm(u)


def test_pod_basis_window_only_and_first_centre():
    torch = torch_cuda()
    p = W.cantilever2d(37, 11)
    snaps = _snapshots(p, 6, 13, 0.5)
    sw, ow = _window(6, snaps)
    N = p.mesh.n_dofs
    phi = torch.zeros((N, 4), dtype=torch.float64, device="cuda")
    ncols, npod = sw.basis(None, 4, phi)
    Phi_o, n_o, _, s_o = O.basis_update(ow.matrix(), None, 4)
    assert ncols == npod == n_o == 4
    P = host(phi)
    for j in range(4):
        assert _match_up_to_sign(P[:, j], Phi_o[:, j]) <= _col_tol(s_o, j, 6)
    # empty window: the basis is the normalised snapshot
    from paper_2004_05756_amd import binding
    empty = binding.SnapshotWindow(ctx(), N, 3)
    u = snaps[2]
    phi1 = torch.zeros((N, 1), dtype=torch.float64, device="cuda")
    assert empty.basis(dev(u, torch.float64), 5, phi1) == (1, 0)
    assert np.abs(host(phi1)[:, 0] - u / np.linalg.norm(u)).max() <= 1e-15
    # zero snapshot on an empty window: nothing to add
    assert empty.basis(torch.zeros(N, dtype=torch.float64, device="cuda"), 5, phi1) == (0, 0)


def test_pod_basis_drops_undetermined_directions_and_spanned_snapshot():
    torch = torch_cuda()
    p = W.mbb2d(60, 20)
    base = _snapshots(p, 4, 17, 0.5)
    snaps = np.concatenate([base, base[:2] + base[2:3], 2.0 * base[3:4]])  # rank 4, 7 columns
    sw, ow = _window(8, snaps)
    rtol = 1e-6
    u = base.T @ np.array([1.0, -2.0, 0.5, 3.0])  # inside the span
    N = p.mesh.n_dofs
    phi = torch.zeros((N, 8), dtype=torch.float64, device="cuda")
    ncols, npod = sw.basis(dev(u, torch.float64), 7, phi, rtol)
    Phi_o, n_o, keep_o, _ = O.basis_update(ow.matrix(), u, 7, rtol)
    assert (n_o, keep_o) == (4, False)
    assert (ncols, npod) == (4, 4)
    P = host(phi)[:, :4]
    assert np.allclose(P @ P.T @ ow.matrix(), ow.matrix(), rtol=0, atol=1e-9 * np.abs(snaps).max())


@pytest.mark.parametrize("n_max", [1, 3])
@pytest.mark.parametrize("phi_dtype", ["f64", "f32"])
def test_rom_exact_at_centre_through_gpu_basis(n_max, phi_dtype):
    """Sec. 4.2: with the basis built on the device from HDM snapshots (computed by the
    oracle's direct solver), the device ROM reproduces the HDM compliance at the centre."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64
    p = W.mbb2d(48, 16)
    m = p.mesh
    snaps = np.stack([O.solve_direct(m, W.rho_smoothed(m, 40 + i), p.f, p.mask) for i in range(5)])
    rho_c = W.rho_smoothed(m, 77)
    u_c = O.solve_direct(m, rho_c, p.f, p.mask)
    J = O.compliance(p.f, u_c)
    sw, _ = _window(3, snaps)
    dt = torch.float32 if phi_dtype == "f32" else torch.float64
    phi = torch.zeros((m.n_dofs, n_max + 1), dtype=dt, device="cuda")
    ncols, npod = sw.basis(dev(u_c, torch.float64), n_max, phi)
    assert (ncols, npod) == (n_max + 1, n_max)
    c = ctx()
    mask = dev(p.mask, torch.uint8)
    f = dev(p.f, torch.float64)
    Kh, fh = c.rom_build(m, phi, ncols, mask, f, dev(rho_c[None], torch.float64), prec=FP64)
    y, Jk = c.rom_solve(Kh, fh)
    Jk = float(host(Jk)[0])
    tol = 1e-9 * J
    if phi_dtype == "f32":
        # Rounding Phi to float32 moves u_c out of the span by at most 2^-24 |c|_1 (c its
        # coefficients in the basis); the compliance error is the square of that distance
        # in the energy norm, hence at most lambda_max(K) (2^-24 |c|_1)^2.
        import scipy.sparse.linalg as spla
        free = O.free_dofs(p.mask)
        K = O.assemble(m, rho_c)[free][:, free]
        lmax = float(spla.eigsh(K, k=1, which="LA", return_eigenvectors=False)[0])
        c1 = np.abs(np.linalg.lstsq(host(phi).astype(np.float64), u_c, rcond=None)[0]).sum()
        tol += lmax * (2.0 ** -24 * c1) ** 2
    assert -1e-10 * J <= J - Jk <= tol  # Galerkin: J_k <= J up to rounding


def test_pod_basis_full_size_bridge_window():
    """The 192 x 96 x 96 bridge (5,447,811 DOF) with a full window of 20 snapshots:
    singular values against the oracle's SVD, orthonormality, and the new snapshot in
    the span, checked on the device."""
    torch = torch_cuda()
    p = W.bridge3d(192, 96, 96)
    N = p.mesh.n_dofs
    snaps = _snapshots(p, 21, 31, 0.8)
    sw, ow = _window(20, snaps[:20])
    u = _new_snapshot(p, snaps[:20], 33)
    ud = dev(u, torch.float64)
    phi = torch.empty((N, 20), dtype=torch.float32, device="cuda")
    sig = torch.zeros(20, dtype=torch.float64, device="cuda")
    ncols, npod = sw.basis(ud, 19, phi, 1e-7, sig)
    s_o = np.linalg.svd(ow.matrix(), compute_uv=False)
    assert (ncols, npod) == (20, 19)
    s = host(sig)
    assert np.all(np.abs(s - s_o) <= 64 * 20 * EPS * s_o[0] ** 2 / s_o + 1e-15 * s_o[0])
    P = phi.double()
    gram = host(P.T @ P)
    assert np.abs(gram - np.eye(20)).max() <= 64 * 20 * EPS * (s_o[0] / s_o[18]) ** 2 + 2.0 ** -22
    co = np.linalg.solve(gram, host(P.T @ ud))  # normal equations: the basis is near-orthonormal
    res = ud - P @ torch.as_tensor(co, device="cuda")
    assert float(torch.linalg.norm(res)) <= 2.0 ** -20 * float(torch.linalg.norm(ud))


def test_pod_argument_errors():
    torch = torch_cuda()
    from paper_2004_05756_amd import binding
    c = ctx()
    N = 100
    u = torch.ones(N, dtype=torch.float64, device="cuda")
    S = torch.zeros((49, N), dtype=torch.float64, device="cuda")
    G = torch.zeros((49, 49), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.TopoError) as e:
        c.pod_push(S, G, [0, 0], u)  # window larger than the maximum
    assert e.value.code == binding.TOPO_EINVAL
    S, G = S[:4].contiguous(), G[:4, :4].contiguous()
    for state in ([5, 0], [2, 1], [4, 4], [-1, 0]):
        with pytest.raises(binding.TopoError):
            c.pod_push(S, G, list(state), u)
    st = [0, 0]
    for _ in range(3):
        c.pod_push(S, G, st, u * (1 + _))
    phi = torch.zeros((N, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.TopoError):
        c.pod_basis(S, G, 3, u, 3, phi)  # 3 POD columns + u need ldphi >= 4
    with pytest.raises(binding.TopoError):
        c.pod_basis(S, G, 3, u, 2, phi, rtol=1.0)
    with pytest.raises(binding.TopoError):
        c.pod_basis(S, G, 0, None, 2, phi)  # nothing to build
    # rank-one window (all pushes parallel): one POD column, u inside its span
    assert c.pod_basis(S, G, 3, u, 2, phi, rtol=1e-6) == (1, 1)
