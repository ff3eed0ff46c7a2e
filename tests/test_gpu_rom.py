"""GPU parity of the ROM path (K_hat contraction on the matrix cores, f_hat, reduced
Cholesky solve, residual error indicator with reduced refinement) against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import ctx, dev, host, problem_tensors, rel, torch_cuda

pytestmark = pytest.mark.gpu

CASES = [  # (problem, k) -- ragged k, several tiles, 2D and 3D
    (W.mbb2d(13, 7), 5), (W.mbb2d(60, 20), 8), (W.cantilever2d(37, 11), 33),
    (W.cantilever3d(7, 5, 3), 17), (W.bridge3d(6, 4, 5), 40), (W.mbb2d(1, 1), 3),
]


def _basis(p, k, dtype, seed=7):
    return W.cosine_basis(p.mesh, p.mask, k, seed, dtype)


def _rhos(p, B, seed=11):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 1.0, (B, p.mesh.n_elems))


@pytest.mark.parametrize("p,k", CASES, ids=lambda v: getattr(v, "name", str(v)))
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_rom_build_matches_oracle(p, k, mode):
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    phi = _basis(p, k, np.float32)
    B = 3
    rhos = _rhos(p, B)
    Kh, fh = ctx().rom_build(p.mesh, dev(phi), k, dev(p.mask, torch.uint8), dev(p.f, torch.float64),
                             dev(rhos, torch.float64), prec=FP64 if mode == "fp64" else MIXED)
    Kh, fh = host(Kh), host(fh)
    tol = 1e-13 if mode == "fp64" else 2e-6
    for b in range(B):
        ref = O.rom_operator(p.mesh, rhos[b], phi, p.mask)
        assert np.array_equal(Kh[b], Kh[b].T)
        assert np.abs(Kh[b] - ref).max() <= tol * np.abs(ref).max()
    assert np.abs(fh - O.rom_load(phi, p.mask, p.f)).max() <= 1e-14 * max(np.abs(fh).max(), 1e-300) + 1e-300


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_rom_build_smooth_basis_entrywise(mode):
    """K_hat of a smooth basis on a 3D mesh of some size, every entry against the oracle
    relative to sqrt(K_ii K_jj) (Cauchy-Schwarz bound of the entry).  K Phi of smooth
    fields cancels element contributions at every node, and Phi^T (K Phi) sums terms far
    larger than the result when a column has a large translation-like part, so the
    contraction runs in float64 in both precisions and must meet the oracle to 1e-10."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    p, k = W.cantilever3d(32, 16, 16), 12
    phi = _basis(p, k, np.float32, seed=21)
    rhos = _rhos(p, 2, 23)
    Kh, _ = ctx().rom_build(p.mesh, dev(phi), k, dev(p.mask, torch.uint8), dev(p.f, torch.float64),
                            dev(rhos, torch.float64), prec=FP64 if mode == "fp64" else MIXED)
    Kh = host(Kh)
    for b in range(2):
        ref = O.rom_operator(p.mesh, rhos[b], phi, p.mask)
        d = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert (np.abs(Kh[b] - ref) / d).max() <= 1e-10


@pytest.mark.parametrize("p,k", CASES[:4], ids=lambda v: getattr(v, "name", str(v)))
def test_rom_solve_and_estimate(p, k):
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    phi = _basis(p, k, np.float32)
    B = 2
    rhos = _rhos(p, B, 5)
    m = dev(p.mask, torch.uint8)
    f = dev(p.f, torch.float64)
    phid = dev(phi)
    for mode, tolJ in (("fp64", 1e-10), ("mixed", 1e-8)):
        prec = FP64 if mode == "fp64" else MIXED
        r = dev(rhos, torch.float64)
        Kh, fh = ctx().rom_build(p.mesh, phid, k, m, f, r, prec=prec)
        y, J = ctx().rom_solve(Kh, fh)
        y, J2, rn = ctx().rom_estimate(p.mesh, phid, k, m, f, r, Kh, y, max_refine=2)
        y, J2, rn = host(y), host(J2), host(rn)
        for b in range(B):
            ev = O.rom_eval(p.mesh, rhos[b], phi, p.mask, p.f)
            assert abs(J2[b] / ev["Jk"] - 1) <= tolJ
            assert abs(rn[b] / ev["resnorm"] - 1) <= 1e-8
            if mode == "fp64":
                assert rel(y[b], ev["yhat"]) <= 1e-8


def test_rom_solve_fp64_matches_cholesky():
    torch = torch_cuda()
    rng = np.random.default_rng(3)
    # register / packed-LDS / global-memory paths of the factorisation and substitution
    for k in (1, 7, 16, 17, 40, 64, 65, 96, 100, 127, 128, 129, 130, 257):
        A = rng.standard_normal((k, k))
        K = A @ A.T + k * np.eye(k)
        fh = rng.standard_normal(k)
        y, J = ctx().rom_solve(dev(K[None]), dev(fh))
        yo, Jo = O.rom_solve(K, fh)
        assert rel(host(y)[0], yo) <= 1e-12
        assert abs(host(J)[0] / Jo - 1) <= 1e-12


def test_estimate_zero_coefficients_is_load_norm():
    torch = torch_cuda()
    p, k = W.mbb2d(60, 20), 8
    phi = _basis(p, k, np.float32)
    rho = W.rho_jitter(p.mesh, 1000)
    y = torch.zeros((1, k), dtype=torch.float64, device="cuda")
    _, J, rn = ctx().rom_estimate(p.mesh, dev(phi), k, dev(p.mask, torch.uint8),
                                  dev(p.f, torch.float64), dev(rho[None], torch.float64), None, y,
                                  max_refine=0)
    assert abs(host(rn)[0] / np.linalg.norm(p.f[p.mask == 0]) - 1) < 1e-15
    assert host(J)[0] == 0.0


def test_exactness_with_snapshot_in_basis():
    """u*(rho) in span(Phi): J_k = J and the indicator vanishes (FP64 basis)."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64
    p = W.mbb2d(60, 20)
    rho = W.rho_jitter(p.mesh, 1000)
    u = O.solve_direct(p.mesh, rho, p.f, p.mask)
    phi = np.column_stack([_basis(p, 7, np.float64), u])
    k = phi.shape[1]
    m, f, r = dev(p.mask, torch.uint8), dev(p.f, torch.float64), dev(rho[None], torch.float64)
    Kh, fh = ctx().rom_build(p.mesh, dev(phi), k, m, f, r, prec=FP64)
    y, J = ctx().rom_solve(Kh, fh)
    y, J, rn = ctx().rom_estimate(p.mesh, dev(phi), k, m, f, r, Kh, y, max_refine=1)
    assert abs(host(J)[0] / O.compliance(p.f, u) - 1) < 1e-11
    assert host(rn)[0] / np.linalg.norm(p.f) < 1e-9


def test_rank_deficient_basis_not_spd():
    torch = torch_cuda()
    from paper_2004_05756_amd import MIXED, TopoError, binding
    p, k = W.mbb2d(30, 10), 6
    phi = _basis(p, k, np.float32)
    phi[:, 5] = phi[:, 2]
    m, f = dev(p.mask, torch.uint8), dev(p.f, torch.float64)
    r = dev(W.rho_jitter(p.mesh, 2)[None], torch.float64)
    Kh, fh = ctx().rom_build(p.mesh, dev(phi), k, m, f, r, prec=MIXED)
    with pytest.raises(TopoError) as ei:
        ctx().rom_solve(Kh, fh)
    assert ei.value.code == binding.TOPO_ENOTSPD
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx().rom_solve(Kh, fh, status=st)
    assert int(st[0]) == binding.TOPO_ENOTSPD


def test_refinement_accepts_and_reverts_per_field():
    """Device-side refinement decisions in one batch: field 0 gets a good K_hat (step
    kept, FP64-accurate J), field 1 a K_hat scaled by 0.1 (the step overshoots, the
    Galerkin residual grows, y is restored), field 2 a K_hat that does not factor (no
    step).  Fields 1 and 2 must report exactly what max_refine=0 reports for their y."""
    torch = torch_cuda()
    from paper_2004_05756_amd import MIXED
    p, k = W.cantilever2d(37, 11), 12
    phi = _basis(p, k, np.float32)
    rhos = _rhos(p, 3, 21)
    m, f, phid = dev(p.mask, torch.uint8), dev(p.f, torch.float64), dev(phi)
    r = dev(rhos, torch.float64)
    Kh, fh = ctx().rom_build(p.mesh, phid, k, m, f, r, prec=MIXED)
    st = torch.zeros(3, dtype=torch.int32, device="cuda")
    y0, _ = ctx().rom_solve(Kh, fh, status=st)
    Kbad = Kh.clone()
    Kbad[1] *= 0.1
    Kbad[2] = -torch.eye(k, dtype=torch.float64, device="cuda")
    y = y0.clone()
    _, J, rn = ctx().rom_estimate(p.mesh, phid, k, m, f, r, Kbad, y, max_refine=2)
    y_ref = y0.clone()
    _, J0, rn0 = ctx().rom_estimate(p.mesh, phid, k, m, f, r, None, y_ref, max_refine=0)
    y, J, rn, J0, rn0, y0 = host(y), host(J), host(rn), host(J0), host(rn0), host(y0)
    ev = O.rom_eval(p.mesh, rhos[0], phi, p.mask, p.f)
    assert abs(J[0] / ev["Jk"] - 1) <= 1e-8
    assert not np.array_equal(y[0], y0[0])
    for b in (1, 2):
        assert np.array_equal(y[b], y0[b])
        assert J[b] == J0[b] and rn[b] == rn0[b]


@pytest.mark.parametrize("k", [64, 80, 96, 112, 128, 144, 200])
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_rom_build_tile_pair_layouts(k, mode):
    """k = 64..200 puts 3 to 8 tile pairs on each wave, in one to three pair groups:
    every layout of the contraction against the oracle's K_hat (3D, batch of 2)."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    p = W.cantilever3d(7, 5, 3)
    phi = _basis(p, k, np.float32, seed=3)
    rhos = _rhos(p, 2, 17)
    Kh, _ = ctx().rom_build(p.mesh, dev(phi), k, dev(p.mask, torch.uint8), dev(p.f, torch.float64),
                            dev(rhos, torch.float64), prec=FP64 if mode == "fp64" else MIXED)
    Kh = host(Kh)
    tol = 1e-13 if mode == "fp64" else 2e-6
    for b in range(2):
        ref = O.rom_operator(p.mesh, rhos[b], phi, p.mask)
        assert np.array_equal(Kh[b], Kh[b].T)
        assert np.abs(Kh[b] - ref).max() <= tol * np.abs(ref).max()


def test_rom_build_mid_size_chunk_slices():
    """A 120x40 mesh: 75 contraction chunks and 38 projection chunks, so the partial sums
    run with 4 and 2 chunk slices (the small cases use 1, the benchmark meshes 32)."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    p, k = W.cantilever2d(120, 40), 24
    phi = _basis(p, k, np.float32, seed=9)
    rhos = _rhos(p, 2, 23)
    for prec, tol in ((FP64, 1e-13), (MIXED, 2e-6)):
        Kh, fh = ctx().rom_build(p.mesh, dev(phi), k, dev(p.mask, torch.uint8), dev(p.f, torch.float64),
                                 dev(rhos, torch.float64), prec=prec)
        Kh, fh = host(Kh), host(fh)
        for b in range(2):
            ref = O.rom_operator(p.mesh, rhos[b], phi, p.mask)
            assert np.abs(Kh[b] - ref).max() <= tol * np.abs(ref).max()
        ref_f = O.rom_load(phi, p.mask, p.f)
        assert np.abs(fh - ref_f).max() <= 1e-14 * np.abs(ref_f).max()


@pytest.mark.parametrize("p,k", CASES[:5], ids=lambda v: getattr(v, "name", str(v)))
def test_rom_gradient_matches_oracle(p, k):
    """dJ_k/drho at the ROM state against the oracle's: FP64 build + solve to 1e-9 of
    the largest entry; the mixed build with FP64 reduced refinement to 1e-6.  Field 1
    alone and inside the batch of two give bitwise the same sensitivities."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    phi = _basis(p, k, np.float32)
    rhos = _rhos(p, 2, 31)
    m, f, phid = dev(p.mask, torch.uint8), dev(p.f, torch.float64), dev(phi)
    r = dev(rhos, torch.float64)
    ref = [O.rom_gradient(p.mesh, rhos[b], phi, p.mask, p.f)[0] for b in range(2)]
    for prec, tol in ((FP64, 1e-9), (MIXED, 1e-6)):
        Kh, fh = ctx().rom_build(p.mesh, phid, k, m, f, r, prec=prec)
        y, _ = ctx().rom_solve(Kh, fh)
        if prec == MIXED:
            y, _, _ = ctx().rom_estimate(p.mesh, phid, k, m, f, r, Kh, y, max_refine=2)
        dJ = host(ctx().rom_gradient(p.mesh, phid, k, m, r, y))
        for b in range(2):
            assert np.abs(dJ[b] - ref[b]).max() <= tol * np.abs(ref[b]).max()
        one = host(ctx().rom_gradient(p.mesh, phid, k, m, r[1:2].contiguous(), y[1:2].contiguous()))
        assert np.array_equal(one[0], dJ[1])


@pytest.mark.parametrize("max_refine", [0, 2])
def test_estimate_fused_sensitivity_equals_separate_call(max_refine):
    """The sensitivity returned with the estimate is the one topo_rom_gradient gives at the
    returned coefficients (bitwise: the same kernels on the same u = Phi y), and in FP64
    it matches the oracle's ROM sensitivity."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    p = W.cantilever2d(37, 11)
    k = 9
    phi = dev(_basis(p, k, np.float32))
    rho = dev(_rhos(p, 2, seed=5), torch.float64)
    m, f = dev(p.mask, torch.uint8), dev(p.f, torch.float64)
    prec = FP64 if max_refine == 0 else MIXED
    Kh, fh = ctx().rom_build(p.mesh, phi, k, m, f, rho, prec=prec)
    y, _ = ctx().rom_solve(Kh, fh)
    dJ = torch.empty_like(rho)
    y, J, rn = ctx().rom_estimate(p.mesh, phi, k, m, f, rho, Kh, y, max_refine=max_refine, dJ=dJ)
    sep = ctx().rom_gradient(p.mesh, phi, k, m, rho, y)
    assert torch.equal(dJ, sep)
    if max_refine == 0:
        for b in range(2):
            go, _ = O.rom_gradient(p.mesh, host(rho)[b], _basis(p, k, np.float32), p.mask, p.f)
            assert np.abs(host(dJ)[b] - go).max() <= 1e-9 * np.abs(go).max()
