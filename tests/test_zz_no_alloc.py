"""The allocation-free reduced solve (topo_rom_solve_noalloc) against topo_rom_solve:
same kernels, so every output must be bitwise equal, on two calls in a row (the second
smaller, reusing the fixed device array the first call left behind), at the largest
size the array holds, and with a size beyond it refused before any device work."""
import numpy as np
import pytest

from gpu_util import ctx as _ctx, torch_cuda

pytestmark = pytest.mark.gpu


def _spd(rng, B, k, bad=()):
    """B seeded SPD k x k matrices (float64), the ones listed in `bad` made indefinite."""
    K = np.empty((B, k, k))
    for b in range(B):
        A = rng.standard_normal((k, k))
        K[b] = A @ A.T / k + np.diag(rng.uniform(0.5, 2.0, k))
        if b in bad:
            K[b, k // 2, k // 2] = -1.0
    return K


def _both(c, torch, Kh, fh):
    dev = torch.device("cuda", 0)
    B, k, _ = Kh.shape
    Kt = torch.as_tensor(Kh).to(dev)
    ft = torch.as_tensor(fh).to(dev)
    ref_st = torch.full((B,), 7, dtype=torch.int32, device=dev)
    y_ref, J_ref = c.rom_solve(Kt, ft, status=ref_st)
    st = torch.full((B,), 7, dtype=torch.int32, device=dev)
    y = torch.full((B, k), np.nan, dtype=torch.float64, device=dev)
    J = torch.full((B,), np.nan, dtype=torch.float64, device=dev)
    c.rom_solve_noalloc(Kt, ft, st, y, J)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (y_ref, J_ref, ref_st, y, J, st)]


def test_noalloc_matches_rom_solve_on_consecutive_calls():
    torch = torch_cuda()
    c = _ctx()
    rng = np.random.default_rng(31)
    # first call larger, second smaller: the second reuses what the first left behind
    for (k, B, bad) in ((150, 9, (4,)), (37, 3, ()), (200, 26, (0, 25))):
        print(f"noalloc case k={k} B={B}", flush=True)
        Kh = _spd(rng, B, k, bad)
        fh = rng.standard_normal(k)
        y_ref, J_ref, st_ref, y, J, st = _both(c, torch, Kh, fh)
        assert np.array_equal(st, st_ref)
        ok = st_ref == 0
        assert ok.sum() == B - len(bad)
        assert np.array_equal(y[ok], y_ref[ok])
        assert np.array_equal(J[ok], J_ref[ok])
        # and the solve itself against numpy on the SPD fields
        for b in np.flatnonzero(ok):
            yo = np.linalg.solve(Kh[b], fh)
            assert np.abs(y[b] - yo).max() <= 1e-9 * np.abs(yo).max()


def test_noalloc_refuses_beyond_the_fixed_array():
    torch = torch_cuda()
    from paper_2004_05756_amd import binding
    c = _ctx()
    cap = binding.load().topo_rom_solve_noalloc_max_bytes()
    assert cap == 8 << 20
    k = 256
    B = cap // (8 * k * k) + 1  # one field too many
    dev = torch.device("cuda", 0)
    Kt = torch.zeros((B, k, k), dtype=torch.float64, device=dev)
    ft = torch.zeros(k, dtype=torch.float64, device=dev)
    st = torch.zeros(B, dtype=torch.int32, device=dev)
    y = torch.zeros((B, k), dtype=torch.float64, device=dev)
    J = torch.zeros(B, dtype=torch.float64, device=dev)
    with pytest.raises(binding.TopoError) as ei:
        c.rom_solve_noalloc(Kt, ft, st, y, J)
    assert ei.value.code == binding.TOPO_EINVAL
