"""GPU tests of the continuous-batching server: each result is the same alone and in
the mix (and matches the oracle), admission never exceeds the HBM budget, jobs of
different workers overlap in time, latency percentiles are reported."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def _server(**kw):
    torch_cuda()
    from paper_2004_05756_amd import binding
    return binding.Server(**kw)


def _setup(srv):
    """Two meshes with bases; returns (mesh records, requests)."""
    from paper_2004_05756_amd import FP64, MIXED
    p2 = W.mbb2d(60, 20)
    p3 = W.cantilever3d(12, 6, 6)
    recs = []
    for p, kmax, seed in ((p2, 24, 1), (p3, 40, 2)):
        mid = srv.register_mesh(p.mesh, p.mask, p.f)
        phi = W.cosine_basis(p.mesh, p.mask, kmax, seed, np.float32)
        bid = srv.register_basis(mid, phi)
        recs.append((p, mid, bid, phi))
    rng = np.random.default_rng(4242)
    reqs = []
    for i in range(40):
        which = int(rng.integers(0, 2))
        p, mid, bid, phi = recs[which]
        rho = rng.uniform(0.05, 1.0, p.mesh.n_elems)
        if i % 5 == 4:
            reqs.append(("hdm", which, rho, None, MIXED if i % 10 == 4 else FP64))
        else:
            k = int(rng.integers(4, phi.shape[1] + 1))
            reqs.append(("rom", which, rho, k, MIXED if i % 2 else FP64))
    return recs, reqs


def _submit_all(srv, recs, reqs, max_refine=3):
    tickets = []
    for kind, which, rho, k, prec in reqs:
        p, mid, bid, _ = recs[which]
        if kind == "hdm":
            tickets.append(srv.submit_hdm(mid, rho, rtol=1e-10, prec=prec))
        else:
            tickets.append(srv.submit_rom(mid, bid, k, rho, prec=prec, max_refine=max_refine))
    return [srv.wait(t) for t in tickets]


def test_results_same_alone_and_in_the_mix():
    alone_srv = _server(max_batch=1, workers=1)
    recs, reqs = _setup(alone_srv)
    alone = _submit_all(alone_srv, recs, reqs)
    errs = [alone_srv.last_error()]
    alone_srv.close()
    mix_srv = _server(max_batch=8, workers=4)
    recs2, _ = _setup(mix_srv)
    mix = _submit_all(mix_srv, recs2, reqs)
    st = mix_srv.stats()
    errs.append(mix_srv.last_error())
    mix_srv.close()
    bad = [(i, req[0], req[4], a["status"], b["status"]) for i, (req, a, b) in enumerate(zip(reqs, alone, mix))
           if a["status"] != 0 or b["status"] != 0]
    assert not bad, (bad, errs)
    assert st["mean_rom_batch"] > 1.0  # fusion happened
    for (kind, which, rho, k, prec), a, b in zip(reqs, alone, mix):
        if kind == "hdm":
            assert a["J"] == b["J"] and a["iters"] == b["iters"]
        else:
            assert abs(a["J"] / b["J"] - 1) <= 1e-10
            assert abs(a["resnorm"] / b["resnorm"] - 1) <= 1e-8
    # a sample against the oracle
    for (kind, which, rho, k, prec), b in list(zip(reqs, mix))[:12]:
        p, _, _, phi = recs[which]
        if kind == "hdm":
            c = O.compliance(p.f, O.solve_direct(p.mesh, rho, p.f, p.mask))
            assert abs(b["J"] / c - 1) <= (1e-10 if prec == 0 else 1e-8)
        else:
            ev = O.rom_eval(p.mesh, rho, phi[:, :k], p.mask, p.f)
            assert abs(b["J"] / ev["Jk"] - 1) <= 1e-8
            assert abs(b["resnorm"] / ev["resnorm"] - 1) <= 1e-6


def test_admission_respects_budget_and_overlap():
    srv = _server(max_batch=4, workers=4, budget_bytes=64 << 20)
    recs, reqs = _setup(srv)
    res = _submit_all(srv, recs, reqs)
    st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert 0 < st["max_held_bytes"] <= st["budget_bytes"]
    assert st["completed"] == len(reqs)
    assert st["p50_latency_s"]["rom"] > 0 and st["p99_latency_s"]["rom"] >= st["p50_latency_s"]["rom"]
    # jobs on different workers overlapped in time
    iv = sorted((r["t_start"], r["t_done"], r["worker"]) for r in res)
    overlap = any(iv[i + 1][0] < iv[i][1] and iv[i + 1][2] != iv[i][2] for i in range(len(iv) - 1))
    assert overlap
    srv.close()


def test_tiny_budget_serialises_and_too_large_fails():
    from paper_2004_05756_amd import FP64, binding
    p = W.mbb2d(60, 20)
    rho = W.rho_jitter(p.mesh, 1000)
    ref = _server(workers=1)
    mid = ref.register_mesh(p.mesh, p.mask, p.f)
    r0 = ref.wait(ref.submit_hdm(mid, rho, prec=FP64))
    ref.close()
    # a budget that holds one small job at a time: results unchanged
    srv = _server(workers=4, budget_bytes=int(2.5 * (1 << 20)))
    mid = srv.register_mesh(p.mesh, p.mask, p.f)
    out = [srv.wait(t) for t in [srv.submit_hdm(mid, rho, prec=FP64) for _ in range(6)]]
    st = srv.stats()
    assert all(o["status"] == 0 and o["J"] == r0["J"] for o in out)
    assert st["max_held_bytes"] <= st["budget_bytes"]
    # a request that can never fit is refused with ENOMEM
    big = W.cantilever3d(40, 20, 20)
    bid = srv.register_mesh(big.mesh, big.mask, big.f)
    r = srv.wait(srv.submit_hdm(bid, np.full(big.mesh.n_elems, 0.5), prec=FP64))
    assert r["status"] == binding.TOPO_ENOMEM
    srv.close()


def test_invalid_requests():
    from paper_2004_05756_amd import TopoError
    srv = _server(workers=1)
    p = W.mbb2d(10, 5)
    mid = srv.register_mesh(p.mesh, p.mask, p.f)
    bid = srv.register_basis(mid, W.cosine_basis(p.mesh, p.mask, 6, 1, np.float32))
    rho = np.full(p.mesh.n_elems, 0.5)
    with pytest.raises(TopoError):
        srv.submit_rom(mid, bid, 7, rho)
    with pytest.raises(TopoError):
        srv.submit_rom(mid + 5, bid, 3, rho)
    with pytest.raises(TopoError):
        srv.submit_hdm(mid, rho, rtol=2.0)
    srv.close()


def test_hdm_requests_fused_bitwise_alone_and_device_densities():
    """HDM requests on one mesh are fused into batched solves (mean HDM batch > 1), each
    result bitwise the one the request gets alone; densities passed as device tensors
    (kept alive by the binding until the result is read) give the same results."""
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, MIXED
    p = W.cantilever3d(12, 6, 6)
    rhos = [W.rho_smoothed(p.mesh, 6100 + i) for i in range(10)]
    alone = _server(max_batch=1, workers=1)
    mid = alone.register_mesh(p.mesh, p.mask, p.f)
    ref = {pr: [alone.wait(alone.submit_hdm(mid, r, rtol=1e-10, prec=pr)) for r in rhos] for pr in (FP64, MIXED)}
    alone.close()
    srv = _server(max_batch=8, workers=2)
    mid = srv.register_mesh(p.mesh, p.mask, p.f)
    for pr in (FP64, MIXED):
        tickets = [srv.submit_hdm(mid, r, rtol=1e-10, prec=pr) for r in rhos]
        # device densities produced on the caller's stream just before the submit
        dev_t = [srv.submit_hdm(mid, torch.as_tensor(r).cuda() * 1.0, rtol=1e-10, prec=pr) for r in rhos[:4]]
        got = [srv.wait(t) for t in tickets]
        got_dev = [srv.wait(t) for t in dev_t]
        for a, b in zip(ref[pr], got):
            assert b["status"] == 0 and a["J"] == b["J"] and a["iters"] == b["iters"]
        for a, b in zip(ref[pr], got_dev):
            assert a["J"] == b["J"] and a["iters"] == b["iters"]
    st = srv.stats()
    assert st["mean_hdm_batch"] > 1.0
    srv.close()


def test_resident_bases_are_charged_to_the_budget():
    """Registered meshes and bases count against the server's HBM budget: a basis that
    would take the resident set past it is refused with TOPO_ENOMEM, and the held bytes
    (resident set + workspace) never exceed the budget."""
    from paper_2004_05756_amd import TopoError, binding
    p = W.cantilever3d(24, 12, 12)  # 14,625 DOF
    budget = 8 << 20
    srv = _server(workers=2, budget_bytes=budget)
    mid = srv.register_mesh(p.mesh, p.mask, p.f)
    small = W.cosine_basis(p.mesh, p.mask, 16, 3, np.float32)  # 0.9 MiB
    bid = srv.register_basis(mid, small)
    too_big = W.cosine_basis(p.mesh, p.mask, 160, 4, np.float32)  # 8.9 MiB
    with pytest.raises(TopoError) as ei:
        srv.register_basis(mid, too_big)
    assert ei.value.code == binding.TOPO_ENOMEM
    st = srv.stats()
    assert st["resident_bytes"] >= small.nbytes + p.mesh.n_dofs * 9
    r = srv.wait(srv.submit_rom(mid, bid, 16, np.full(p.mesh.n_elems, 0.5)))
    assert r["status"] == 0
    st = srv.stats()
    assert st["max_held_bytes"] <= budget
    srv.close()


def test_context_budget_refuses_larger_workspace():
    torch = torch_cuda()
    from paper_2004_05756_amd import FP64, TopoError, binding
    small = W.mbb2d(30, 10)
    big = W.cantilever3d(48, 24, 24)  # about 7 MB of float64 PCG workspace
    c = binding.Context(0, budget_bytes=2 << 20)
    d = torch.device("cuda", 0)
    u, inf = c.hdm_solve(small.mesh, torch.full((small.mesh.n_elems,), 0.5, dtype=torch.float64, device=d),
                         torch.as_tensor(small.mask).to(d), torch.as_tensor(small.f).to(d), prec=FP64)
    assert inf["status"] == 0
    with pytest.raises(TopoError) as ei:
        c.hdm_solve(big.mesh, torch.full((big.mesh.n_elems,), 0.5, dtype=torch.float64, device=d),
                    torch.as_tensor(big.mask).to(d), torch.as_tensor(big.f).to(d), prec=FP64)
    assert ei.value.code == binding.TOPO_ENOMEM
    assert c.workspace_bytes() <= 2 << 20
    c.close()
