#!/usr/bin/env python3
"""Benchmark of the ROM-accelerated SIMP compliance hot path on one MI355X.

One step = one pass of the whole hot path over one batch of B density fields on one
mesh (default: the 192x96x96 H8 bridge, B = 16, k = 200, mixed precision):
  batched HDM state solve (Jacobi-PCG, float32 inner / float64 refinement, rtol 1e-8)
  -> compliances -> element sensitivities -> ROM build (K_hat of the B fields by the
  per-element MFMA contraction, f_hat) -> reduced float64 Cholesky solves -> residual
  error indicator with one reduced refinement step and the ROM sensitivity fused in.
Headline value: PCG DOF-iterations per second over the whole timed step
(sum over fields of N_u x inner PCG iterations / wall time, ROM work included).

The B fields are candidate designs of a trust-region subproblem: points on a seeded
smooth design path through a centre design (a seeded smoothed field); the basis is the
one the method builds at that centre: GramSchmidt([POD of the HDM snapshots at 8
earlier centres on the same path, u*(centre)]) on the device, completed to k columns
with smooth cosine fields and orthonormalised.

    python bench.py [--steps K] [--warmup W] [--workload bridge3d_192x96x96]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFS = 157.3
FP64_MFMA_PEAK_TFS = 78.6
SNAPSHOTS = 8  # earlier trust-region centres in the basis window


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bridge3d_192x96x96")
    ap.add_argument("--fields", type=int, default=None, help="density fields per step (default: the workload's)")
    ap.add_argument("--prec", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--rtol", type=float, default=None)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--max-refine", type=int, default=1)
    ap.add_argument("--rom-evals", type=int, default=5, help="batched ROM evaluations per precision")
    ap.add_argument("--timing-every", type=int, default=4,
                    help="sample one run of 8 consecutive launches in N of each hot kernel (with graphs: "
                         "the first 8 iterations of one chunk replay in N)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision, 2D batch, per-config, basis, filter and trust-region legs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-workers", type=int, default=4)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (5 times), the "
                         "reference kernel that scales the HBM byte counters")
    ap.add_argument("--profile-step", action="store_true",
                    help="only set up and run warmup + steps of the headline step (for profilers)")
    return ap.parse_args()


# ----------------------------------------------------------------------------------
# Algorithmic costs
# ----------------------------------------------------------------------------------

def pcg_bytes(n_dofs, n_nodes, n_elems, word, dim=2):
    """Algorithmic HBM bytes of one field's share of one launch of each PCG kernel
    (each array once).
    step  (2D float64, one kernel per iteration): read r, w, s (stencil), p, mask,
          alpha, 1/sum(alpha) per node; read/write x (float64); write r, w, s, p
    apply (two-kernel form): read z, p_old (stencil), alpha, mask; write p_new, q
    update (two-kernel form): read r; write r, z; read q, 1/sum(alpha) per node; and at
          the last update of each group of G (x takes G steps at a time: G = 2 in 2D,
          8 in 3D) read and write x (float64) and read the group's G directions: on
          average (16 + G w) / G bytes per DOF
    In 3D the update applies the mask, as one byte of mask bits per node (the apply reads
    none), and the float32 apply reads r and 1/sum(alpha) per node and forms z itself,
    so its update writes no z."""
    forms_z = dim == 3 and word == 4
    mask_apply = 1 if dim == 2 else 0
    group = 8 if dim == 3 else 2
    x_bytes = (16 + group * word) / group
    return {
        "pcg_step": n_dofs * (8 * word + 17) + n_nodes * word + n_elems * word,
        "pcg_apply": n_dofs * (4 * word + mask_apply) + n_elems * word + (n_nodes * word if forms_z else 0),
        "pcg_update": n_dofs * ((3 if forms_z else 4) * word + x_bytes) + n_nodes * (word + 1 - mask_apply),
    }


def pcg_kernel_name(kind, dim, word):
    """Symbol (as rocprofv3 prints it) of a PCG kernel.  The 3D apply is named with its
    index type: 32-bit for float32 on the meshes measured here (per-field arrays under
    4 GiB), 64-bit for float64."""
    t = "float" if word == 4 else "double"
    apply3 = "k_pcg_apply3<float, unsigned int>" if word == 4 else "k_pcg_apply3<double, unsigned long>"
    return {"pcg_step": f"k_cg1_step2<{t}>", "pcg_apply": apply3 if dim == 3 else f"k_pcg_apply2<{t}>",
            "pcg_update": f"k_pcg_update<{dim},{t}>"}[kind]


def rom_contract_flops(n_elems, k, ne):
    """Flops of the per-element K_hat contraction for one density field as the paper's
    cost analysis counts them (Sec. 3.4: K_e Phi_e, then Phi_e^T (K_e Phi_e))."""
    return n_elems * (2 * k * ne * ne + 2 * k * k * ne)


def rom_gemm_flops(n_dofs, k):
    """Algorithmic flops of K_hat = Phi^T W for one field on the float64 matrix cores: the
    k (k + 1) / 2 distinct entries of the symmetric product, a multiply-add per DOF each
    (W = K Phi is formed by the apply beforehand, on the vector units)."""
    return n_dofs * k * (k + 1)


# Device sources of the PCG kernels: measured HBM traffic recorded under profiles/ is
# used only while these files are unchanged since the counters were taken.
KERNEL_SOURCES = ("paper_2004_05756_amd/csrc/hdm.hip", "paper_2004_05756_amd/csrc/stencil.hpp",
                  "paper_2004_05756_amd/csrc/march3.hpp", "paper_2004_05756_amd/csrc/elemfac.hpp",
                  "paper_2004_05756_amd/csrc/internal.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes of one field's share of a launch of `kernel` (a batched launch moves
    this per active field) from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary under
    profiles/ (each counter scaled by what it reads for a plain copy of known size), or
    None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json: "):
                rec = json.loads(line[len("traffic-json: "):]).get(kernel)
                if rec and rec.get("source_hash") == kernel_source_hash():
                    return rec["bytes_per_field_launch"]
    return None


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))] if xs else None


def _ms(x):
    return None if x is None else 1e3 * x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ----------------------------------------------------------------------------------
# Inputs of the headline workload
# ----------------------------------------------------------------------------------

def candidate_ts(B):
    """Path parameters of the B candidate designs of the step: t = 1/32 .. B/32."""
    return [(b + 1) / 32.0 for b in range(B)]


def headline_inputs(W, cfg, B):
    """The centre design, B candidate designs of its trust-region subproblem (the step's
    fields) and SNAPSHOTS earlier centres (the basis window), all on one seeded smooth
    design path through the centre (W.path_fields: earlier centres at t = -1/8 .. -1,
    candidates at t = 1/32 .. B/32)."""
    m = cfg.problem.mesh
    centre = cfg.rho(0)
    fields = W.path_fields(m, centre, candidate_ts(B), cfg.rho_seed0 + 100)
    snaps = W.path_fields(m, centre, [-(j + 1) / 8.0 for j in range(SNAPSHOTS)], cfg.rho_seed0 + 100)
    return centre, fields, snaps


def build_basis(torch, W, binding, ctx, cfg, centre, snaps, k, rtol, dev):
    """The basis of the method at a trust-region centre on the device,
    GramSchmidt([POD(HDM snapshots at the earlier centres), u*(centre)]), completed to k
    columns with smooth cosine fields and orthonormalised as a whole (Cholesky QR twice,
    float64, on the host: the k = 200 reduced operator of an unorthogonalised mix of
    unit POD columns and O(1)-entry cosine fields is too ill-conditioned for its float32
    contraction); float32 [N_u][k]."""
    from paper_2004_05756_amd.binding import MIXED
    p = cfg.problem
    m = p.mesh
    mask = torch.as_tensor(p.mask).to(dev)
    f = torch.as_tensor(p.f).to(dev)
    rhos = torch.as_tensor(np.vstack([centre[None], snaps])).to(dev)
    u, infos = ctx.hdm_solve_batch(m, rhos, mask, f, rtol=rtol, prec=MIXED, check=False)
    win = binding.SnapshotWindow(ctx, m.n_dofs, SNAPSHOTS)
    for j in range(SNAPSHOTS):
        win.push(u[1 + j])
    nmax = min(SNAPSHOTS, k - 1)
    pod = torch.zeros((m.n_dofs, nmax + 1), dtype=torch.float64, device=dev)
    ncols, npod = win.basis(u[0], nmax, pod)
    torch.cuda.synchronize()
    cols = [pod[:, :ncols].cpu().numpy()]
    del u, win, pod
    rest = k - ncols
    if rest > 0:
        cols.append(W.cosine_basis(m, p.mask, rest, cfg.basis_seed, np.float64))
    phi = torch.as_tensor(W.orthonormalize_tall(np.hstack(cols), p.mask, np.float32)).to(dev)
    del cols
    torch.cuda.synchronize()
    return phi, {"snapshots": SNAPSHOTS, "pod_columns": npod, "snapshot_columns": ncols,
                 "cosine_columns": max(rest, 0), "orthonormalised": "Cholesky QR x2 (float64, host)",
                 "snapshot_iters": [i["iters"] for i in infos]}


# ----------------------------------------------------------------------------------
# Side legs
# ----------------------------------------------------------------------------------

def batch_scaling_leg(torch, W, binding, FP64, MIXED, counts=(1, 4, 16)):
    """The 600x200 cantilever solved for B = 1 / 4 / 16 fields per launch in both
    precisions: wall time, PCG iterations, DOF-iter/s and the HBM fraction of the PCG
    kernels (algorithmic bytes of the active fields over the sampled launch times)."""
    cfg = W.config("cantilever2d_600x200")
    p, m = cfg.problem, cfg.problem.mesh
    dev = torch.device("cuda", 0)
    mask = torch.as_tensor(p.mask).to(dev)
    f = torch.as_tensor(p.f).to(dev)
    allr = torch.as_tensor(np.stack([cfg.rho(i) for i in range(max(counts))])).to(dev)
    ctx = binding.Context(0)
    out = {"workload": cfg.name, "n_dofs": m.n_dofs, "rtol": cfg.rtol}
    for name, pr in (("mixed", MIXED), ("fp64", FP64)):
        w = 4 if pr == MIXED else 8
        kinds = ["pcg_apply", "pcg_update"] if pr == MIXED else ["pcg_step"]
        pb = pcg_bytes(m.n_dofs, m.n_nodes, m.n_elems, w, m.dim)
        res = {}
        for B in counts:
            R = allr[:B].contiguous()
            ctx.hdm_solve_batch(m, R, mask, f, rtol=cfg.rtol, prec=pr, check=False)  # warm
            for kd in kinds:
                ctx.kernel_time(kd, reset=True)
            ctx.set_timing(4)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = ctx.hdm_solve_batch(m, R, mask, f, rtol=cfg.rtol, prec=pr, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ctx.set_timing(0)
            its = [i["iters"] for i in infos]
            rec = {"ms": 1e3 * dt, "iters": its, "dof_iter_per_s": m.n_dofs * sum(its) / dt,
                   "solves_per_s": B / dt}
            for kd in kinds:
                n, ms, nl = ctx.kernel_time(kd, reset=True, launches=True)
                if n and nl:
                    avg = 1e-3 * ms / n
                    nbytes = pb[kd] * sum(its) / nl  # the active fields of an average launch
                    rec[kd] = {"avg_us": 1e6 * avg, "launches": nl, "GB_s": nbytes / avg / 1e9,
                               "hbm_frac": nbytes / avg / 1e9 / HBM_PEAK_GBS}
            res[f"B{B}"] = rec
        out[name] = res
    ctx.close()
    return out


def config_leg(torch, W, binding, FP64, MIXED, name, rom_evals=20):
    """One field of a named workload: HDM time to solution in both precisions, and ROM
    evaluations (build + reduced solve + estimate) per second with p50 / p99 in both
    precisions (mixed with one reduced refinement step)."""
    cfg = W.config(name)
    p, m = cfg.problem, cfg.problem.mesh
    dev = torch.device("cuda", 0)
    rho = torch.as_tensor(cfg.rho(0)).to(dev)
    mask = torch.as_tensor(p.mask).to(dev)
    f = torch.as_tensor(p.f).to(dev)
    phi = torch.as_tensor(W.cosine_basis(m, p.mask, cfg.k, cfg.basis_seed, np.float32)).to(dev)
    ctx = binding.Context(0)
    out = {"n_dofs": m.n_dofs, "k": cfg.k, "rtol": cfg.rtol}
    for pname, pr in (("mixed", MIXED), ("fp64", FP64)):
        ctx.hdm_solve(m, rho, mask, f, rtol=cfg.rtol, prec=pr, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = ctx.hdm_solve(m, rho, mask, f, rtol=cfg.rtol, prec=pr, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"hdm_ms": 1e3 * dt, "iters": inf["iters"], "dof_iter_per_s": m.n_dofs * inf["iters"] / dt,
               "rel_resid": inf["rel_resid"], "fp64_fallback": inf["fp64_fallback"]}
        R1 = rho.view(1, -1)
        lat = []
        for i in range(rom_evals + 2):
            t0 = time.perf_counter()
            Kh, fh = ctx.rom_build(m, phi, cfg.k, mask, f, R1, prec=pr)
            y, _ = ctx.rom_solve(Kh, fh)
            ctx.rom_estimate(m, phi, cfg.k, mask, f, R1, Kh, y, max_refine=1 if pr == MIXED else 0)
            torch.cuda.synchronize()
            if i >= 2:
                lat.append(time.perf_counter() - t0)
        rec.update({"rom_evals_per_s": len(lat) / sum(lat), "rom_p50_ms": _ms(_pct(lat, 0.5)),
                    "rom_p99_ms": _ms(_pct(lat, 0.99))})
        out[pname] = rec
    out["faster_hdm"] = min(("mixed", "fp64"), key=lambda q: out[q]["hdm_ms"])
    ctx.close()
    return out


def serving_leg(args, torch, W, binding, FP64, MIXED):
    """The serving workload: the seeded stream of ROM / HDM requests over four meshes,
    (a) plain FP64 one request at a time through the context, (b) the continuous-
    batching server in FP64 with every request submitted at once, (c) the same server
    in mixed precision, and (d) the mixed server with Poisson arrivals at 0.7x the FP64
    sequential rate (latency under load).  Densities and bases are resident on the
    device for (a); the server receives host densities (copied at submit)."""
    dev = torch.device("cuda", 0)
    cfgs = [W.config(nm) for nm in W.SERVING_MESHES]
    kmax = 128
    reqs = W.serving_stream(args.serving_requests, kmax=kmax)
    pool = [[c.rho(i) for i in range(8)] for c in cfgs]
    phis = [W.cosine_basis(c.problem.mesh, c.problem.mask, kmax, c.basis_seed, np.float32) for c in cfgs]
    D = []
    for c, phi, rp in zip(cfgs, phis, pool):
        p = c.problem
        D.append({"mask": torch.as_tensor(p.mask).to(dev), "f": torch.as_tensor(p.f).to(dev),
                  "phi": torch.as_tensor(phi).to(dev),
                  "rho": [torch.as_tensor(r).to(dev).view(1, -1) for r in rp]})

    # (a) plain FP64, one at a time
    ctx = binding.Context(0)

    def run_fp64(q):
        c, d = cfgs[q.mesh], D[q.mesh]
        m = c.problem.mesh
        rho = d["rho"][q.rho_id]
        if q.kind == "hdm":
            _, inf = ctx.hdm_solve(m, rho.view(-1), d["mask"], d["f"], rtol=c.rtol, prec=FP64)
            return inf["compliance_corr"]
        Kh, fh = ctx.rom_build(m, d["phi"], q.k, d["mask"], d["f"], rho, prec=FP64)
        y, _ = ctx.rom_solve(Kh, fh)
        _, J, _ = ctx.rom_estimate(m, d["phi"], q.k, d["mask"], d["f"], rho, Kh, y, max_refine=0)
        return float(J[0])

    seen = set()
    for q in reqs:  # warm-up: one request of each (mesh, kind)
        if (q.mesh, q.kind) not in seen:
            seen.add((q.mesh, q.kind))
            run_fp64(q)
    torch.cuda.synchronize()
    lat_a, J_a = [], []
    for q in reqs:
        t = time.perf_counter()
        J_a.append(run_fp64(q))
        torch.cuda.synchronize()
        lat_a.append(time.perf_counter() - t)
    fp64_rate = len(reqs) / sum(lat_a)
    ctx.close()

    def make_server():
        srv = binding.Server(0, budget_bytes=32 << 30, max_batch=16, workers=args.serving_workers)
        ids = []
        for c, phi in zip(cfgs, phis):
            p = c.problem
            mid = srv.register_mesh(p.mesh, p.mask, p.f)
            ids.append((mid, srv.register_basis(mid, phi)))
        return srv, ids

    def submit(srv, ids, q, prec):
        c = cfgs[q.mesh]
        mid, bid = ids[q.mesh]
        rho = pool[q.mesh][q.rho_id]
        if q.kind == "hdm":
            return srv.submit_hdm(mid, rho, rtol=c.rtol, prec=prec)
        return srv.submit_rom(mid, bid, q.k, rho, prec=prec, max_refine=1 if prec == MIXED else 0)

    def saturated(prec):
        srv, ids = make_server()
        warm, seen2 = [], set()
        for q in reqs:
            if (q.mesh, q.kind) not in seen2:
                seen2.add((q.mesh, q.kind))
                warm.append(submit(srv, ids, q, prec))
        for t in warm:
            srv.wait(t)
        t0 = time.perf_counter()
        res = [srv.wait(t) for t in [submit(srv, ids, q, prec) for q in reqs]]
        dt = time.perf_counter() - t0
        return srv, ids, res, dt

    def job_busy(res):
        """Device-side service time of the jobs (a fused ROM batch is one job: its
        requests share worker and start time), summed per kind."""
        jobs = {}
        for r, q in zip(res, reqs):
            key = (r["worker"], r["t_start"], q.kind)
            jobs[key] = max(jobs.get(key, 0.0), r["t_done"] - r["t_start"])
        return {kd: sum(v for (_, _, k2), v in jobs.items() if k2 == kd) for kd in ("hdm", "rom")}, len(jobs)

    def rel_diff(res, kind):
        d = [abs(r["J"] / ja - 1.0) for r, ja, q in zip(res, J_a, reqs) if q.kind == kind and ja != 0]
        return max(d) if d else None

    def lat(res, kind=None):
        return [r["t_done"] - r["t_submit"] for r, q in zip(res, reqs) if kind in (None, q.kind)]

    out = {"requests": len(reqs),
           "mix": {"meshes": list(W.SERVING_MESHES), "rom_frac": 0.8, "k": [8, kmax],
                   "hdm": sum(q.kind == "hdm" for q in reqs)},
           "fp64_sequential": {"evals_per_s": fp64_rate, "p50_ms": _ms(_pct(lat_a, 0.5)),
                               "p99_ms": _ms(_pct(lat_a, 0.99))}}
    failed = 0
    for name, prec in (("served_fp64_saturated", FP64), ("served_mixed_saturated", MIXED)):
        srv, ids, res, dt = saturated(prec)
        busy, njobs = job_busy(res)
        st = srv.stats()
        failed += sum(1 for r in res if r["status"] != 0)
        out[name] = {"evals_per_s": len(reqs) / dt, "makespan_s": dt,
                     "p50_ms": _ms(_pct(lat(res), 0.5)), "p99_ms": _ms(_pct(lat(res), 0.99)),
                     "speedup_vs_fp64_sequential": (len(reqs) / dt) / fp64_rate,
                     "jobs": njobs, "mean_rom_batch": st["mean_rom_batch"],
                     "mean_hdm_batch": st.get("mean_hdm_batch"),
                     "job_service_s": busy, "overlap": (busy["hdm"] + busy["rom"]) / dt,
                     "max_rel_diff_vs_fp64_sequential": {"hdm_J": rel_diff(res, "hdm"), "rom_Jk": rel_diff(res, "rom")},
                     "max_held_gb": st["max_held_bytes"] / 2**30}
        if prec == MIXED:
            arr = W.poisson_arrivals(len(reqs), 0.7 * fp64_rate)
            tickets = []
            t0 = time.perf_counter()
            for q, ta in zip(reqs, arr):
                dtw = t0 + ta - time.perf_counter()
                if dtw > 0:
                    time.sleep(dtw)
                tickets.append(submit(srv, ids, q, MIXED))
            res_c = [srv.wait(t) for t in tickets]
            failed += sum(1 for r in res_c if r["status"] != 0)
            out["served_mixed_poisson"] = {
                "arrival_rate_per_s": 0.7 * fp64_rate,
                "p50_ms": _ms(_pct(lat(res_c), 0.5)), "p99_ms": _ms(_pct(lat(res_c), 0.99)),
                "p50_ms_rom": _ms(_pct(lat(res_c, "rom"), 0.5)), "p99_ms_rom": _ms(_pct(lat(res_c, "rom"), 0.99)),
                "p50_ms_hdm": _ms(_pct(lat(res_c, "hdm"), 0.5)), "p99_ms_hdm": _ms(_pct(lat(res_c, "hdm"), 0.99))}
        srv.close()
    out["failed"] = failed
    out["workers"] = args.serving_workers
    return out


def basis_leg(torch, binding, ctx, n, L=20, nmax=19):
    """Reduced-basis update at a trust-region centre on a full window of L snapshots of
    length n: one push (rank-two update: the new snapshot replaces the oldest) and one
    GramSchmidt([POD(window), u]) into a float32 basis.  Snapshots are synthetic
    (a common random field plus perturbations of geometrically decreasing size).
    Algorithmic bytes: push streams the L - 1 other snapshots, u, and writes u; the
    basis call streams the window and u three times (dots, remainder norm, basis rows)
    and writes n x (nmax + 1) floats."""
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    base = torch.randn(n, device=dev, dtype=torch.float64, generator=gen)
    win = binding.SnapshotWindow(ctx, n, L)
    snaps = [base + 0.6 ** i * torch.randn(n, device=dev, dtype=torch.float64, generator=gen)
             for i in range(L + 1)]
    for sn in snaps[:L]:
        win.push(sn)
    u = snaps[L]
    phi = torch.empty((n, nmax + 1), device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    ev[0].record()
    for i in range(reps):
        win.push(snaps[i % (L + 1)])
    ev[1].record()
    torch.cuda.synchronize()
    push_ms = ev[0].elapsed_time(ev[1]) / reps
    lat = []
    for _ in range(5):
        t0 = time.perf_counter()
        ncols, npod = win.basis(u, nmax, phi)
        lat.append(time.perf_counter() - t0)
    lat.sort()
    basis_ms = 1e3 * lat[len(lat) // 2]
    push_bytes = (L + 1) * n * 8
    basis_bytes = 3 * (L + 1) * n * 8 + ncols * n * 4
    out = {"n": n, "window": L, "nmax": nmax, "columns": ncols,
           "push_ms": push_ms, "push_GB_s": push_bytes / (push_ms * 1e-3) / 1e9,
           "basis_ms": basis_ms, "basis_GB_s": basis_bytes / (basis_ms * 1e-3) / 1e9}
    out["push_hbm_frac"] = out["push_GB_s"] / HBM_PEAK_GBS
    out["basis_hbm_frac"] = out["basis_GB_s"] / HBM_PEAK_GBS
    del win, snaps, phi
    return out


def helmholtz_length(R):
    """Helmholtz length r of a filter radius R: the conic filter's second moment
    matched, r = R / (2 sqrt(3)) (the relation of the filter reference the paper cites
    for Sec. 2.2; its text prints the inverse factor, which gives a filter about 12
    times wider)."""
    return R / (2.0 * np.sqrt(3.0))


def filter_leg(torch, ctx, mesh, R=3.0, rtol=1e-10):
    """Helmholtz filter forward (psi -> rho) and adjoint (dJ/drho -> dJ/dpsi) on one field
    of the mesh with filter radius R (in element sizes): wall time per call (each
    synchronises) and PCG iterations."""
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(13)
    r = helmholtz_length(R)
    psi = torch.rand((1, mesh.n_elems), device=dev, dtype=torch.float64, generator=gen)
    v = -torch.rand((1, mesh.n_elems), device=dev, dtype=torch.float64, generator=gen)
    rho = torch.empty_like(psi)
    g = torch.empty_like(psi)
    out = {"R": R, "r": r, "rtol": rtol, "n_nodes": mesh.n_nodes}
    for name, fn, x, y in (("forward", ctx.filter_forward, psi, rho), ("adjoint", ctx.filter_adjoint, v, g)):
        fn(mesh, r, x, y, rtol=rtol)
        lat = []
        for _ in range(5):
            t0 = time.perf_counter()
            _, its = fn(mesh, r, x, y, rtol=rtol)
            lat.append(time.perf_counter() - t0)
        lat.sort()
        out[f"{name}_ms"] = 1e3 * lat[len(lat) // 2]
        out[f"{name}_iters"] = its
    return out


def tr_leg(torch, ctx, problem, R=3.0, vf=0.5, iters=3):
    """Three outer iterations of the ROM trust-region method (residual trust region,
    window 5, n_max 4) from the uniform design on the mesh: wall time, HDM solves, model
    evaluations and the compliance at each centre."""
    from paper_2004_05756_amd.trdriver import TrustRegion
    r = helmholtz_length(R)
    drv = TrustRegion(ctx, problem.mesh, problem.mask, problem.f, r, vf, kind="res", window=5, nmax=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, hist = drv.run(iters=iters, tau=0.1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"R": R, "r": r, "vf": vf, "outer_iters": iters, "seconds": dt, "hdm_solves": drv.hdm_solves,
            "model_evals": drv.model_evals, "J_centres": [h["J"] for h in hist],
            "accepted": [bool(h["accepted"]) for h in hist], "ratios": [float(h["ratio"]) for h in hist]}


# ----------------------------------------------------------------------------------
# CPU baseline and accuracy (the only part of the benchmark that runs the oracle)
# ----------------------------------------------------------------------------------

def _oracle_cg_worker(args):
    """One field of the CPU sample, in a fresh process: the oracle's FP64 Jacobi-CG
    solve (assembly included) of the bridge problem at the sample's size."""
    nel, seed0, b, rtol = args
    sys.path.insert(0, ROOT)
    from threadpoolctl import threadpool_limits
    import oracle as O
    import workloads as W
    with threadpool_limits(1):
        p = W.bridge3d(*nel)
        centre = W.rho_smoothed(p.mesh, seed0)
        rho = W.path_fields(p.mesh, centre, [(b + 1) / 32.0], seed0 + 100)[0]
        info = {}
        t0 = time.perf_counter()
        _, res = O.solve_cg(p.mesh, rho, p.f, p.mask, rtol=rtol, info=info)
        dt = time.perf_counter() - t0
    return {"seconds": dt, "iters": info["iters"], "n_dofs": p.mesh.n_dofs, "rel_resid": res}


def cpu_baseline_leg(cfg, rtol, fields_np, gpu, phi_cols, cores=None):
    """(cpu_baseline, accuracy).

    cpu_baseline: the oracle as it stands on the host cores: its FP64 Jacobi-CG solves
    (sparse assembly + scipy CG on the assembled matrix, restarted on the true
    residual) of the workload's problem at a quarter of its linear size (48x24x24 for
    the bridge, 91,875 DOF: the oracle's CG takes 0.1 s per iteration at 698,691 DOF
    already), one candidate field per
    process on every available core, to the workload's tolerance; value = sum of
    N_u x CG iterations / wall time of the parallel run.

    accuracy: each timed result of the GPU step (field 0) against the oracle at the
    GPU's own state (the oracle cannot solve 5.4M DOF within the sample): the true
    residual of u recomputed element by element in FP64, the corrected compliance from
    that residual, the element sensitivities at u, and for the ROM the residual norm and
    compliance at the GPU's coefficients and three columns of K_hat from the oracle's
    own products K Phi_j."""
    import multiprocessing as mp
    import oracle as O
    ncores = cores or max(1, min(16, len(os.sched_getaffinity(0))))
    sample_nel = tuple(max(1, n // 4) for n in cfg.problem.mesh.nel)
    ctxm = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctxm.Pool(ncores) as pool:
        recs = pool.map(_oracle_cg_worker, [(sample_nel, cfg.rho_seed0, b, rtol) for b in range(ncores)])
    wall = time.perf_counter() - t0
    dof_iters = sum(r["n_dofs"] * r["iters"] for r in recs)
    base = {"value": dof_iters / wall, "unit": "DOF-iter/s", "cores": ncores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"oracle FP64 Jacobi-CG (sparse assembly + scipy CG, restarted on the true residual) of "
                       f"the bridge problem at {sample_nel[0]}x{sample_nel[1]}x{sample_nel[2]} "
                       f"({recs[0]['n_dofs']} DOF), {ncores} candidate designs in parallel "
                       f"processes (one per core, one thread each) to rel. residual {rtol:g}; value = sum of "
                       f"N_u x CG iterations / wall time of the parallel run, assembly included"),
            "seconds": wall, "iters": [r["iters"] for r in recs],
            "oracle_solve_s": [r["seconds"] for r in recs]}

    p, m = cfg.problem, cfg.problem.mesh
    rho0 = fields_np[0]
    u = gpu["u0"]
    acc = {"field": 0, "definition": "relative errors of the GPU step's results for field 0 against the "
                                     "oracle evaluated at the GPU's state (FP64)"}
    ta = time.perf_counter()
    Ku = O.apply_ebe(m, rho0, p.mask, u)
    free = p.mask == 0
    r = np.where(free, p.f - Ku, 0.0)
    nf = np.linalg.norm(np.where(free, p.f, 0.0))
    acc["hdm_rel_resid_oracle"] = float(np.linalg.norm(r) / nf)
    acc["hdm_rel_resid_gpu"] = gpu["rel_resid0"]
    c_or = float(np.dot(np.where(free, p.f, 0.0), u) + np.dot(u, r))
    acc["compliance_rel_err"] = abs(gpu["compliance0"] / c_or - 1.0)
    g_or = O.sensitivity(m, rho0, u)
    acc["gradient_rel_err"] = float(np.abs(gpu["dc0"] - g_or).max() / np.abs(g_or).max())
    # ROM at the GPU's coefficients: u_k = Phi y, r = f - K u_k, J_k = f^T u_k (the float32
    # basis promoted exactly, in row chunks)
    P = phi_cols
    ch = 1 << 20

    def p_y(y):
        return np.concatenate([P[i:i + ch].astype(np.float64) @ y for i in range(0, P.shape[0], ch)])

    def pt_v(v):
        return sum(P[i:i + ch].astype(np.float64).T @ v[i:i + ch] for i in range(0, P.shape[0], ch))

    uk = np.where(free, p_y(gpu["y0"]), 0.0)
    rk = np.where(free, p.f - O.apply_ebe(m, rho0, p.mask, uk), 0.0)
    acc["rom_resnorm_rel_err"] = abs(gpu["resnorm0"] / np.linalg.norm(rk) - 1.0)
    acc["rom_resnorm_over_f"] = float(np.linalg.norm(rk) / nf)
    Jk_or = float(np.dot(np.where(free, p.f, 0.0), uk))
    acc["rom_Jk_rel_err"] = abs(gpu["Jk0"] / Jk_or - 1.0)
    acc["rom_Jk_over_compliance"] = Jk_or / c_or
    cols = [0, P.shape[1] // 2, P.shape[1] - 1]
    errs = []
    for j in cols:
        kcol = pt_v(O.apply_ebe(m, rho0, p.mask, np.where(free, P[:, j].astype(np.float64), 0.0)))
        errs.append(float(np.abs(gpu["Khat0"][:, j] - kcol).max() / np.abs(kcol).max()))
    acc["rom_Khat_columns"] = cols
    acc["rom_Khat_rel_err"] = max(errs)
    acc["seconds"] = time.perf_counter() - ta
    return base, acc


def small_config_accuracy(torch, W, binding, FP64, MIXED):
    """Configs 1 and 2 (the oracle factorises them): compliance, sensitivity, J_k and
    ||r|| of the GPU path in both precisions against the oracle's direct solve and its
    assembled Phi^T (K Phi).  Runs the oracle, so it belongs to the CPU-baseline leg."""
    import oracle as O
    dev = torch.device("cuda", 0)
    ctx = binding.Context(0)
    out = {}
    for name in ("mbb2d_60x20", "cantilever2d_600x200"):
        cfg = W.config(name)
        p, m = cfg.problem, cfg.problem.mesh
        rho_np = cfg.rho(0)
        phi_np = W.cosine_basis(m, p.mask, cfg.k, cfg.basis_seed, np.float32)
        uo = O.solve_direct(m, rho_np, p.f, p.mask)
        co = O.compliance(p.f, uo)
        go = O.sensitivity(m, rho_np, uo)
        ev = O.rom_eval(m, rho_np, phi_np, p.mask, p.f)
        rho = torch.as_tensor(rho_np).to(dev)
        mask = torch.as_tensor(p.mask).to(dev)
        f = torch.as_tensor(p.f).to(dev)
        phi = torch.as_tensor(phi_np).to(dev)
        rec = {}
        for pname, pr in (("fp64", FP64), ("mixed", MIXED)):
            u, inf = ctx.hdm_solve(m, rho, mask, f, rtol=cfg.rtol, prec=pr)
            g = ctx.hdm_gradient(m, rho, u).cpu().numpy()
            Kh, fh = ctx.rom_build(m, phi, cfg.k, mask, f, rho.view(1, -1), prec=pr)
            y, _ = ctx.rom_solve(Kh, fh)
            _, Je, rn = ctx.rom_estimate(m, phi, cfg.k, mask, f, rho.view(1, -1), Kh, y,
                                         max_refine=1 if pr == MIXED else 0)
            rec[pname] = {"compliance_rel_err": abs(inf["compliance_corr"] / co - 1),
                          "gradient_rel_err": float(np.abs(g - go).max() / np.abs(go).max()),
                          "Jk_rel_err": abs(float(Je[0]) / ev["Jk"] - 1),
                          "resnorm_rel_err": abs(float(rn[0]) / ev["resnorm"] - 1)}
        out[name] = rec
    ctx.close()
    return out


# ----------------------------------------------------------------------------------
# Main
# ----------------------------------------------------------------------------------

def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only: multi-GPU sharding is designed "
                                   "but not implemented, so no figure at several GPUs is produced",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2004_05756_amd import binding
    from paper_2004_05756_amd.binding import FP64, MIXED

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "launches": 5}))
        return

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    cfg = W.config(args.workload)
    p = cfg.problem
    m = p.mesh
    B = args.fields or cfg.batch
    k = args.k or cfg.k
    rtol = args.rtol or cfg.rtol
    prec = MIXED if args.prec == "mixed" else FP64
    word = 4 if prec == MIXED else 8
    dev = torch.device("cuda", 0)
    one_red = m.dim == 2 and prec == FP64

    progress(f"inputs: {cfg.name}, {B} fields, k = {k}")
    centre, fields_np, snaps_np = headline_inputs(W, cfg, B)
    mask = torch.as_tensor(p.mask).to(dev)
    f = torch.as_tensor(p.f).to(dev)
    R = torch.as_tensor(fields_np).to(dev)
    ctx = binding.Context(0)
    progress("basis from the snapshot window")
    phi, basis_info = build_basis(torch, W, binding, ctx, cfg, centre, snaps_np, k, rtol, dev)

    U = torch.empty((B, m.n_dofs), dtype=torch.float64, device=dev)
    DC = torch.empty((B, m.n_elems), dtype=torch.float64, device=dev)
    KH = torch.empty((B, k, k), dtype=torch.float64, device=dev)
    FH = torch.empty(k, dtype=torch.float64, device=dev)
    Y = torch.empty((B, k), dtype=torch.float64, device=dev)
    J = torch.empty(B, dtype=torch.float64, device=dev)
    JE = torch.empty(B, dtype=torch.float64, device=dev)
    RN = torch.empty(B, dtype=torch.float64, device=dev)
    DJ = torch.empty((B, m.n_elems), dtype=torch.float64, device=dev)
    ST = torch.empty(B, dtype=torch.int32, device=dev)
    phases = {"hdm": 0.0, "rom": 0.0}

    def step(pr=prec, refine=args.max_refine, record=None):
        t0 = time.perf_counter()
        _, infos = ctx.hdm_solve_batch(m, R, mask, f, u=U, rtol=rtol, prec=pr, check=False)
        ctx.hdm_gradient_batch(m, R, U, dc=DC)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.rom_build(m, phi, k, mask, f, R, prec=pr, Khat=KH, fhat=FH)
        ctx.rom_solve(KH, FH, status=ST, yhat=Y, Jk=J)
        ctx.rom_estimate(m, phi, k, mask, f, R, KH, Y, max_refine=refine if pr == MIXED else 0, Jk=JE,
                         resnorm=RN, dJ=DJ)
        if record is not None:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            record["hdm"] += t1 - t0
            record["rom"] += t2 - t1
        return infos

    if args.profile_step:
        for i in range(args.warmup + args.steps):
            infos = step()
            torch.cuda.synchronize()
            progress(f"profile step {i}: iters {[x['iters'] for x in infos]}")
        return

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        progress(f"warmup {i} done")
    names = ["pcg_step", "pcg_apply", "pcg_update", "residual", "rom_contract", "rom_reduce", "phit_v",
             "phi_y", "chol", "chol_solve", "gradient", "rom_apply"]
    for nm in names:
        ctx.kernel_time(nm, reset=True)
    ctx.set_timing(args.timing_every)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    field_iters = 0
    infos_all = []
    for i in range(args.steps):
        infos = step(record=phases)
        field_iters += sum(x["iters"] for x in infos)
        infos_all.append(infos)
        progress(f"step {i}: iters {[x['iters'] for x in infos]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(0)
    elapsed = t1 - t0
    value = m.n_dofs * field_iters / elapsed

    # live per-kernel durations from the sampled HIP events of the timed region
    ktimes = {}
    for nm in names:
        n, ms, nl = ctx.kernel_time(nm, launches=True)
        if n:
            ktimes[nm] = {"samples": n, "avg_us": 1e3 * ms / n, "launches": nl,
                          "est_total_ms": ms / n * nl}
    pcg_kinds = ["pcg_step"] if one_red else ["pcg_apply", "pcg_update"]
    share = {nm: ktimes[nm]["est_total_ms"] for nm in pcg_kinds + ["rom_contract"] if nm in ktimes}
    dominant = max(share, key=share.get) if share else None
    pb = pcg_bytes(m.n_dofs, m.n_nodes, m.n_elems, word, m.dim)

    def pcg_roofline(kd):
        kt = ktimes[kd]
        avg_s = kt["avg_us"] * 1e-6
        per_launch = pb[kd] * field_iters / kt["launches"]  # bytes of the active fields per launch
        gbs = per_launch / avg_s / 1e9
        kname = pcg_kernel_name(kd, m.dim, word)
        tf = measured_traffic(cfg.name, kname)
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS,
                "traffic": None if tf is None else tf * field_iters / kt["launches"],
                "kernel": kname, "bytes_per_launch": per_launch, "bytes_per_field_launch": pb[kd],
                "mean_active_fields": field_iters / kt["launches"], "avg_us": kt["avg_us"]}

    def contract_roofline():
        # one launch per field: K_hat = Phi^T W on the matrix cores
        kt = ktimes["rom_contract"]
        ne = m.dim * 2 ** m.dim
        fl = rom_gemm_flops(m.n_dofs, k)
        avg_s = kt["avg_us"] * 1e-6
        peak = FP64_MFMA_PEAK_TFS  # the product accumulates in float64 in both precisions
        tfs = fl / avg_s / 1e12
        out = {"bound": "mfma", "achieved": tfs, "peak": peak, "unit": "TFLOP/s", "frac": tfs / peak,
               "traffic": None, "kernel": "k_rom_gemm", "flops_per_launch": fl, "fields_per_launch": 1,
               "avg_us": kt["avg_us"],
               "paper_flops_per_field": rom_contract_flops(m.n_elems, k, ne)}
        if "rom_apply" in ktimes:  # W = K Phi (and the transposed basis), per field
            out["apply_avg_us_per_field"] = ktimes["rom_apply"]["avg_us"]
        return out

    roofline = None
    if dominant in pb:
        roofline = pcg_roofline(dominant)
    elif dominant == "rom_contract":
        roofline = contract_roofline()
    rooflines = {kd: pcg_roofline(kd) for kd in pcg_kinds if kd in ktimes}
    if "rom_contract" in ktimes:
        rooflines["rom_contract"] = contract_roofline()

    last = infos_all[-1]
    out = {
        "metric": "PCG DOF-iter/s (%HBM peak); ROM evals/s + p99 latency, mixed vs plain FP64",
        "value_definition": "PCG DOF-iterations per second of the whole hot-path step (batched HDM solve of "
                            "the fields, sensitivities, ROM build, reduced solves, estimate with the ROM "
                            "sensitivity fused in, all inside the timed region): sum over fields of N_u x "
                            "inner PCG iterations / wall time; the %HBM peak is roofline.frac, the ROM "
                            "evals/s and p99 latencies in each precision are under rom",
        "value": value,
        "unit": "DOF-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "fields": B, "k": k, "n_dofs": m.n_dofs, "n_elems": m.n_elems,
                   "rtol": rtol, "precision": args.prec, "max_refine": args.max_refine,
                   "fields_recipe": "candidate designs on a seeded smooth design path through a smoothed centre (t = 1/32 .. 16/32, amplitude 0.1); basis window from the earlier centres on the same path (t = -1/8 .. -1)",
                   "basis": basis_info},
        "roofline": roofline,
        "rooflines": rooflines,
        "time_to_solution": {args.prec: {"hdm_s_per_step": phases["hdm"] / args.steps,
                                         "rom_s_per_step": phases["rom"] / args.steps,
                                         "hdm_solves_per_s": B * args.steps / phases["hdm"],
                                         "rom_evals_per_s": B * args.steps / phases["rom"]}},
        "pcg_iters_per_step": field_iters / args.steps,
        "iters_per_field": [x["iters"] for x in last],
        "refinements": [x["refinements"] for x in last],
        "fp64_fallback": [x["fp64_fallback"] for x in last],
        "rel_resid_max": max(x["rel_resid"] for x in last),
        "status": [x["status"] for x in last],
        "rom_Jk_over_compliance": float((JE / torch.tensor([x["compliance_corr"] for x in last],
                                                             dtype=torch.float64, device=dev)).mean()),
        "rom_resnorm_over_f": float(RN.max() / torch.linalg.vector_norm(f)),
        "kernels": ktimes,
    }
    torch.cuda.synchronize()
    gpu0 = {"u0": U[0].cpu().numpy(), "dc0": DC[0].cpu().numpy(), "y0": Y[0].cpu().numpy(),
            "Khat0": KH[0].cpu().numpy(), "Jk0": float(JE[0]), "resnorm0": float(RN[0]),
            "compliance0": last[0]["compliance_corr"], "rel_resid0": last[0]["rel_resid"]}

    # ROM evaluations per second and latency of the batch, mixed vs plain FP64
    rom = {}
    for pname, pr in (("mixed", MIXED), ("fp64", FP64)):
        lat = []
        for i in range(args.rom_evals + 1):
            ta = time.perf_counter()
            ctx.rom_build(m, phi, k, mask, f, R, prec=pr, Khat=KH, fhat=FH)
            ctx.rom_solve(KH, FH, status=ST, yhat=Y, Jk=J)
            ctx.rom_estimate(m, phi, k, mask, f, R, KH, Y, max_refine=args.max_refine if pr == MIXED else 0,
                             Jk=JE, resnorm=RN, dJ=DJ)
            torch.cuda.synchronize()
            if i > 0:
                lat.append(time.perf_counter() - ta)
        rom[pname] = {"evals_per_s": B * len(lat) / sum(lat), "batch": B,
                      "p50_ms": _ms(_pct(lat, 0.5)), "p99_ms": _ms(_pct(lat, 0.99)),
                      "latency": "per batched evaluation of all fields"}
    out["rom"] = rom
    progress("rom legs done")

    if not args.no_extra:
        # the same step in the other precision: time to solution of each half
        other = "fp64" if args.prec == "mixed" else "mixed"
        rec = {"hdm": 0.0, "rom": 0.0}
        infos = step(pr=FP64 if other == "fp64" else MIXED, record=rec)
        out["time_to_solution"][other] = {"hdm_s_per_step": rec["hdm"], "rom_s_per_step": rec["rom"],
                                          "hdm_solves_per_s": B / rec["hdm"], "rom_evals_per_s": B / rec["rom"],
                                          "iters_per_field": [x["iters"] for x in infos]}
        tts = out["time_to_solution"]
        out["faster_precision"] = {"hdm": min(tts, key=lambda q: tts[q]["hdm_s_per_step"]),
                                   "rom": min(tts, key=lambda q: tts[q]["rom_s_per_step"])}
        progress("precision leg done")
    del KH, DJ
    ctx.close()
    torch.cuda.empty_cache()

    if not args.no_extra:
        extra = {}
        extra["batch_2d"] = batch_scaling_leg(torch, W, binding, FP64, MIXED)
        progress("2D batch leg done")
        extra["configs"] = {nm: config_leg(torch, W, binding, FP64, MIXED, nm)
                            for nm in ("mbb2d_60x20", "cantilever2d_600x200", "cantilever3d_96x48x48")}
        progress("per-config legs done")
        c2 = W.config("cantilever2d_600x200")
        ctx2 = binding.Context(0)
        extra["basis"] = basis_leg(torch, binding, ctx2, c2.problem.mesh.n_dofs)
        extra["basis_bridge"] = basis_leg(torch, binding, ctx2, m.n_dofs)
        extra["filter"] = filter_leg(torch, ctx2, c2.problem.mesh)
        extra["filter_bridge"] = filter_leg(torch, ctx2, m)
        extra["trust_region"] = tr_leg(torch, ctx2, c2.problem)
        ctx2.close()
        progress("basis / filter / trust-region legs done")
        out["extra"] = extra

    if not args.no_serving:
        out["serving"] = serving_leg(args, torch, W, binding, FP64, MIXED)
        progress("serving leg done")

    if not args.no_cpu_baseline:
        phi_np = phi.cpu().numpy()
        base, acc = cpu_baseline_leg(cfg, rtol, fields_np, gpu0, phi_np)
        out["cpu_baseline"] = base
        out["accuracy"] = {cfg.name: acc}
        out["accuracy"].update(small_config_accuracy(torch, W, binding, FP64, MIXED))
        progress("cpu baseline and accuracy done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
