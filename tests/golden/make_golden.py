"""Writes the stored expected values of the full-size 3D cantilever workload
(cantilever3d_96x48x48, 698,691 DOF, density field 0, k = 100 cosine basis) by calling
the oracle only:

  * the compliance of the FP64 Jacobi-CG solution certified on the assembled matrix
    (restarted on the true residual until it reaches 1e-13 or stops improving), its
    residual-corrected value c~ = f^T u + u^T r, the relative residual reached, and an
    estimate of lambda_min(K_ff) (LOBPCG with the Jacobi preconditioner) for the bracket
    c* - c~ = r^T K^-1 r <= ||r||^2 / lambda_min (the compliance error identity of the
    ROM error analysis, applied to the HDM iterate);
  * J_k and ||f - K Phi y|| of the Galerkin ROM with the workload's k = 100 float32
    cosine basis from the assembled Phi^T (K Phi).

    python tests/golden/make_golden.py      (about 10 minutes on one core)
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    t0 = time.time()
    cfg = W.config("cantilever3d_96x48x48")
    p, m = cfg.problem, cfg.problem.mesh
    rho = cfg.rho(0)
    info = {}
    u, res = O.solve_cg(m, rho, p.f, p.mask, rtol=1e-13, restarts=40, info=info)
    K = O.assemble(m, rho)
    free = O.free_dofs(p.mask)
    Kff = K[free][:, free].tocsr()
    r = p.f[free] - Kff @ u[free]
    c_raw = O.compliance(p.f, u)
    c_corr = c_raw + float(u[free] @ r)
    # smallest eigenvalue estimate of K_ff (Jacobi-preconditioned LOBPCG)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((Kff.shape[0], 4))
    M = sp.diags(1.0 / Kff.diagonal())
    lam, _ = spla.lobpcg(Kff, X, M=M, largest=False, tol=1e-6, maxiter=400)
    lam_min = float(np.min(lam))
    phi = W.cosine_basis(m, p.mask, cfg.k, cfg.basis_seed, np.float32)
    ev = O.rom_eval(m, rho, phi, p.mask, p.f)
    out = {
        "_source": "written by tests/golden/make_golden.py from the oracle only (FP64)",
        "workload": cfg.name,
        "field": 0,
        "rho_seed": cfg.rho_seed0,
        "k": cfg.k,
        "basis_seed": cfg.basis_seed,
        "cg_iters": info["iters"],
        "rel_resid": float(np.linalg.norm(r) / np.linalg.norm(p.f[free])),
        "compliance_raw": c_raw,
        "compliance_corr": c_corr,
        "lambda_min_estimate": lam_min,
        "bracket": float(np.dot(r, r) / lam_min),
        "Jk": ev["Jk"],
        "resnorm": ev["resnorm"],
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "cantilever3d_96x48x48.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
