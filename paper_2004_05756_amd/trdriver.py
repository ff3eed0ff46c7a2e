"""Host driver of the ROM trust-region method for compliance (Algorithm 2, Sec. 4.3) over
libtopo_rom.

Every evaluation runs in the library on the device: the Helmholtz filter and its
adjoint (Sec. 2.2, 2.4), the HDM solve (Sec. 2.1), the basis update at each centre
(POD of the snapshot window plus one Gram-Schmidt step, Sec. 4.2), the reduced model
with its residual (Sec. 3.1, 3.3) and its sensitivity (Sec. 3.2).  The host keeps the
design vector psi and takes the optimiser's decisions:

* feasible set C = {0 <= psi <= 1, sum psi_e <= vf N_e} (equal elements), Euclidean
  projection by bisection on the volume multiplier;
* the subproblem is approximated as the paper does with its MMA iterations: steps of an
  optimiser on min_{psi in C} m_k(psi), stopped once the trust-region constraint is
  violated; the steps here are projected gradient steps psi - t g with t = move / max|g|,
  halved until m decreases by at least 1e-4 g^T (psi - new) (a first step outside the
  trust region is halved until it is inside);
* ratio of actual to predicted reduction, acceptance at ratio >= 0.1, radius update with
  the paper's constants (0.5 on failure, kept when successful, doubled up to 100 Delta_0
  when very successful, ratio >= 0.75);
* the trust region is the ROM residual norm (kind "res") or the distance to the centre
  (kind "dist"); Delta_0 = tau |f| or tau |psi_0|.

Consecutive filter solves start from the previous nodal solution (the designs the
optimiser evaluates one after the other are close).
"""
from __future__ import annotations

import numpy as np

from . import binding
from .binding import FP64

ETA1, ETA2, GAMMA1, GAMMA2 = 0.1, 0.75, 0.5, 1.0


def project_box_volume(psi: np.ndarray, vmax: float, iters: int = 200) -> np.ndarray:
    """Projection onto {0 <= x <= 1, sum x <= vmax}: x = clip(psi - lam), the smallest
    lam >= 0 that meets the volume, by bisection (the volume decreases in lam)."""
    x = np.clip(psi, 0.0, 1.0)
    if x.sum() <= vmax:
        return x
    lo, hi = 0.0, float(psi.max())
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.clip(psi - mid, 0.0, 1.0).sum() > vmax:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * max(1.0, hi):
            break
    return np.clip(psi - hi, 0.0, 1.0)


class TrustRegion:
    """ROM trust-region optimisation of the compliance of one problem on one device."""

    def __init__(self, ctx, mesh, mask, f, r, vf, kind="res", window=5, nmax=4, prec=FP64,
                 hdm_rtol=1e-10, filter_rtol=1e-13, move=0.1, steps=10):
        import torch
        self.torch = torch
        self.ctx, self.mesh, self.r, self.vf, self.kind = ctx, mesh, r, vf, kind
        self.prec, self.hdm_rtol, self.filter_rtol = prec, hdm_rtol, filter_rtol
        self.move, self.steps, self.nmax = move, steps, nmax
        self.dev = torch.device("cuda", ctx.device if hasattr(ctx, "device") else 0)
        self.mask = torch.as_tensor(np.ascontiguousarray(mask, dtype=np.uint8)).to(self.dev)
        self.f = torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64)).to(self.dev)
        self.fnorm = float(np.linalg.norm(np.asarray(f)[np.asarray(mask) == 0]))
        self.vmax = vf * mesh.n_elems
        self.win = binding.SnapshotWindow(ctx, mesh.n_dofs, window, device=self.dev)
        self.phi = torch.zeros((mesh.n_dofs, nmax + 1), dtype=torch.float64, device=self.dev)
        self.k = 0
        self.model_evals = 0
        self.hdm_solves = 0
        # nodal filter solutions of the last forward / adjoint solve, warm starts for the next
        self.phi_nodal = torch.zeros((1, mesh.n_nodes), dtype=torch.float64, device=self.dev)
        self.mu_nodal = torch.zeros((1, mesh.n_nodes), dtype=torch.float64, device=self.dev)
        self.warm_phi = self.warm_mu = False

    # -- evaluations on the device -------------------------------------------------
    def _rho(self, psi):
        x = self.torch.as_tensor(np.ascontiguousarray(psi, dtype=np.float64)[None]).to(self.dev)
        rho, _ = self.ctx.filter_forward(self.mesh, self.r, x, phi=self.phi_nodal, rtol=self.filter_rtol,
                                         warm=self.warm_phi)
        self.warm_phi = True
        return rho

    def hdm(self, psi):
        """J(psi) (residual-corrected compliance) and the HDM state at rho*(psi)."""
        rho = self._rho(psi)
        u, inf = self.ctx.hdm_solve(self.mesh, rho[0], self.mask, self.f, rtol=self.hdm_rtol, prec=self.prec)
        self.hdm_solves += 1
        return inf["compliance_corr"], u

    def new_centre(self, u):
        """Basis at a new centre: GramSchmidt([POD(window), u]), then u joins the window."""
        self.k, _ = self.win.basis(u, self.nmax, self.phi)
        self.win.push(u)

    def model(self, psi, want_grad=False):
        """m_k(psi), the ROM residual norm, and (optionally) dm_k/dpsi on the host."""
        rho = self._rho(psi)
        Kh, fh = self.ctx.rom_build(self.mesh, self.phi, self.k, self.mask, self.f, rho, prec=self.prec)
        y, Jk = self.ctx.rom_solve(Kh, fh)
        self.model_evals += 1
        rn = 0.0
        dJ = self.torch.empty_like(rho) if want_grad else None
        if self.kind == "res":  # the sensitivity comes with the estimate (same u = Phi y)
            y, Je, resn = self.ctx.rom_estimate(self.mesh, self.phi, self.k, self.mask, self.f, rho, Kh, y,
                                                max_refine=0, dJ=dJ)
            rn = float(resn[0])
        elif want_grad:
            dJ = self.ctx.rom_gradient(self.mesh, self.phi, self.k, self.mask, rho, y, dJ=dJ)
        g = None
        if want_grad:
            gd, _ = self.ctx.filter_adjoint(self.mesh, self.r, dJ, mu=self.mu_nodal, rtol=self.filter_rtol,
                                            warm=self.warm_mu)
            self.warm_mu = True
            g = gd[0].cpu().numpy()
        return float(Jk[0]), rn, g

    # -- the optimiser (host) ------------------------------------------------------
    def subproblem(self, centre, delta):
        def theta(psi, rn):
            return rn if self.kind == "res" else float(np.linalg.norm(psi - centre))

        m0, _, g = self.model(centre, want_grad=True)
        psi, mval = centre.copy(), m0
        for s in range(self.steps):
            gmax = float(np.abs(g).max())
            if gmax == 0.0:
                break
            t = self.move / gmax
            found = None
            for _ in range(30):
                trial = project_box_volume(psi - t * g, self.vmax)
                mt, rn, _ = self.model(trial)
                inside = theta(trial, rn) <= delta
                if mt <= mval - 1e-4 * float(g @ (psi - trial)) and (inside or s > 0):
                    found = (trial, mt, inside)
                    break
                t *= 0.5
            if found is None or not found[2]:
                break
            psi, mval = found[0], found[1]
            _, _, g = self.model(psi, want_grad=True)
        return psi, m0, mval

    def run(self, iters=5, tau=0.1, psi0=None):
        """Outer iterations of Algorithm 2 from psi0 (default: the uniform design vf).
        Returns the final centre and the per-iteration history."""
        psi = np.full(self.mesh.n_elems, self.vf) if psi0 is None else np.asarray(psi0, dtype=np.float64)
        delta = tau * (self.fnorm if self.kind == "res" else float(np.linalg.norm(psi)))
        delta_max = 100.0 * delta
        J, u = self.hdm(psi)
        fresh = True
        hist = []
        for _ in range(iters):
            if fresh:
                self.new_centre(u)
                fresh = False
            cand, m0, mc = self.subproblem(psi, delta)
            pred = m0 - mc
            if pred > 0.0:
                Jc, uc = self.hdm(cand)
                ratio = (J - Jc) / pred
            else:
                Jc, uc, ratio = J, u, -np.inf
            accepted = ratio >= ETA1
            hist.append(dict(J=J, model_center=m0, model_cand=mc, J_cand=Jc, ratio=ratio, delta=delta,
                             accepted=accepted, basis=self.k, model_evals=self.model_evals,
                             hdm_solves=self.hdm_solves))
            if ratio < ETA1:
                delta = GAMMA1 * delta
            elif ratio < ETA2:
                delta = GAMMA2 * delta
            else:
                delta = min(2.0 * delta, delta_max)
            if accepted:
                psi, J, u = cand, Jc, uc
                fresh = True
        return psi, hist
