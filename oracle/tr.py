"""ROM trust-region topology optimisation of the oracle: Algorithm 2 of Sec. 4.3 (the
error-aware trust-region method with on-the-fly reduced models) for compliance, with
the residual trust region (ROM-TR-RES) or the distance trust region (ROM-TR-DIST).

Every evaluation uses the oracle: Helmholtz filter by direct solves, HDM by the sparse
direct solver, basis by SVD + Gram-Schmidt (Sec. 4.2), reduced model from the
assembled matrix.  Readings where the paper leaves a choice (each stated again where
it is used):

* feasible set C = {0 <= psi <= 1, sum_e psi_e |Omega_e| <= V}; the subproblem solver is
  projected gradient (the paper uses MMA) on min_{psi in C} m_k(psi), stopped at the
  first iterate outside the trust region, as the paper stops its MMA iterations;
* a projected-gradient step moves psi - t g onto C with t = move / max|g|, halving the
  move until the Armijo condition m(new) <= m(old) - 1e-4 g^T (old - new) holds; a first
  step outside the trust region is halved until it is inside;
* radius update with the paper's constants (gamma_1 = 0.5, gamma_2 = 1, eta_1 = 0.1,
  eta_2 = 0.75, Delta_max = 100 Delta_0): unsuccessful -> gamma_1 Delta, successful ->
  Delta, very successful -> min(2 Delta, Delta_max);
* a rejected step keeps the centre, so the model (basis) is kept and only the radius
  shrinks.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .basis import SnapshotWindow, basis_update
from .fem import compliance, solve_direct
from .filter import filter_adjoint, filter_forward
from .rom import rom_eval, rom_gradient

GAMMA1, GAMMA2, ETA1, ETA2 = 0.5, 1.0, 0.1, 0.75


def project_feasible(psi, vmax, weights=None):
    """Euclidean projection onto {0 <= psi <= 1, sum w_e psi_e <= vmax} (w = 1 by default):
    clip(psi - lambda w, 0, 1) with the smallest lambda >= 0 meeting the volume, found
    exactly from the sorted breakpoints of the piecewise-linear volume(lambda)."""
    psi = np.asarray(psi, dtype=np.float64)
    w = np.ones_like(psi) if weights is None else np.asarray(weights, dtype=np.float64)
    x = np.clip(psi, 0.0, 1.0)
    if np.dot(w, x) <= vmax:
        return x
    # volume(lam) = sum w clip(psi - lam w, 0, 1) decreases piecewise linearly in lam
    bps = np.unique(np.concatenate([(psi - 1.0) / w, psi / w]))
    bps = bps[bps >= 0.0]
    vol = lambda lam: float(np.dot(w, np.clip(psi - lam * w, 0.0, 1.0)))
    lo = 0.0
    for b in bps:
        if vol(b) <= vmax:
            hi = b
            break
        lo = b
    else:
        hi = bps[-1]
    vlo, vhi = vol(lo), vol(hi)
    lam = hi if vlo == vhi else lo + (vlo - vmax) * (hi - lo) / (vlo - vhi)
    return np.clip(psi - lam * w, 0.0, 1.0)


def update_radius(delta, ratio, delta_max):
    """Trust-region radius update of Algorithm 2 with the paper's constants."""
    if ratio < ETA1:
        return GAMMA1 * delta
    if ratio < ETA2:
        return GAMMA2 * delta
    return min(2.0 * delta, delta_max)


class Problem:
    """Compliance minimisation on a mesh with a Helmholtz filter of length r and volume
    fraction vf (V = vf |Omega|)."""

    def __init__(self, mesh, mask, f, r, vf):
        self.mesh, self.mask, self.f, self.r, self.vf = mesh, mask, np.asarray(f, dtype=np.float64), r, vf
        self.vmax = vf * mesh.n_elems  # equal elements: volumes counted in elements

    def hdm(self, psi):
        """J(psi) and the HDM state at rho*(psi) (Sec. 2)."""
        rho, _ = filter_forward(self.mesh, self.r, psi)
        u = solve_direct(self.mesh, rho, self.f, self.mask)
        return compliance(self.f, u), u, rho

    def model(self, psi, phi, want_grad=False):
        """m_k(psi) = J_k(rho*(psi)) with the residual norm (Sec. 3.3), and its gradient
        with respect to psi through the filter (Sec. 3.2, 2.4) when asked."""
        rho, _ = filter_forward(self.mesh, self.r, psi)
        ev = rom_eval(self.mesh, rho, phi, self.mask, self.f)
        g = None
        if want_grad:
            dJ, _ = rom_gradient(self.mesh, rho, phi, self.mask, self.f)
            g, _ = filter_adjoint(self.mesh, self.r, dJ)
        return ev["Jk"], ev["resnorm"], g


def subproblem(prob, phi, center, delta, kind, move=0.1, steps=10):
    """Approximate trust-region subproblem (see the module readings).  Returns the
    candidate, the model value at the centre and at the candidate, and the number of
    model evaluations."""
    nevals = 0

    def theta(psi, resnorm):
        return resnorm if kind == "res" else float(np.linalg.norm(psi - center))

    m0, _, g = prob.model(center, phi, want_grad=True)
    nevals += 1
    psi, mval = center.copy(), m0
    for s in range(steps):
        gmax = np.abs(g).max()
        if gmax == 0.0:
            break
        t = move / gmax
        accepted = None
        for _ in range(30):
            trial = project_feasible(psi - t * g, prob.vmax)
            mt, rn, _ = prob.model(trial, phi)
            nevals += 1
            inside = theta(trial, rn) <= delta
            armijo = mt <= mval - 1e-4 * float(g @ (psi - trial))
            if armijo and (inside or s > 0):
                accepted = (trial, mt, inside)
                break
            t *= 0.5
        if accepted is None:
            break
        trial, mt, inside = accepted
        if not inside:  # left the trust region: keep the last iterate inside
            break
        psi, mval = trial, mt
        _, _, g = prob.model(psi, phi, want_grad=True)
        nevals += 1
    return psi, m0, mval, nevals


def rom_tr(prob, kind="res", tau=0.1, iters=5, window=5, nmax=4, move=0.1, steps=10):
    """Algorithm 2 for `iters` outer iterations from the uniform design psi0 = vf.
    Returns the final centre and the per-iteration history."""
    psi = np.full(prob.mesh.n_elems, prob.vf)
    free = np.asarray(prob.mask) == 0
    delta = tau * (float(np.linalg.norm(prob.f[free])) if kind == "res" else float(np.linalg.norm(psi)))
    delta_max = 100.0 * delta
    win = SnapshotWindow(window)
    J, u, _ = prob.hdm(psi)
    phi = None
    hist = []
    for k in range(iters):
        if phi is None:  # model update at a new centre (Sec. 4.2)
            phi, n, keep, _ = basis_update(win.matrix(prob.mesh.n_dofs), u, nmax)
            win.push(u)
        cand, m0, mc, nev = subproblem(prob, phi, psi, delta, kind, move, steps)
        pred = m0 - mc
        if pred > 0.0:
            Jc, uc, _ = prob.hdm(cand)
            ratio = (J - Jc) / pred
        else:
            Jc, uc, ratio = J, u, -np.inf
        accepted = ratio >= ETA1
        hist.append(dict(J=J, model_center=m0, model_cand=mc, J_cand=Jc, ratio=ratio, delta=delta,
                         accepted=accepted, basis=phi.shape[1], model_evals=nev))
        delta = update_radius(delta, ratio, delta_max)
        if accepted:
            psi, J, u = cand, Jc, uc
            phi = None
    return psi, hist
