"""Reduced-order (ROM) side of the oracle: Galerkin operator, reduced load, reduced
Cholesky solve, ROM compliance and the residual-norm error indicator.  FP64.

The reduced operator is formed from the *assembled* sparse K(rho) as Phi^T (K Phi),
which is algorithmically different from the per-element contraction the paper
recommends (Sec. 3.1, remark on dense assembly) and the HIP path uses.

Dirichlet convention: rows of Phi and entries of f on constrained DOFs are ignored
(taken as zero), so Phi^T K Phi = Phi_f^T K_ff Phi_f.  A float32 basis is promoted
exactly to float64, so both sides project onto the same space.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fem import assemble, sensitivity


def _masked(phi, mask):
    a = np.array(phi, dtype=np.float64, copy=True)
    a[np.asarray(mask) != 0] = 0.0
    return a


def rom_operator(mesh, rho, phi, mask, plane_stress=True):
    """K_hat(rho) = Phi^T K(rho) Phi  (Sec. 3.1, Galerkin reduced stiffness)."""
    P = _masked(phi, mask)
    K = assemble(mesh, rho, plane_stress)
    return P.T @ (K @ P)


def rom_load(phi, mask, f):
    """f_hat = Phi^T f  (Sec. 3.1, reduced load)."""
    P = _masked(phi, mask)
    ff = np.where(np.asarray(mask) != 0, 0.0, np.asarray(f, dtype=np.float64))
    return P.T @ ff


def rom_solve(Khat, fhat):
    """y_hat = K_hat^{-1} f_hat by dense Cholesky, and the ROM compliance
    J_k = f^T Phi y_hat = f_hat^T y_hat  (Sec. 3.1 and the ROM objective definition)."""
    c = sla.cho_factor(np.asarray(Khat, dtype=np.float64), lower=True)
    y = sla.cho_solve(c, np.asarray(fhat, dtype=np.float64))
    return y, float(np.dot(fhat, y))


def rom_residual(mesh, rho, phi, mask, f, yhat, plane_stress=True):
    """Residual of the reconstructed ROM state u_k = Phi y_hat:
    r = f - K(rho) u_k on the free DOFs (zero on constrained ones), and ||r||_2
    (Sec. 3.3, primal residual; Sec. 4.3, residual trust-region constraint)."""
    P = _masked(phi, mask)
    uk = P @ np.asarray(yhat, dtype=np.float64)
    K = assemble(mesh, rho, plane_stress)
    free = np.asarray(mask) == 0
    r = np.where(free, np.asarray(f, dtype=np.float64) - K @ uk, 0.0)
    return r, float(np.linalg.norm(r)), uk


def rom_eval(mesh, rho, phi, mask, f, plane_stress=True):
    """One full ROM evaluation: K_hat, f_hat, y_hat, J_k and ||r||."""
    Kh = rom_operator(mesh, rho, phi, mask, plane_stress)
    fh = rom_load(phi, mask, f)
    y, J = rom_solve(Kh, fh)
    _, rn, _ = rom_residual(mesh, rho, phi, mask, f, y, plane_stress)
    return dict(Khat=Kh, fhat=fh, yhat=y, Jk=J, resnorm=rn)


def rom_gradient(mesh, rho, phi, mask, f, plane_stress=True):
    """Sensitivity of the ROM compliance J_k(rho) = f_hat^T K_hat(rho)^{-1} f_hat with
    respect to the densities: dJ_k/drho_e = -y_hat^T (dK_hat/drho_e) y_hat
    = -alpha'(rho_e) u_k,e^T K_e u_k,e with u_k = Phi y_hat.  For the compliance the
    reduced adjoint equals the reduced state (Sec. 3.2), so this is the element
    sensitivity of Sec. 2.4 evaluated at the ROM state.  Returns (dJ_k, J_k)."""
    ev = rom_eval(mesh, rho, phi, mask, f, plane_stress)
    uk = _masked(phi, mask) @ ev["yhat"]
    return sensitivity(mesh, rho, uk, plane_stress), ev["Jk"]
