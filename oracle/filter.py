"""Helmholtz density filter of the oracle (Sec. 2.2) and its adjoint (Sec. 2.4 gradient
through the filter, and the adjoint appendix).  FP64.

Forward map psi -> rho*(psi):
  H phi = b(psi),   H = sum_e Q_e H_e Q_e^T,   b(psi) = sum_e psi_e Q_e b_e,
  rho_e = (1 / N_v^e) 1^T Q_e^T phi,
with H_e = r^2 (element Laplacian) + (element mass) of the scalar bilinear / trilinear
element, b_e = the integrals of the element's shape functions, homogeneous Neumann
boundary (no constrained node).  The Helmholtz length r is an argument; Sec. 2.2
prints r = 2 sqrt(3) R for a filter radius R, the cited filter reference has
r = R / (2 sqrt(3)) (filter_radius / filter_radius_cited).

Adjoint: for v in R^{N_e}, (d rho*/d psi)^T v has entries b_e^T Q_e^T mu, where
H^T mu = q(v) = sum_e (v_e / N_v^e) Q_e 1.  The paper prints this with a leading minus
sign; its own definitions (dR/dpsi_e = -Q_e b_e, d phi*/d psi = -(dR/dphi)^{-1} dR/dpsi)
give the plus sign, which the pins (finite differences, the dot-product test) confirm.

Element matrices by their own 2-point Gauss rule per axis (exact for these integrands);
assembly COO -> CSR; sparse direct solve.  Test infrastructure only (see the package
docstring).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def helmholtz_element(dim, h, r):
    """H_e = r^2 int grad N_i . grad N_j + int N_i N_j and b_e = int N_i over the box
    element with sides h (Sec. 2.2); local node order x fastest, then y, then z."""
    h = np.asarray(h, dtype=np.float64)[:dim]
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    corners = list(itertools.product((0, 1), repeat=dim))
    corners = [c[::-1] for c in corners]  # x fastest
    nen = len(corners)
    H = np.zeros((nen, nen))
    b = np.zeros(nen)
    jac = np.prod(h) / 2.0 ** dim  # reference cube [-1, 1]^dim
    for gp in itertools.product(g, repeat=dim):
        N = np.empty(nen)
        dN = np.empty((nen, dim))
        for a, c in enumerate(corners):
            s = [(1 + (2 * c[d] - 1) * gp[d]) / 2.0 for d in range(dim)]
            N[a] = np.prod(s)
            for d in range(dim):
                ds = (2 * c[d] - 1) / 2.0 * (2.0 / h[d])  # d s_d / d x_d
                dN[a, d] = ds * np.prod([s[e] for e in range(dim) if e != d])
        H += (r * r * dN @ dN.T + np.outer(N, N)) * jac
        b += N * jac
    return H, b


def element_nodes(mesh):
    """Global node index of each element's local nodes (x fastest)."""
    nx, ny = mesh.nel[0], mesh.nel[1]
    nz = mesh.nel[2] if mesh.dim == 3 else 1
    n1x, n1y = nx + 1, ny + 1
    out = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if mesh.dim == 2:
                    out.append([i + n1x * j, i + 1 + n1x * j, i + n1x * (j + 1), i + 1 + n1x * (j + 1)])
                else:
                    base = lambda di, dj, dk: (i + di) + n1x * ((j + dj) + n1y * (k + dk))
                    out.append([base(di, dj, dk) for dk in (0, 1) for dj in (0, 1) for di in (0, 1)])
    return np.array(out, dtype=np.int64)


def helmholtz_assemble(mesh, r):
    """The assembled Helmholtz matrix H (N_v x N_v, CSR) and the element load b_e."""
    He, be = helmholtz_element(mesh.dim, mesh.h, r)
    en = element_nodes(mesh)
    nen = en.shape[1]
    rows = np.repeat(en, nen, axis=1).ravel()
    cols = np.tile(en, (1, nen)).ravel()
    vals = np.tile(He.ravel(), en.shape[0])
    H = sp.coo_matrix((vals, (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    return H, be


def filter_load(mesh, r, psi):
    """b(psi) = sum_e psi_e Q_e b_e (Sec. 2.2)."""
    _, be = helmholtz_element(mesh.dim, mesh.h, r)
    en = element_nodes(mesh)
    b = np.zeros(mesh.n_nodes)
    np.add.at(b, en.ravel(), (np.asarray(psi, dtype=np.float64)[:, None] * be[None, :]).ravel())
    return b


def filter_forward(mesh, r, psi):
    """rho*(psi): nodal Helmholtz solve H phi = b(psi), then element averages of phi
    (Sec. 2.2).  Returns (rho, phi)."""
    H, _ = helmholtz_assemble(mesh, r)
    phi = spla.spsolve(H.tocsc(), filter_load(mesh, r, psi))
    en = element_nodes(mesh)
    return phi[en].mean(axis=1), phi


def filter_adjoint(mesh, r, v):
    """(d rho*/d psi)^T v: mu = H^{-T} q(v), q(v) = sum_e (v_e / N_v^e) Q_e 1, then
    entry e = b_e^T Q_e^T mu (Sec. 2.4 and the adjoint appendix, with the sign the
    definitions give).  Returns (g, mu)."""
    H, be = helmholtz_assemble(mesh, r)
    en = element_nodes(mesh)
    nen = en.shape[1]
    q = np.zeros(mesh.n_nodes)
    np.add.at(q, en.ravel(), np.repeat(np.asarray(v, dtype=np.float64) / nen, nen))
    mu = spla.spsolve(H.T.tocsc(), q)
    return mu[en] @ be, mu


def filter_radius(R):
    """r = 2 sqrt(3) R for the filter's characteristic radius R, as Sec. 2.2 prints it."""
    return 2.0 * np.sqrt(3.0) * R


def filter_radius_cited(R):
    """r = R / (2 sqrt(3)): the Helmholtz length whose filter kernel has the second moment
    of the conic density filter of radius R, the relation of the filter reference that
    Sec. 2.2 cites (the paper's text prints the inverse factor; see filter_radius)."""
    return R / (2.0 * np.sqrt(3.0))
