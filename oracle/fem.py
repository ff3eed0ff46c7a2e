"""Full-order (HDM) side of the oracle: element stiffness, SIMP law, assembled K(rho),
direct / CG solve, compliance and the element sensitivity.  FP64 throughout.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ----------------------------------------------------------------------------------
# Material law  (Sec. 2.1: alpha(rho) = rho_l + (1 - rho_l) rho^p, here written with
# the stiffness bounds E0 / Emin: alpha = Emin + (E0 - Emin) rho^p; the paper's law is
# the special case E0 = 1, Emin = rho_l.)
# ----------------------------------------------------------------------------------

def simp_alpha(rho, E0, Emin, p):
    """Stiffness factor of an element of density rho (Sec. 2.1, material law)."""
    return Emin + (E0 - Emin) * np.asarray(rho, dtype=np.float64) ** p


def simp_alpha_prime(rho, E0, Emin, p):
    """d alpha / d rho = p (E0 - Emin) rho^(p-1) (Sec. 2.4, sensitivity expression)."""
    return p * (E0 - Emin) * np.asarray(rho, dtype=np.float64) ** (p - 1)


# ----------------------------------------------------------------------------------
# Element stiffness of the unit-density bilinear / trilinear element  (Sec. 2.1)
# ----------------------------------------------------------------------------------

def constitutive(dim, E, nu, plane_stress=True):
    """Isotropic linear-elastic material matrix in Voigt form with engineering shear
    strains: 2D [exx, eyy, gxy] (plane stress or plane strain), 3D
    [exx, eyy, ezz, gyz, gxz, gxy]."""
    if dim == 2:
        if plane_stress:
            c = E / (1.0 - nu * nu)
            return c * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, (1.0 - nu) / 2.0]])
        c = E / ((1.0 + nu) * (1.0 - 2.0 * nu))
        return c * np.array([[1.0 - nu, nu, 0.0], [nu, 1.0 - nu, 0.0],
                             [0.0, 0.0, (1.0 - 2.0 * nu) / 2.0]])
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[:3, :3] += 2.0 * mu * np.eye(3)
    D[3:, 3:] = mu * np.eye(3)
    return D


def _local_nodes(dim):
    """Tensor-order local nodes: a = ax + 2 ay (+ 4 az), each offset in {0, 1}."""
    return [tuple((a >> d) & 1 for d in range(dim)) for a in range(2 ** dim)]


def element_stiffness(dim, h, E=1.0, nu=0.3, plane_stress=True, ngauss=2):
    """Unit-density element stiffness K_e (Sec. 2.1), integrated with an ngauss^dim
    Gauss-Legendre rule (2 points per axis integrate the rectangular Q1 element
    exactly).  Local DOF ordering: dim * a + c for tensor-order local node a and
    displacement component c.  Unit thickness in 2D."""
    h = np.asarray(h, dtype=np.float64)
    D = constitutive(dim, E, nu, plane_stress)
    xg, wg = np.polynomial.legendre.leggauss(ngauss)
    nodes = _local_nodes(dim)
    nen = len(nodes)
    ne = dim * nen
    nstr = 3 if dim == 2 else 6
    K = np.zeros((ne, ne))
    detJ = np.prod(h) / 2.0 ** dim
    for idx in np.ndindex(*([ngauss] * dim)):
        xi = np.array([xg[i] for i in idx])
        w = np.prod([wg[i] for i in idx])
        # physical derivatives of the shape functions at this point
        dN = np.zeros((nen, dim))
        for a, off in enumerate(nodes):
            s = 2.0 * np.array(off) - 1.0
            for d in range(dim):
                val = s[d] / 2.0
                for e in range(dim):
                    if e != d:
                        val *= (1.0 + s[e] * xi[e]) / 2.0
                dN[a, d] = val * 2.0 / h[d]
        B = np.zeros((nstr, ne))
        for a in range(nen):
            if dim == 2:
                dx, dy = dN[a]
                B[0, 2 * a] = dx
                B[1, 2 * a + 1] = dy
                B[2, 2 * a] = dy
                B[2, 2 * a + 1] = dx
            else:
                dx, dy, dz = dN[a]
                c0 = 3 * a
                B[0, c0] = dx
                B[1, c0 + 1] = dy
                B[2, c0 + 2] = dz
                B[3, c0 + 1] = dz
                B[3, c0 + 2] = dy
                B[4, c0] = dz
                B[4, c0 + 2] = dx
                B[5, c0] = dy
                B[5, c0 + 1] = dx
        K += w * detJ * B.T @ D @ B
    return K


# ----------------------------------------------------------------------------------
# Assembly  (Sec. 2.1: K(rho) = sum_e alpha(rho_e) P_e K_e P_e^T)
# ----------------------------------------------------------------------------------

def element_dofs(mesh):
    """Global DOF index of every element DOF, shape [n_elems, dim * 2^dim], in the
    local ordering of element_stiffness (the assembly operator P_e of Sec. 2.1)."""
    dim = mesh.dim
    nel = mesh.nel
    nn = mesh.nn
    n_nodes = mesh.n_nodes
    e = np.arange(mesh.n_elems)
    ex = e % nel[0]
    ey = (e // nel[0]) % nel[1]
    ez = e // (nel[0] * nel[1]) if dim == 3 else np.zeros_like(e)
    cols = []
    for off in _local_nodes(dim):
        oz = off[2] if dim == 3 else 0
        node = (ex + off[0]) + nn[0] * ((ey + off[1]) + nn[1] * (ez + oz))
        for c in range(dim):
            cols.append(c * n_nodes + node)
    return np.stack(cols, axis=1)


def free_dofs(mask):
    return np.flatnonzero(np.asarray(mask) == 0)


def _K0(mesh, plane_stress=True):
    return element_stiffness(mesh.dim, mesh.h, 1.0, mesh.nu, plane_stress)


def assemble(mesh, rho, plane_stress=True):
    """Assembled sparse K(rho) over all DOFs (constrained ones included), CSR."""
    K0 = _K0(mesh, plane_stress)
    alpha = simp_alpha(rho, mesh.E0, mesh.Emin, mesh.penal)
    edofs = element_dofs(mesh)
    ne = edofs.shape[1]
    rows = np.repeat(edofs, ne, axis=1).ravel()
    cols = np.tile(edofs, (1, ne)).ravel()
    vals = (alpha[:, None] * K0.ravel()[None, :]).ravel()
    n = mesh.n_dofs
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def apply_masked(mesh, rho, mask, x, plane_stress=True):
    """y = K(rho) x with Dirichlet DOFs eliminated: y_f = K_ff x_f, y_c = 0
    (Sec. 2.1, last paragraph: constrained DOFs are removed from the residual)."""
    K = assemble(mesh, rho, plane_stress)
    free = np.asarray(mask) == 0
    xf = np.where(free, x, 0.0)
    return np.where(free, K @ xf, 0.0)


def apply_ebe(mesh, rho, mask, x, plane_stress=True, chunk=1 << 18):
    """y = K(rho) x with Dirichlet DOFs eliminated (as apply_masked), summed element by
    element without assembling K (for meshes whose assembled matrix does not fit in
    host memory): y = sum_e alpha_e P_e K_e P_e^T x, in chunks of elements."""
    K0 = _K0(mesh, plane_stress)
    alpha = simp_alpha(rho, mesh.E0, mesh.Emin, mesh.penal)
    free = np.asarray(mask) == 0
    xf = np.where(free, np.asarray(x, dtype=np.float64), 0.0)
    y = np.zeros(mesh.n_dofs)
    edofs = element_dofs(mesh)
    for e0 in range(0, mesh.n_elems, chunk):
        ed = edofs[e0:e0 + chunk]
        ye = (xf[ed] @ K0.T) * alpha[e0:e0 + chunk, None]
        y += np.bincount(ed.ravel(), weights=ye.ravel(), minlength=mesh.n_dofs)
    return np.where(free, y, 0.0)


def apply_rows(mesh, rho, mask, x, nodes, plane_stress=True):
    """(K(rho) x) at the listed nodes only, summed element by element without any
    assembly (for meshes too large to assemble in a test).  Same Dirichlet convention
    as apply_masked.  Returns [dim, len(nodes)]."""
    K0 = _K0(mesh, plane_stress)
    dim = mesh.dim
    nel, nn = mesh.nel, mesh.nn
    alpha = simp_alpha(rho, mesh.E0, mesh.Emin, mesh.penal)
    free = np.asarray(mask) == 0
    xf = np.where(free, x, 0.0)
    locs = _local_nodes(dim)
    out = np.zeros((dim, len(nodes)))
    for t, node in enumerate(nodes):
        ijk = [node % nn[0], (node // nn[0]) % nn[1]]
        if dim == 3:
            ijk.append(node // (nn[0] * nn[1]))
        for a, off in enumerate(locs):
            eijk = [ijk[d] - off[d] for d in range(dim)]
            if any(eijk[d] < 0 or eijk[d] >= nel[d] for d in range(dim)):
                continue
            e = eijk[0] + nel[0] * (eijk[1] + (nel[1] * eijk[2] if dim == 3 else 0))
            ue = np.zeros(dim * len(locs))
            for b, offb in enumerate(locs):
                nb = sum((eijk[d] + offb[d]) * int(np.prod(nn[:d])) for d in range(dim))
                for c in range(dim):
                    ue[dim * b + c] = xf[c * mesh.n_nodes + nb]
            ye = alpha[e] * (K0 @ ue)
            for c in range(dim):
                out[c, t] += ye[dim * a + c]
    for c in range(dim):
        out[c] = np.where(free[c * mesh.n_nodes + np.asarray(nodes)], out[c], 0.0)
    return out


# ----------------------------------------------------------------------------------
# State solve, compliance, sensitivity  (Sec. 2.1, 2.3, 2.4 and the adjoint appendix)
# ----------------------------------------------------------------------------------

def solve_direct(mesh, rho, f, mask, plane_stress=True):
    """u* = K_ff(rho)^{-1} f_f on the free DOFs, u = 0 on Dirichlet DOFs, by a sparse
    direct factorisation with a fill-reducing ordering (the paper's HDM solver, Sec.
    2.5 item 5).  SuperLU with symmetric-mode pivoting on the SPD matrix."""
    K = assemble(mesh, rho, plane_stress)
    free = free_dofs(mask)
    Kff = K[free][:, free].tocsc()
    lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    u = np.zeros(mesh.n_dofs)
    u[free] = lu.solve(np.asarray(f, dtype=np.float64)[free])
    return u


def solve_cg(mesh, rho, f, mask, rtol=1e-13, maxiter=200000, plane_stress=True,
             x0=None, restarts=20, info=None):
    """FP64 Jacobi-preconditioned CG on the assembled K_ff, for meshes too large for a
    direct factorisation in host memory.  CG is restarted from its iterate until the
    *true* residual ||f_f - K_ff u_f|| / ||f_f|| is at most rtol (or the restart budget
    is spent).  Returns (u, relative true residual); a dict passed as info receives the
    number of CG iterations ("iters")."""
    K = assemble(mesh, rho, plane_stress)
    free = free_dofs(mask)
    Kff = K[free][:, free].tocsr()
    d = Kff.diagonal()
    M = sp.diags(1.0 / d)
    b = np.asarray(f, dtype=np.float64)[free]
    nb = np.linalg.norm(b)
    xf = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64)[free].copy()
    res = np.linalg.norm(b - Kff @ xf) / nb
    its = [0]

    def count(_xk):
        its[0] += 1

    for _ in range(restarts):
        if res <= rtol:
            break
        r = b - Kff @ xf
        # solve the correction equation to a relative accuracy that lands below rtol
        dx, _info = spla.cg(Kff, r, rtol=max(rtol / res * 0.5, 1e-15), atol=0.0,
                            maxiter=maxiter, M=M, callback=count)
        xf += dx
        res = np.linalg.norm(b - Kff @ xf) / nb
    u = np.zeros(mesh.n_dofs)
    u[free] = xf
    if info is not None:
        info["iters"] = its[0]
    return u, res


def compliance(f, u):
    """j_c = f^T u (Sec. 2.3)."""
    return float(np.dot(np.asarray(f, dtype=np.float64), np.asarray(u, dtype=np.float64)))


def sensitivity(mesh, rho, u, plane_stress=True):
    """Element sensitivity of the compliance with respect to the filtered density:
    dc/drho_e = -alpha'(rho_e) u_e^T K_e u_e, using lambda* = u* (Sec. 2.4, the
    compliance remark, and the adjoint appendix)."""
    K0 = _K0(mesh, plane_stress)
    ue = np.asarray(u, dtype=np.float64)[element_dofs(mesh)]
    quad = np.einsum("ei,ij,ej->e", ue, K0, ue)
    return -simp_alpha_prime(rho, mesh.E0, mesh.Emin, mesh.penal) * quad
