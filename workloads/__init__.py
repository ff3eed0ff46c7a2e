"""Seeded synthetic inputs for the SIMP compliance / ROM hot path.

This module is shared by the oracle tests, the HIP-path tests and the benchmark.
It only describes *inputs*: structured-grid geometry, homogeneous Dirichlet masks,
nodal load vectors, element density fields and reduced bases.  It contains none of
the method's arithmetic (no element stiffness, no operator, no solve).

Conventions (shared by every consumer):

* structured grid of ``nel = (nx, ny[, nz])`` elements of size ``h``;
  nodes ``(i, j[, k])`` are numbered ``i + (nx+1) * (j + (ny+1) * k)`` (x fastest);
* elements ``(ex, ey[, ez])`` are numbered ``ex + nx * (ey + ny * ez)``;
* DOF vectors are structure-of-arrays: DOF of component ``c`` at node ``n`` is
  ``c * n_nodes + n``;
* ``mask[dof] = 1`` marks a homogeneous Dirichlet DOF (the paper eliminates those DOFs
  from the residual, Sec. 2.1);
* bases are row-major ``[n_dofs][k]`` with rows indexed like DOF vectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

__all__ = [
    "Mesh", "Problem", "mbb2d", "cantilever2d", "cantilever3d", "bridge3d",
    "paper_mbb", "paper_cantilever", "paper_ssbeam",
    "rho_jitter", "rho_smoothed", "rho_batch", "trust_region_fields", "cosine_basis", "orthonormalize",
    "orthonormalize_tall",
    "config", "CONFIG_NAMES", "SERVING_MESHES", "ServingRequest", "serving_stream", "poisson_arrivals",
]


@dataclass(frozen=True)
class Mesh:
    """Structured Q4 (2D) / H8 (3D) grid plus the SIMP material constants."""

    nel: Tuple[int, ...]
    h: Tuple[float, ...] = None
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    penal: float = 3.0

    def __post_init__(self):
        if self.h is None:
            object.__setattr__(self, "h", tuple(1.0 for _ in self.nel))
        if len(self.nel) not in (2, 3) or len(self.h) != len(self.nel):
            raise ValueError("mesh must be 2D or 3D with one h per axis")

    @property
    def dim(self) -> int:
        return len(self.nel)

    @property
    def nn(self) -> Tuple[int, ...]:
        """Nodes per axis."""
        return tuple(n + 1 for n in self.nel)

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.nn))

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.nel))

    @property
    def n_dofs(self) -> int:
        return self.dim * self.n_nodes

    def node(self, i, j, k=0):
        nx1, ny1 = self.nn[0], self.nn[1]
        return i + nx1 * (j + ny1 * k)

    def dof(self, c, node):
        return c * self.n_nodes + node

    def node_coords(self):
        """Integer grid coordinates of every node, shape [dim, n_nodes]."""
        grids = np.meshgrid(*[np.arange(n) for n in self.nn], indexing="ij")
        # meshgrid 'ij' gives axis 0 = x; flatten in Fortran order so x is fastest
        return np.stack([g.ravel(order="F") for g in grids])


@dataclass
class Problem:
    """A mesh with its Dirichlet mask and load vector (both length n_dofs)."""

    name: str
    mesh: Mesh
    mask: np.ndarray  # uint8 [n_dofs]
    f: np.ndarray     # float64 [n_dofs]
    notes: str = ""

    @property
    def n_free(self) -> int:
        return int(self.mesh.n_dofs - self.mask.sum())


def _edge_weights(n_seg: int) -> np.ndarray:
    """Consistent nodal weights of a unit uniform line load on n_seg linear segments."""
    w = np.ones(n_seg + 1)
    w[0] = w[-1] = 0.5
    return w / n_seg


def _face_weights(n1: int, n2: int) -> np.ndarray:
    """Consistent nodal weights of a unit uniform pressure on an n1 x n2 bilinear face."""
    return np.outer(_edge_weights(n1), _edge_weights(n2))


# ---------------------------------------------------------------------------------
# Problems of the benchmark suite (geometry and supports only)
# ---------------------------------------------------------------------------------

def mbb2d(nx: int = 60, ny: int = 20, **mat) -> Problem:
    """Half MBB beam: x-roller symmetry on x=0, y-support at the bottom-right node,
    unit downward load at the top-left node."""
    m = Mesh((nx, ny), **mat)
    mask = np.zeros(m.n_dofs, np.uint8)
    for j in range(ny + 1):
        mask[m.dof(0, m.node(0, j))] = 1
    mask[m.dof(1, m.node(nx, 0))] = 1
    f = np.zeros(m.n_dofs)
    f[m.dof(1, m.node(0, ny))] = -1.0
    return Problem(f"mbb2d_{nx}x{ny}", m, mask, f)


def cantilever2d(nx: int = 600, ny: int = 200, **mat) -> Problem:
    """Cantilever: left edge clamped, unit downward load at the right mid-edge node."""
    m = Mesh((nx, ny), **mat)
    mask = np.zeros(m.n_dofs, np.uint8)
    for j in range(ny + 1):
        for c in range(2):
            mask[m.dof(c, m.node(0, j))] = 1
    f = np.zeros(m.n_dofs)
    f[m.dof(1, m.node(nx, ny // 2))] = -1.0
    return Problem(f"cantilever2d_{nx}x{ny}", m, mask, f)


def cantilever3d(nx: int = 96, ny: int = 48, nz: int = 48, **mat) -> Problem:
    """3D cantilever: x=0 face clamped; unit total downward (-z) line load on the
    bottom edge (x=nx, z=0) of the free end, with consistent edge weights."""
    m = Mesh((nx, ny, nz), **mat)
    mask = np.zeros(m.n_dofs, np.uint8)
    jj, kk = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    face = m.node(0, jj.ravel(), kk.ravel())
    for c in range(3):
        mask[m.dof(c, face)] = 1
    f = np.zeros(m.n_dofs)
    w = _edge_weights(ny)
    nodes = m.node(nx, np.arange(ny + 1), 0)
    f[m.dof(2, nodes)] = -w
    return Problem(f"cantilever3d_{nx}x{ny}x{nz}", m, mask, f)


def bridge3d(nx: int = 192, ny: int = 96, nz: int = 96, **mat) -> Problem:
    """Quarter of an MBB-style bridge (y vertical): symmetry planes u_x=0 on x=0 and
    u_z=0 on z=0, a point support u_y=0 at the bottom corner node (nx, 0, nz), and a
    unit total downward (-y) pressure on the top face y=ny with consistent weights."""
    m = Mesh((nx, ny, nz), **mat)
    mask = np.zeros(m.n_dofs, np.uint8)
    jj, kk = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    mask[m.dof(0, m.node(0, jj.ravel(), kk.ravel()))] = 1
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    mask[m.dof(2, m.node(ii.ravel(), jj.ravel(), 0))] = 1
    mask[m.dof(1, m.node(nx, 0, nz))] = 1
    f = np.zeros(m.n_dofs)
    ii, kk = np.meshgrid(np.arange(nx + 1), np.arange(nz + 1), indexing="ij")
    w = _face_weights(nx, nz)
    f[m.dof(1, m.node(ii.ravel(), ny, kk.ravel()))] = -w.ravel()
    return Problem(f"bridge3d_{nx}x{ny}x{nz}", m, mask, f)


# Problems of the paper's numerical experiments (Sec. 5), used for soft pins only.
# Geometry figures: MBB on [0,3]x[0,1], rollers along x=0 and at (3,0), load at the
# top-left corner; cantilever on [0,40]x[0,25] clamped at x=0 with the load at
# mid-height of x=40; simply supported beam on [0,30]x[0,15], pin at (0,0), roller
# at (30,0), load at the bottom mid-span.  Each point load is a unit-intensity
# distributed load over a short segment (0.3, 3 and 3 long).

def _segment_load(m: Mesh, f, comp, nodes_along, x0, x1, hseg, q):
    """Consistent nodal load of intensity q on the segment [x0,x1] of a boundary line
    whose nodes sit at coordinates i*hseg (i = 0..len(nodes_along)-1)."""
    n = len(nodes_along)
    xs = np.arange(n) * hseg
    for i in range(n - 1):
        a, b = xs[i], xs[i + 1]
        lo, hi = max(a, x0), min(b, x1)
        if hi <= lo + 1e-14:
            continue
        # integrate the two linear shape functions over [lo, hi]
        def shape_int(s0, s1, node_left):
            # int of (b - x)/h (left) or (x - a)/h (right) over [s0, s1]
            if node_left:
                return ((b - s0) ** 2 - (b - s1) ** 2) / (2 * hseg)
            return ((s1 - a) ** 2 - (s0 - a) ** 2) / (2 * hseg)
        f[m.dof(comp, nodes_along[i])] += q * shape_int(lo, hi, True)
        f[m.dof(comp, nodes_along[i + 1])] += q * shape_int(lo, hi, False)


def paper_mbb(nx: int = 180, ny: int = 60) -> Problem:
    m = Mesh((nx, ny), h=(3.0 / nx, 1.0 / ny), Emin=1e-3)
    mask = np.zeros(m.n_dofs, np.uint8)
    for j in range(ny + 1):
        mask[m.dof(0, m.node(0, j))] = 1
    mask[m.dof(1, m.node(nx, 0))] = 1
    f = np.zeros(m.n_dofs)
    top = [m.node(i, ny) for i in range(nx + 1)]
    _segment_load(m, f, 1, top, 0.0, 0.3, 3.0 / nx, -1.0)
    return Problem("paper_mbb", m, mask, f)


def paper_cantilever(nx: int = 160, ny: int = 100) -> Problem:
    m = Mesh((nx, ny), h=(40.0 / nx, 25.0 / ny), Emin=1e-3)
    mask = np.zeros(m.n_dofs, np.uint8)
    for j in range(ny + 1):
        for c in range(2):
            mask[m.dof(c, m.node(0, j))] = 1
    f = np.zeros(m.n_dofs)
    right = [m.node(nx, j) for j in range(ny + 1)]
    _segment_load(m, f, 1, right, 11.0, 14.0, 25.0 / ny, -1.0)
    return Problem("paper_cantilever", m, mask, f)


def paper_ssbeam(nx: int = 180, ny: int = 90) -> Problem:
    m = Mesh((nx, ny), h=(30.0 / nx, 15.0 / ny), Emin=1e-3)
    mask = np.zeros(m.n_dofs, np.uint8)
    mask[m.dof(0, m.node(0, 0))] = 1
    mask[m.dof(1, m.node(0, 0))] = 1
    mask[m.dof(1, m.node(nx, 0))] = 1
    f = np.zeros(m.n_dofs)
    bottom = [m.node(i, 0) for i in range(nx + 1)]
    _segment_load(m, f, 1, bottom, 13.5, 16.5, 30.0 / nx, -1.0)
    return Problem("paper_ssbeam", m, mask, f)


# ---------------------------------------------------------------------------------
# Density fields and bases
# ---------------------------------------------------------------------------------

def rho_jitter(mesh: Mesh, seed: int, center=0.5, half=0.2, lo=0.01, hi=1.0):
    """rho = center + U(-half, half), clipped to [lo, hi]; element-lexicographic."""
    rng = np.random.default_rng(seed)
    r = center + rng.uniform(-half, half, mesh.n_elems)
    return np.clip(r, lo, hi)


def rho_smoothed(mesh: Mesh, seed: int, sigma=3.0, lo=0.05, hi=1.0):
    """Per-element U(0,1), Gaussian-smoothed (sigma in elements, reflecting edges,
    truncated at 4 sigma), then affinely mapped onto [lo, hi]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    shape = tuple(reversed(mesh.nel))  # C-order array with x fastest in memory
    u = rng.uniform(0.0, 1.0, shape)
    s = gaussian_filter(u, sigma=sigma, mode="reflect", truncate=4.0)
    a, b = s.min(), s.max()
    s = (s - a) / (b - a) if b > a else np.zeros_like(s)
    return (lo + (hi - lo) * s).ravel()


def trust_region_fields(mesh: Mesh, centre: np.ndarray, count: int, seed: int, step: float = 0.1,
                        lo: float = 0.05, hi: float = 1.0) -> np.ndarray:
    """count densities around a centre design, as the trust-region iterates that a ROM is
    evaluated on: rho_b = clip(centre + step (2 s_b - 1), lo, hi) with s_b a seeded
    smoothed field in [0, 1] (rho_smoothed's recipe).  Returns [count][n_elems]."""
    out = np.empty((count, mesh.n_elems))
    for b in range(count):
        s = rho_smoothed(mesh, seed + b, lo=0.0, hi=1.0)
        out[b] = np.clip(centre + step * (2.0 * s - 1.0), lo, hi)
    return out


def path_fields(mesh: Mesh, centre: np.ndarray, ts, seed: int, amp: float = 0.1, lo: float = 0.05,
                hi: float = 1.0) -> np.ndarray:
    """Densities on a smooth design path through a trust-region centre, as an optimiser
    visits them: rho(t) = clip(centre + amp (t d1 + t^2 d2 / 2), lo, hi) with d1, d2
    seeded smoothed fields in [-1, 1] (rho_smoothed's recipe).  Negative t are the
    earlier centres (the snapshot window of the basis), small positive t the candidate
    designs of the current trust-region subproblem.  Returns [len(ts)][n_elems]."""
    d1 = 2.0 * rho_smoothed(mesh, seed, lo=0.0, hi=1.0) - 1.0
    d2 = 2.0 * rho_smoothed(mesh, seed + 1, lo=0.0, hi=1.0) - 1.0
    out = np.empty((len(ts), mesh.n_elems))
    for b, t in enumerate(ts):
        out[b] = np.clip(centre + amp * (t * d1 + 0.5 * t * t * d2), lo, hi)
    return out


def rho_batch(mesh: Mesh, base_seed: int, count: int, kind="smoothed"):
    fn = rho_smoothed if kind == "smoothed" else rho_jitter
    return np.stack([fn(mesh, base_seed + i) for i in range(count)])


def cosine_basis(mesh: Mesh, mask: np.ndarray, k: int, seed: int, dtype=np.float32):
    """k smooth, linearly independent nodal fields: products of low-order cosines with
    seeded distinct wave numbers and phases, one displacement component each, zero on
    Dirichlet DOFs.  Row-major [n_dofs][k]."""
    rng = np.random.default_rng(seed)
    d = mesh.dim
    nn = mesh.nn
    L = np.array(mesh.nel, dtype=np.float64)
    # columns are built one contiguous row of phi^T at a time (in float64, then stored
    # in dtype), the node value being the product of per-axis cosine factors
    phit = np.zeros((k, mesh.n_dofs), dtype=dtype)
    fixed = mask.astype(bool)
    used = set()
    maxw = 1
    col = 0
    while col < k:
        c = int(rng.integers(0, d))
        wav = tuple(int(x) for x in rng.integers(0, maxw + 1, d))
        if (c,) + wav in used:
            maxw += 1
            continue
        used.add((c,) + wav)
        ph = rng.uniform(0, np.pi, d)
        vals = None
        for a in range(d):  # x fastest: ((f_x f_y) f_z), the product taken axis by axis
            fa = np.cos(np.pi * wav[a] * np.arange(nn[a], dtype=np.float64) / L[a] + ph[a])
            vals = fa if vals is None else np.multiply.outer(fa, vals).ravel()
        rowv = phit[col]
        rowv[c * mesh.n_nodes:(c + 1) * mesh.n_nodes] = vals
        rowv[fixed] = 0
        col += 1
    return np.ascontiguousarray(phit.T)


def snapshot_fields(mesh: Mesh, mask: np.ndarray, count: int, seed: int, decay: float = 0.5,
                    rank: int = 0) -> np.ndarray:
    """count smooth displacement-like snapshots with a geometric spread of singular
    values: u_i = c_0 + sum_{j=1..r-1} a_ij decay^j c_j with c_j the fields of
    cosine_basis, a_ij ~ N(0, 1) seeded, r = rank or count + 1.  Zero on Dirichlet DOFs.
    Returns [count][n_dofs] float64 (one contiguous snapshot per row)."""
    r = rank if rank > 0 else count + 1
    C = cosine_basis(mesh, mask, r, seed, np.float64)
    rng = np.random.default_rng(seed + 1)
    A = rng.standard_normal((count, r)) * decay ** np.arange(r)
    A[:, 0] = 1.0
    return np.ascontiguousarray(A @ C.T)


def orthonormalize(cols: np.ndarray, mask: np.ndarray, dtype=np.float64):
    """Orthonormal basis (Householder QR in float64) of the given columns after zeroing
    Dirichlet rows; returned in ``dtype``."""
    a = np.array(cols, dtype=np.float64, copy=True)
    a[mask.astype(bool), :] = 0.0
    q, _ = np.linalg.qr(a)
    return q.astype(dtype)


def orthonormalize_tall(cols: np.ndarray, mask: np.ndarray, dtype=np.float64, passes: int = 2):
    """Orthonormal basis of tall columns (rows >> columns) by Cholesky QR repeated
    `passes` times in float64 (Gram matrix, its Cholesky factor, a triangular solve):
    the same span as orthonormalize, an order of magnitude faster for millions of rows
    (the Gram matrix of well-conditioned columns loses nothing in the second pass)."""
    import scipy.linalg as sla
    a = np.array(cols, dtype=np.float64, copy=True)
    a[mask.astype(bool), :] = 0.0
    for _ in range(passes):
        L = np.linalg.cholesky(a.T @ a)
        a = np.ascontiguousarray(sla.solve_triangular(L, a.T, lower=True).T)
    return a.astype(dtype)


# ---------------------------------------------------------------------------------
# Request stream of the serving workload
# ---------------------------------------------------------------------------------

SERVING_MESHES = ("mbb2d_60x20", "cantilever2d_600x200", "cantilever3d_48x24x24",
                  "cantilever3d_96x48x48")


@dataclass
class ServingRequest:
    mesh: int     # index into SERVING_MESHES
    kind: str     # "rom" or "hdm"
    k: int        # ROM basis size (0 for HDM)
    rho_id: int   # index into the per-mesh pool of density fields


def serving_stream(n: int = 512, seed: int = 5150, rom_frac: float = 0.8, kmin: int = 8,
                   kmax: int = 128, rho_pool: int = 8):
    """Seeded request mix: mesh uniform over SERVING_MESHES, ROM with probability
    rom_frac (k uniform in [kmin, kmax]), else HDM; densities drawn from a pool of
    rho_pool smoothed fields per mesh."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        mesh = int(rng.integers(0, len(SERVING_MESHES)))
        rom = bool(rng.random() < rom_frac)
        k = int(rng.integers(kmin, kmax + 1)) if rom else 0
        out.append(ServingRequest(mesh, "rom" if rom else "hdm", k, int(rng.integers(0, rho_pool))))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 5151):
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


# ---------------------------------------------------------------------------------
# Named configurations of the benchmark suite
# ---------------------------------------------------------------------------------

CONFIG_NAMES = ("mbb2d_60x20", "cantilever2d_600x200", "cantilever3d_96x48x48",
                "bridge3d_192x96x96", "cantilever3d_48x24x24")


@dataclass
class Config:
    name: str
    problem: Problem
    rho_kind: str
    rho_seed0: int
    k: int
    batch: int
    rtol: float
    basis_seed: int
    extra: dict = field(default_factory=dict)

    def rho(self, i: int = 0):
        m = self.problem.mesh
        if self.rho_kind == "jitter":
            return rho_jitter(m, self.rho_seed0 + i)
        return rho_smoothed(m, self.rho_seed0 + i)

    def rhos(self, count=None):
        return np.stack([self.rho(i) for i in range(count or self.batch)])


def config(name: str, scale: int = 1) -> Config:
    """One of the named workloads.  ``scale`` > 1 divides every axis (a reduced copy
    with the same boundary conditions, for quick tests)."""
    s = scale
    if name == "mbb2d_60x20":
        return Config(name, mbb2d(60 // s, 20 // s), "jitter", 1000, 8, 1, 1e-10, 2000)
    if name == "cantilever2d_600x200":
        return Config(name, cantilever2d(600 // s, 200 // s), "smoothed", 2000, 32, 1, 1e-10, 4000)
    if name == "cantilever3d_96x48x48":
        return Config(name, cantilever3d(96 // s, 48 // s, 48 // s), "smoothed", 3000, 100, 1, 1e-10, 6000)
    if name == "bridge3d_192x96x96":
        return Config(name, bridge3d(192 // s, 96 // s, 96 // s), "smoothed", 4000, 200, 16, 1e-8, 8000)
    if name == "cantilever3d_48x24x24":
        return Config(name, cantilever3d(48 // s, 24 // s, 24 // s), "smoothed", 5000, 128, 1, 1e-8, 10000)
    raise KeyError(name)
