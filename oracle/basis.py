"""Reduced-basis construction of the oracle: POD of a snapshot window, one Gram-Schmidt
step of the new snapshot against it, and the limited-memory window of the L most
recent snapshots (Sec. 4.2, basis construction at a trust-region centre, the remark
on compliance output, and the remark on retaining only the L most recent centres).
FP64.

POD_n(U) is taken straight from its definition: the n leading left singular vectors of
U, from a LAPACK SVD of the whole snapshot matrix.  The Gram-Schmidt step is the
classical one, written out.  Readings where the paper is silent:

* a POD direction whose singular value is at most ``rtol`` times the largest is not
  kept (it is not determined by the data);
* the new snapshot adds no column when what is left of it after the step has norm at
  most ``rtol`` times its own (it already lies in the span);
* n_k = min(m, n_max) for a window of m snapshots, before the rule above.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from collections import deque

import numpy as np


def pod(U, n):
    """POD_n(U): the n leading left singular vectors of the snapshot matrix U
    (columns = snapshots) and all its singular values, descending (Sec. 4.2)."""
    U = np.asarray(U, dtype=np.float64)
    W, s, _ = np.linalg.svd(U, full_matrices=False)
    return W[:, :n], s


def gram_schmidt_step(Phi, u):
    """One classical Gram-Schmidt step of u against the orthonormal columns of Phi:
    c = Phi^T u, v = u - Phi c.  Returns (v / ||v||, ||v||, c) (Sec. 4.2, remark on
    compliance output: one step suffices because the POD columns are orthonormal)."""
    u = np.asarray(u, dtype=np.float64)
    Phi = np.asarray(Phi, dtype=np.float64).reshape(u.shape[0], -1)
    c = Phi.T @ u
    v = u - Phi @ c
    nv = float(np.linalg.norm(v))
    q = v / nv if nv > 0 else v
    return q, nv, c


def basis_update(U, u_new, n_max, rtol=1e-7):
    """Phi = GramSchmidt([POD_{n_k}(U), u_new]) with n_k = min(m, n_max) for the m
    snapshots of the window U (Sec. 4.2, basis for compliance output; n_k rule of the
    practical-details paragraph).  U may have zero columns (first centre); u_new may be
    None (POD only).  Returns (Phi [N][j], n, keep_new, sigma)."""
    U = np.asarray(U, dtype=np.float64)
    N = U.shape[0] if U.ndim == 2 else np.asarray(u_new).shape[0]
    m = U.shape[1] if U.ndim == 2 else 0
    sigma = np.zeros(0)
    Pod = np.zeros((N, 0))
    if m > 0:
        W, sigma = pod(U, min(m, n_max))
        keep = [i for i in range(W.shape[1]) if sigma[i] > rtol * sigma[0]]
        Pod = W[:, keep]
    n = Pod.shape[1]
    if u_new is None:
        return Pod, n, False, sigma
    q, nv, _ = gram_schmidt_step(Pod, u_new)
    keep_new = nv > rtol * float(np.linalg.norm(u_new))
    Phi = np.concatenate([Pod, q[:, None]], axis=1) if keep_new else Pod
    return Phi, n, keep_new, sigma


class SnapshotWindow:
    """The L most recent snapshots, oldest first (Sec. 4.2, remark on retaining only
    the L most recent trust-region centres: once L are held, a new snapshot replaces
    the oldest)."""

    def __init__(self, L):
        self.L = int(L)
        self.cols = deque(maxlen=self.L)

    def push(self, u):
        self.cols.append(np.array(u, dtype=np.float64, copy=True))

    def matrix(self, N=None):
        if not self.cols:
            return np.zeros((N or 0, 0))
        return np.stack(list(self.cols), axis=1)

    def __len__(self):
        return len(self.cols)
