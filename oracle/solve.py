"""Right-hand side and plain direct solve of the assembled system (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

* The source is a point source on a grid node with a delta signature
  (Sec. 3.1): s = delta(x - x_s), which on the grid is amp / h^3 at the source
  node (the discrete delta integrates to amp).  Sources are not allowed inside
  the PML, where the symmetric form would also scale them by Xi.
* The paper solves the system with a sparse direct (LU) solver (Sec. 3.1).
  Here: dense LAPACK solve for small systems, SuperLU otherwise.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["point_source_rhs", "solve", "relative_residual", "in_interior"]


def in_interior(src, dims, npml):
    """True if the node (i, j, k) lies outside the PML layers."""
    nx, ny, nz = dims
    if np.isscalar(npml):
        npml = (int(npml),) * 3
    i, j, k = src
    return all(p <= q < n - p for q, n, p in ((i, nx, npml[0]), (j, ny, npml[1]), (k, nz, npml[2])))


def point_source_rhs(dims, h, sources, amps=None):
    """Right-hand sides for point sources (Sec. 3.1), one column per source:
    b[:, s] = amp_s / h^3 at node sources[s] = (i, j, k), x fastest."""
    nx, ny, nz = dims
    n = nx * ny * nz
    b = np.zeros((n, len(sources)), dtype=np.complex128)
    for s, (i, j, k) in enumerate(sources):
        amp = 1.0 if amps is None else amps[s]
        b[i + nx * (j + ny * k), s] = amp / h ** 3
    return b


def solve(A, b):
    """Direct solve of A u = b: dense LU for N <= 4096, SuperLU above."""
    A = sp.csr_matrix(A)
    if A.shape[0] <= 4096:
        return np.linalg.solve(A.toarray(), b)
    lu = spla.splu(A.tocsc())
    return lu.solve(np.asarray(b, dtype=np.complex128))


def relative_residual(A, u, b):
    """||b - A u||_2 / ||b||_2 per right-hand side (columns)."""
    u = np.asarray(u)
    b = np.asarray(b)
    r = b - A @ u
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
