"""Per-row weight selection, PML profiles and explicit CSR assembly (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What is assembled (Sec. 2.1, the matrix form [M + S] p = s):

* stiffness  S = w_s1 S_1 + w_s2 <S_2> + w_s3 <S_3>, each weight taken per row
  (the adaptive "GA" stencil of Sec. 3.1 picks a row's weights by its local G);
  <S_2> is the average of the three stencils rotated 45 degrees about an axis,
  <S_3> the average of the four cube-diagonal stencils.  In a homogeneous,
  unstretched medium their plane-wave symbols are the ones inside the square
  root of the phase-velocity equation of Sec. 2.2; written with the 1D
  second-difference T_a along each axis those symbols are exactly

      S_1   = sum_a T_a
      <S_2> = sum_a T_a + (h^2/6) sum_{a<b} T_a T_b
      <S_3> = sum_a T_a + (h^2/2) sum_{a<b} T_a T_b + (3 h^4/8) T_x T_y T_z

  (a 27-point stencil with cubic symmetry is fixed by its symbol, so these
  are the paper's interior stencils, not an approximation of them);
* consistent mass, second form of Sec. 2.1 (bulk modulus at the collocation
  point): k_i^2 [w_m0 p_0 + w_m1 sum_6 p + w_m2 sum_12 p + w_m3 sum_8 p] with
  per-point mass weights (see ``table``);
* PML by complex coordinate stretching d/dx -> (1/xi) d/dx (Sec. 2.1).

Readings:

* G = c / (f h); a row takes the table entry nearest its G, ties going up:
  idx = clamp(floor((G - gmin)/dG + 1/2), 0, N_G - 1), every step in IEEE
  binary64 with no fused multiply-add; rows outside the table are clamped and
  counted.
* PML profile (the paper defers it to earlier work): on each face a layer of
  npml nodes of width L = npml h, gamma(d) = gamma_max (1 - cos(pi d / (2L)))
  at distance d into the layer, gamma_max = c_ref ln(1/R) / (2 L (1 - 2/pi)),
  xi = 1 + i gamma / omega, evaluated at nodes and half nodes (the same formula
  beyond the last node); R = 1e-3; c_ref = the largest velocity of the model.
* The stretched operator is written in the symmetric form obtained after
  multiplying the equation by Xi = xi_x xi_y xi_z: every 1D factor is
  stretched,
      T_a[i, i+-1] = 1 / (h^2 xi_a(i +- 1/2)),  T_a[i, i] = -(T_a[i,i-1] + T_a[i,i+1]),
      U_a[i, i+-1] = xi_a(i +- 1/2) / 2,         X_a = diag(xi_a(i)),
  an axis absent from a product contributes X_a, and the mass classes are
  M_0 = X X X, M_1 = 2 sum U X X, M_2 = 4 sum U U X, M_3 = 8 U U U.
  In the interior (xi = 1) this is exactly the paper's stencil; the right-hand
  side is multiplied by Xi, which is 1 wherever a source may sit.
* Dirichlet: neighbours outside the grid are dropped.
* Grid order: x fastest, lin = i + nx (j + ny k); CSR columns ascending.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "select_index", "pml_profile", "row_weights", "assemble", "assemble_csr",
    "stencil_offsets",
]


def select_index(c, f, h, gmin, dg, n_g, spacing="G"):
    """Table index of every grid point (Sec. 3.1: each row gets the weights of
    its local wavelength): the nearest table abscissa, ties upward, clamped to
    the table.  spacing "G": the abscissa is G = c/(f h); "invG": it is
    s = 1/G = (f h)/c.  ``c`` is widened to binary64 exactly; every step is
    one binary64 operation.  Returns (idx int64 array, number of clamped
    points)."""
    c = np.asarray(c, dtype=np.float32).astype(np.float64)
    fh = np.float64(f) * np.float64(h)
    v = c / fh if spacing == "G" else fh / c
    t = (v - np.float64(gmin)) / np.float64(dg)
    raw = np.floor(t + 0.5)
    idx = np.clip(raw, 0, n_g - 1).astype(np.int64)
    n_clamped = int(np.count_nonzero((raw < 0) | (raw > n_g - 1)))
    return idx, n_clamped


def pml_profile(n, npml, h, omega, c_ref, R=1e-3):
    """Stretching factors xi along one axis (Sec. 2.1, xi = 1 + i gamma/omega).

    Returns (xi_node[n], xi_half[n+1]) where xi_half[k] is taken at the half
    node (k - 1/2) h, so node i sits between xi_half[i] and xi_half[i+1]."""
    xn = np.arange(n, dtype=np.float64) * h
    xh = (np.arange(n + 1, dtype=np.float64) - 0.5) * h
    if npml <= 0:
        return np.ones(n, complex), np.ones(n + 1, complex)
    L = npml * h
    left = npml * h
    right = (n - 1 - npml) * h
    gmax = c_ref * math.log(1.0 / R) / (2.0 * L * (1.0 - 2.0 / math.pi))

    def xi(x):
        d = np.maximum(np.maximum(left - x, x - right), 0.0)
        gamma = gmax * (1.0 - np.cos(np.pi * d / (2.0 * L)))
        return 1.0 + 1j * gamma / omega

    return xi(xn), xi(xh)


def row_weights(mode, idx=None, table_w=None, fixed_w=None, dims=None):
    """Seven weights per row, (N, 7) in the order (w_s1, w_s2, w_s3, w_m0,
    w_m1, w_m2, w_m3).

    mode "GA"    : the table entry of the row's own G (Sec. 3.1);
    mode "GAm"   : the mean of the table entries of the row's stencil points
                   that lie inside the grid (Sec. 3.1, second adaptive variant);
    mode "fixed" : the same weights on every row ("G4" / "Gm", Sec. 3.1).
    ``table_w`` is (N_G, 7); ``fixed_w`` is (7,)."""
    if mode == "fixed":
        n = int(np.prod(dims))
        return np.broadcast_to(np.asarray(fixed_w, np.float64), (n, 7)).copy()
    per_point = np.asarray(table_w, np.float64)[np.asarray(idx).ravel()]
    if mode == "GA":
        return per_point
    if mode == "GAm":
        nx, ny, nz = dims
        wp = per_point.reshape(nz, ny, nx, 7)
        acc = np.zeros_like(wp)
        cnt = np.zeros((nz, ny, nx, 1))
        shape = (nz, ny, nx)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    # rows p whose neighbour p + d lies in the grid
                    rows = tuple(slice(max(0, -d), n - max(0, d)) for d, n in zip((dz, dy, dx), shape))
                    nbrs = tuple(slice(max(0, d), n - max(0, -d)) for d, n in zip((dz, dy, dx), shape))
                    acc[rows] += wp[nbrs]
                    cnt[rows] += 1.0
        return (acc / cnt).reshape(-1, 7)
    raise ValueError(mode)


def _1d_factors(xi_node, xi_half, h):
    """1D matrices T (stretched second difference, includes 1/h^2), U
    (stretched neighbour average) and X = diag(xi) along one axis."""
    n = len(xi_node)
    inv = 1.0 / xi_half  # 1/xi at half nodes k - 1/2, k = 0..n
    lower = inv[1:n]       # entry (i, i-1) = 1/xi(i - 1/2) for i = 1..n-1
    diag = -(inv[0:n] + inv[1:n + 1])
    T = sp.diags([lower, diag, lower], [-1, 0, 1], shape=(n, n), format="csr") / (h * h)
    uo = 0.5 * xi_half[1:n]
    U = sp.diags([uo, uo], [-1, 1], shape=(n, n), format="csr")
    X = sp.diags([xi_node], [0], shape=(n, n), format="csr")
    return T, U, X


def _k3(fz, fy, fx):
    """3D operator from 1D factors, x fastest: kron(Z, kron(Y, X))."""
    return sp.kron(fz, sp.kron(fy, fx, format="csr"), format="csr")


def complex_velocity(c, Q=None):
    """Velocity with constant-Q attenuation (the paper's medium parameters
    allow a complex bulk modulus): c (1 - i/(2Q)) for the exp(-i omega t)
    convention, so that k = omega / c~ has a positive imaginary part and
    outgoing waves decay; c itself without attenuation (Q None or inf)."""
    c = np.asarray(c, dtype=np.float64)
    if Q is None or not np.isfinite(Q):
        return c
    return c * (1.0 - 0.5j / Q)


def assemble(c, f, h, npml, w_rows, omega=None, c_ref=None, R=1e-3, mass_form="b",
             shift=0.0, Q=None):
    """Assemble A = M + S (Sec. 2.1) as a scipy sparse matrix (values only;
    use ``assemble_csr`` for the full 27-entry pattern).

    c        : velocity [nz, ny, nx] (float32 values, widened exactly)
    w_rows   : (N, 7) per-row weights from ``row_weights``
    npml     : layer width in nodes, int or (npml_x, npml_y, npml_z)
    mass_form: "b" = bulk modulus at the collocation point (default);
               "a" = each mass term uses its own point's bulk modulus
               (first consistent-mass form of Sec. 2.1)
    shift    : k^2 -> (1 + i shift) k^2 in the mass (complex-shifted operator
               used by the multigrid preconditioner; 0 for the physical one)
    Q        : constant quality factor: k^2 = (omega / c~)^2 with the complex
               velocity c~ = c (1 - i/(2Q)) (None: no attenuation); the table
               index and the PML use the real c
    """
    c = np.asarray(c, dtype=np.float32).astype(np.float64)
    nz, ny, nx = c.shape
    if omega is None:
        omega = 2.0 * math.pi * f
    if c_ref is None:
        c_ref = float(c.max())
    if np.isscalar(npml):
        npml = (int(npml),) * 3
    fac = []
    for n, p in zip((nx, ny, nz), npml):
        xn, xh = pml_profile(n, p, h, omega, c_ref, R)
        fac.append(_1d_factors(xn, xh, h))
    (Tx, Ux, Xx), (Ty, Uy, Xy), (Tz, Uz, Xz) = fac

    S1 = _k3(Xz, Xy, Tx) + _k3(Xz, Ty, Xx) + _k3(Tz, Xy, Xx)
    P2 = _k3(Xz, Ty, Tx) + _k3(Tz, Xy, Tx) + _k3(Tz, Ty, Xx)      # sum_{a<b} T_a T_b
    P3 = _k3(Tz, Ty, Tx)                                            # T_x T_y T_z
    S2 = S1 + (h * h / 6.0) * P2
    S3 = S1 + (h * h / 2.0) * P2 + (3.0 * h ** 4 / 8.0) * P3
    M0 = _k3(Xz, Xy, Xx)
    M1 = 2.0 * (_k3(Xz, Xy, Ux) + _k3(Xz, Uy, Xx) + _k3(Uz, Xy, Xx))
    M2 = 4.0 * (_k3(Xz, Uy, Ux) + _k3(Uz, Xy, Ux) + _k3(Uz, Uy, Xx))
    M3 = 8.0 * _k3(Uz, Uy, Ux)

    w = np.asarray(w_rows, np.float64)
    k2 = (omega / complex_velocity(c.ravel(), Q)) ** 2 * (1.0 + 1j * shift)
    D = lambda v: sp.diags([v], [0], format="csr")  # noqa: E731
    A = D(w[:, 0]) @ S1 + D(w[:, 1]) @ S2 + D(w[:, 2]) @ S3
    if mass_form == "b":
        A = A + D(k2) @ (D(w[:, 3]) @ M0 + D(w[:, 4]) @ M1 + D(w[:, 5]) @ M2 + D(w[:, 6]) @ M3)
    elif mass_form == "a":
        K = D(k2)
        A = A + (D(w[:, 3]) @ M0 + D(w[:, 4]) @ M1 + D(w[:, 5]) @ M2 + D(w[:, 6]) @ M3) @ K
    else:
        raise ValueError(mass_form)
    return A.tocsr()


def stencil_offsets():
    """The 27 offsets (dz, dy, dx) in ascending column order."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def assemble_csr(c, f, h, npml, w_rows, **kw):
    """CSR of A with the full 27-point pattern: every in-grid neighbour is an
    explicit entry (even if its value happens to be zero), rows in grid order,
    columns ascending.  Returns (indptr int64, indices int64, data complex128,
    shape)."""
    A = assemble(c, f, h, npml, w_rows, **kw)
    nz, ny, nx = np.asarray(c).shape
    N = nx * ny * nz
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    cols = np.full((N, 27), -1, dtype=np.int64)
    vals = np.zeros((N, 27), dtype=np.complex128)
    for s, (dz, dy, dx) in enumerate(stencil_offsets()):
        ok = ((ii + dx >= 0) & (ii + dx < nx) & (jj + dy >= 0) & (jj + dy < ny)
              & (kk + dz >= 0) & (kk + dz < nz))
        off = dx + nx * (dy + ny * dz)
        rows = np.nonzero(ok)[0]
        cols[rows, s] = rows + off
        if off >= 0:
            dvals = A.diagonal(off)          # entries (r, r + off), r = 0..N-off-1
            vals[rows, s] = dvals[rows]
        else:
            dvals = A.diagonal(off)          # entries (r - off... ) indexed by column
            vals[rows, s] = dvals[rows + off]
    mask = cols >= 0
    indptr = np.concatenate([[0], np.cumsum(mask.sum(axis=1))]).astype(np.int64)
    return indptr, cols[mask], vals[mask], (N, N)


def csr_matrix(indptr, indices, data, shape):
    return sp.csr_matrix((data, indices, indptr), shape=shape)


def _row_vec(M, r):
    """Row r of a sparse matrix as a 1 x n CSR matrix."""
    return sp.csr_matrix(M.getrow(r))


def assemble_rows(c, f, h, npml, w_rows, rows, omega=None, c_ref=None, R=1e-3, shift=0.0, Q=None):
    """Selected rows of the same A as ``assemble`` (second mass form), for
    grids too large to assemble whole: row (i, j, k) of a Kronecker product
    kron(Z, kron(Y, X)) is kron(Z[k], kron(Y[j], X[i])), so each row is the
    weighted sum of the Kronecker products of the 1D factors' rows.
    ``w_rows`` are the weights of the selected rows, (len(rows), 7).
    Returns a len(rows) x N CSR matrix."""
    c = np.asarray(c, dtype=np.float32)
    nz, ny, nx = c.shape
    if omega is None:
        omega = 2.0 * math.pi * f
    if c_ref is None:
        c_ref = float(c.astype(np.float64).max())
    if np.isscalar(npml):
        npml = (int(npml),) * 3
    fac = []
    for n, p in zip((nx, ny, nz), npml):
        xn, xh = pml_profile(n, p, h, omega, c_ref, R)
        fac.append(_1d_factors(xn, xh, h))
    (Tx, Ux, Xx), (Ty, Uy, Xy), (Tz, Uz, Xz) = fac
    out = []
    cflat = c.reshape(-1).astype(np.float64)
    for r, w in zip(rows, np.asarray(w_rows, np.float64)):
        i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
        tx, ux, xx = _row_vec(Tx, i), _row_vec(Ux, i), _row_vec(Xx, i)
        ty, uy, xy = _row_vec(Ty, j), _row_vec(Uy, j), _row_vec(Xy, j)
        tz, uz, xz = _row_vec(Tz, k), _row_vec(Uz, k), _row_vec(Xz, k)
        s1 = _k3(xz, xy, tx) + _k3(xz, ty, xx) + _k3(tz, xy, xx)
        p2 = _k3(xz, ty, tx) + _k3(tz, xy, tx) + _k3(tz, ty, xx)
        p3 = _k3(tz, ty, tx)
        s2 = s1 + (h * h / 6.0) * p2
        s3 = s1 + (h * h / 2.0) * p2 + (3.0 * h ** 4 / 8.0) * p3
        m0 = _k3(xz, xy, xx)
        m1 = 2.0 * (_k3(xz, xy, ux) + _k3(xz, uy, xx) + _k3(uz, xy, xx))
        m2 = 4.0 * (_k3(xz, uy, ux) + _k3(uz, xy, ux) + _k3(uz, uy, xx))
        m3 = 8.0 * _k3(uz, uy, ux)
        k2 = (omega / complex_velocity(cflat[r], Q)) ** 2 * (1.0 + 1j * shift)
        row = (w[0] * s1 + w[1] * s2 + w[2] * s3
               + k2 * (w[3] * m0 + w[4] * m1 + w[5] * m2 + w[6] * m3))
        out.append(row)
    return sp.vstack(out).tocsr()
