"""Pins of the oracle's right-hand side and direct solve (CPU only)."""
import math

import numpy as np
import pytest
from scipy.fft import dstn, idstn

from oracle import analytic as An
from oracle import operator as O
from oracle import solve as S
from oracle import table as T
import synth


@pytest.fixture(scope="module")
def w7_table():
    Gs, W = T.build_table()
    return Gs, T.complete_weights(W)


def _ga(c, f, h, npml, Gs, W7, **kw):
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    return O.assemble(c, f, h, npml, O.row_weights("GA", idx, W7), **kw), idx


def test_dense_equals_superlu(w7_table):
    """Brute-force dense solve equals the sparse direct solve."""
    Gs, W7 = w7_table
    dims = (12, 11, 10)
    c = synth.gradient_z(dims, 25.0)
    A, _ = _ga(c, 5.0, 25.0, 3, Gs, W7)
    b = S.point_source_rhs(dims, 25.0, [(5, 5, 4), (6, 4, 5)])
    ud = np.linalg.solve(A.toarray(), b)
    import scipy.sparse.linalg as spla
    us = spla.splu(A.tocsc()).solve(b)
    assert np.linalg.norm(ud - us) / np.linalg.norm(ud) < 1e-11
    assert np.all(S.relative_residual(A, ud, b) < 1e-12)


def test_dst_solve_uniform_shifted(w7_table):
    """Uniform weights, no PML, complex-shifted k^2 (off resonance): the solve
    equals the DST-I spectral solve u = DST^-1(DST(b) / lambda)."""
    Gs, W7 = w7_table
    dims = (9, 8, 7)
    nx, ny, nz = dims
    h, f = 20.0, 10.0
    c = synth.homogeneous(dims, 2000.0)
    A, idx = _ga(c, f, h, 0, Gs, W7, shift=0.5)
    b = synth.random_vectors(nx * ny * nz, 1, 6)[0]
    u = S.solve(A, b[:, None])[:, 0]
    mz, my, mx = np.meshgrid(np.arange(1, nz + 1) * np.pi / (nz + 1),
                             np.arange(1, ny + 1) * np.pi / (ny + 1),
                             np.arange(1, nx + 1) * np.pi / (nx + 1), indexing="ij")
    w = W7[idx.ravel()[0]]
    k = 2 * math.pi * f / 2000.0
    q = np.stack([mx, my, mz], -1) / h
    # symbol with k^2 -> (1 + 0.5 i) k^2 in the mass term
    lam = An.symbol(q, h, 0.0, w) + (1 + 0.5j) * (An.symbol(q, h, k, w) - An.symbol(q, h, 0.0, w))
    u_ref = idstn(dstn(b.reshape(nz, ny, nx), type=1, norm="ortho") / lam, type=1, norm="ortho").ravel()
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-12


@pytest.mark.slow
def test_homogeneous_greens_function(w7_table):
    """Point source in a homogeneous medium with PML (Sec. 3.2): away from the
    source the solution is alpha * (-exp(i k r) / (4 pi r)), where alpha is the
    residue factor of the discrete symbol at its root (from the paper's
    dispersion analysis).  Without alpha the misfit is alpha - 1 ~ 3.4%."""
    Gs, W7 = w7_table
    n, npml, h, cv, G = 25, 6, 20.0, 2000.0, 10.0
    f = cv / (G * h)
    c = synth.homogeneous((n, n, n), cv)
    A, idx = _ga(c, f, h, npml, Gs, W7)
    s = (n // 2, n // 2, n // 2)
    b = S.point_source_rhs((n, n, n), h, [s])
    u = S.solve(A, b)[:, 0]
    assert S.relative_residual(A, u[:, None], b)[0] < 1e-12
    k = 2 * math.pi * f / cv
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([(ii - s[0]) * h, (jj - s[1]) * h, (kk - s[2]) * h], -1).reshape(-1, 3)
    r = np.linalg.norm(X, axis=1)
    inner = ((ii >= npml) & (ii < n - npml) & (jj >= npml) & (jj < n - npml)
             & (kk >= npml) & (kk < n - npml)).ravel() & (r >= 2 * h)
    alpha, kt = An.amplitude_factor([1, 0, 0], h, k, W7[idx.ravel()[0]])
    assert abs(kt / k - 1) < 1e-5          # adaptive weights: negligible dispersion at G = 10
    g = An.greens(r[inner], k)
    raw = np.linalg.norm(u[inner] - g) / np.linalg.norm(g)
    scaled = np.linalg.norm(u[inner] - alpha * g) / np.linalg.norm(alpha * g)
    assert abs(raw - abs(alpha - 1)) < 0.005
    assert scaled < 3e-3
    # the fitted complex amplitude agrees with the predicted alpha
    fit = np.vdot(g, u[inner]) / np.vdot(g, g)
    assert abs(fit - alpha) < 2e-3


def test_reciprocity_homogeneous(w7_table):
    """Complex-symmetric A (homogeneous, PML): u_s(x_r) = u_r(x_s)."""
    Gs, W7 = w7_table
    dims = (14, 13, 12)
    c = synth.homogeneous(dims, 2000.0)
    A, _ = _ga(c, 8.0, 20.0, 3, Gs, W7)
    s, r = (4, 5, 6), (9, 7, 4)
    b = S.point_source_rhs(dims, 20.0, [s, r])
    u = S.solve(A, b)
    lin = lambda p: p[0] + dims[0] * (p[1] + dims[1] * p[2])  # noqa: E731
    a, bb = u[lin(r), 0], u[lin(s), 1]
    assert abs(a - bb) <= 1e-12 * abs(a)


def test_heterogeneous_is_unsymmetric(w7_table):
    """Adaptive rows in a heterogeneous model give an unsymmetric matrix
    (Sec. 1 calls the system unsymmetric)."""
    Gs, W7 = w7_table
    dims = (8, 8, 8)
    c = synth.gradient_z(dims, 25.0, a=20.0)
    A, _ = _ga(c, 5.0, 25.0, 2, Gs, W7)
    assert abs(A - A.T).max() > 1e-8 * abs(A).max()


def test_point_source_rhs():
    b = S.point_source_rhs((4, 3, 2), 10.0, [(1, 2, 1)], amps=[2.0])
    assert b.shape == (24, 1)
    assert b[1 + 4 * (2 + 3 * 1), 0] == 2.0 / 1000.0
    assert np.count_nonzero(b) == 1
    assert S.in_interior((5, 5, 5), (11, 11, 11), 3)
    assert not S.in_interior((2, 5, 5), (11, 11, 11), 3)
