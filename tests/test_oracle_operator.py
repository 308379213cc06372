"""Pins of the oracle's index selection, PML and CSR assembly (CPU only)."""
import math

import numpy as np
import pytest
import scipy.ndimage
from scipy.fft import dstn, idstn

from oracle import analytic as An
from oracle import operator as O
from oracle import table as T
import synth


@pytest.fixture(scope="module")
def w7_table():
    Gs, W = T.build_table()
    return Gs, T.complete_weights(W)


def _grid(nx, ny, nz):
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ii.ravel(), jj.ravel(), kk.ravel()


def test_select_index_nearest_entry():
    """Each point gets a table entry nearest its G (Sec. 3.1, picking by local
    wavelength)."""
    rng = np.random.default_rng(3)
    c = rng.uniform(1500, 5000, 20000).astype(np.float32)
    f, h = 5.0, 25.0
    Gs = T.g_grid(3.0, 40.0, 0.05)
    idx, ncl = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    G = c.astype(np.float64) / (f * h)
    assert ncl == 0
    d = np.abs(Gs[idx] - G)
    assert np.all(d <= 0.025 * (1 + 1e-9))
    # no other entry is strictly closer
    alt = np.minimum(np.abs(Gs[np.clip(idx - 1, 0, None)] - G), np.abs(Gs[np.clip(idx + 1, None, len(Gs) - 1)] - G))
    assert np.all(d <= alt + 1e-12)


def test_select_index_ties_up_and_clamps():
    """Exact ties go to the upper entry; out-of-range G is clamped and counted."""
    c = np.array([0.25, 0.75, 0.0, 100.0, 1.0], np.float32)   # G = c with f h = 1
    idx, ncl = O.select_index(c, 1.0, 1.0, 0.0, 0.5, 3)
    assert idx.tolist() == [1, 2, 0, 2, 2]
    assert ncl == 1


def test_interior_rows_act_as_the_paper_symbol(w7_table):
    """Interior rows applied to a plane wave return P(q) times the wave, with P
    from the phase-velocity analysis of Sec. 2.2."""
    Gs, W7 = w7_table
    nx = ny = nz = 9
    h, f = 20.0, 10.0
    c = synth.homogeneous((nx, ny, nz), 2000.0)
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    w = O.row_weights("GA", idx, W7)
    A = O.assemble(c, f, h, 0, w)
    ii, jj, kk = _grid(nx, ny, nz)
    inner = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1) & (kk > 0) & (kk < nz - 1)
    k = 2 * math.pi * f / 2000.0
    for q in ([0.3, 0.2, 0.5], [1.1, -0.4, 2.0], [0.0, 0.0, 0.9]):
        q = np.array(q) / h
        pw = np.exp(1j * (q[0] * ii + q[1] * jj + q[2] * kk) * h)
        y = A @ pw
        P = An.symbol(q, h, k, W7[idx.ravel()[0]])
        scale = 6.0 / h ** 2
        assert np.max(np.abs(y[inner] / pw[inner] - P)) < 1e-12 * scale


def test_dst_diagonalises_uniform_dirichlet_operator(w7_table):
    """With uniform weights, no PML and Dirichlet ends, the 3D DST-I
    (scipy.fft.dstn type 1) diagonalises A; its eigenvalues are the symbol at
    q_m = pi m / ((n+1) h)."""
    Gs, W7 = w7_table
    nx, ny, nz = 7, 6, 5
    h, f = 20.0, 10.0
    c = synth.homogeneous((nx, ny, nz), 2000.0)
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    A = O.assemble(c, f, h, 0, O.row_weights("GA", idx, W7))
    u = synth.random_vectors(nx * ny * nz, 1, 4)[0]
    uh = dstn(u.reshape(nz, ny, nx), type=1, norm="ortho")
    mz, my, mx = np.meshgrid(np.arange(1, nz + 1) * np.pi / (nz + 1),
                             np.arange(1, ny + 1) * np.pi / (ny + 1),
                             np.arange(1, nx + 1) * np.pi / (nx + 1), indexing="ij")
    lam = An.symbol(np.stack([mx, my, mz], -1) / h, h, 2 * math.pi * f / 2000.0, W7[idx.ravel()[0]])
    y_ref = idstn(lam * uh, type=1, norm="ortho").ravel()
    y = A @ u
    assert np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref) < 1e-14


def test_seven_point_reduces_to_ndimage_laplace():
    """w_s1 = 1 and lumped mass (w_m0 = 1): A u = Laplacian_7pt(u) + k^2 u with
    zero Dirichlet ends (scipy.ndimage.laplace, mode='constant')."""
    nx, ny, nz = 6, 5, 7
    h, f = 10.0, 7.0
    c = synth.homogeneous((nx, ny, nz), 1800.0)
    w = O.row_weights("fixed", fixed_w=[1, 0, 0, 1, 0, 0, 0], dims=(nx, ny, nz))
    A = O.assemble(c, f, h, 0, w)
    u = synth.random_vectors(nx * ny * nz, 1, 5)[0]
    lap = (scipy.ndimage.laplace(u.real.reshape(nz, ny, nx), mode="constant")
           + 1j * scipy.ndimage.laplace(u.imag.reshape(nz, ny, nx), mode="constant")).ravel() / h ** 2
    k2 = (2 * math.pi * f / 1800.0) ** 2
    assert np.allclose(A @ u, lap + k2 * u, rtol=1e-13, atol=1e-16)


def test_uniform_weights_with_pml_symmetric(w7_table):
    """Homogeneous model with PML: the impedance matrix is complex symmetric."""
    Gs, W7 = w7_table
    dims = (10, 9, 8)
    c = synth.homogeneous(dims, 2000.0)
    idx, _ = O.select_index(c, 10.0, 20.0, 3.0, 0.05, len(Gs))
    A = O.assemble(c, 10.0, 20.0, 3, O.row_weights("GA", idx, W7))
    assert abs(A - A.T).max() == 0.0
    assert abs(A.imag).max() > 0   # the PML is active


def test_csr_pattern(w7_table):
    """27-point pattern: nnz = prod(3 n_a - 2), columns ascending, neighbours
    only."""
    Gs, W7 = w7_table
    dims = (7, 5, 4)
    c = synth.gradient_z(dims, 25.0)
    idx, _ = O.select_index(c, 5.0, 25.0, 3.0, 0.05, len(Gs))
    ip, ind, val, shape = O.assemble_csr(c, 5.0, 25.0, 1, O.row_weights("GA", idx, W7))
    assert len(ind) == (3 * 7 - 2) * (3 * 5 - 2) * (3 * 4 - 2)
    assert ip[-1] == len(ind)
    for r in range(shape[0]):
        cols = ind[ip[r]:ip[r + 1]]
        assert np.all(np.diff(cols) > 0)
        i, j, k = r % 7, (r // 7) % 5, r // 35
        for col in cols:
            ci, cj, ck = col % 7, (col // 7) % 5, col // 35
            assert max(abs(ci - i), abs(cj - j), abs(ck - k)) <= 1
    # interior row of a 3x3x3 neighbourhood has all 27
    assert ip[1 + 7 * (1 + 5 * 1) + 1] - ip[1 + 7 * (1 + 5 * 1)] == 27


def test_pml_profile_shape():
    """xi = 1 inside, grows into the layer, gamma at the outer node is
    gamma_max = c ln(1/R) / (2 L (1 - 2/pi)), symmetric on both faces, and
    gamma at the layer's mid-depth is gamma_max (1 - cos(pi/4))."""
    n, npml, h, om, c = 30, 8, 20.0, 2 * math.pi * 10, 2000.0
    xn, xh = O.pml_profile(n, npml, h, om, c, 1e-3)
    assert np.all(xn[npml:n - npml] == 1.0)
    L = npml * h
    gmax = c * math.log(1e3) / (2 * L * (1 - 2 / math.pi))
    assert abs(xn[0].imag * om - gmax) < 1e-9 * gmax
    assert np.allclose(xn[::-1], xn) and np.allclose(xh[::-1], xh)
    assert abs(xn[npml // 2].imag * om - gmax * (1 - math.cos(math.pi / 4))) < 1e-9 * gmax
    assert np.all(np.diff(xn[:npml + 1].imag) < 0)
    # reflection coefficient of the continuous profile: exp(-2/c int gamma) = R
    d = np.linspace(0, L, 20001)
    integral = np.trapezoid(gmax * (1 - np.cos(np.pi * d / (2 * L))), d)
    assert abs(math.exp(-2 * integral / c) - 1e-3) < 1e-6


def test_mass_forms_agree_in_homogeneous_medium(w7_table):
    Gs, W7 = w7_table
    dims = (6, 6, 6)
    c = synth.homogeneous(dims, 2500.0)
    idx, _ = O.select_index(c, 8.0, 30.0, 3.0, 0.05, len(Gs))
    w = O.row_weights("GA", idx, W7)
    Aa = O.assemble(c, 8.0, 30.0, 2, w, mass_form="a")
    Ab = O.assemble(c, 8.0, 30.0, 2, w, mass_form="b")
    assert abs(Aa - Ab).max() <= 1e-15 * abs(Ab).max()


def test_gam_equals_ga_where_uniform_and_averages_at_interface(w7_table):
    Gs, W7 = w7_table
    dims = (5, 5, 6)
    c = synth.homogeneous(dims, 2000.0)
    c[3:] = 3000.0
    idx, _ = O.select_index(c, 10.0, 20.0, 3.0, 0.05, len(Gs))
    ga = O.row_weights("GA", idx, W7).reshape(6, 5, 5, 7)
    gam = O.row_weights("GAm", idx, W7, dims=dims).reshape(6, 5, 5, 7)
    assert np.allclose(ga[0], gam[0]) and np.allclose(ga[5], gam[5])
    # plane 2 sees planes 1,2 (slow) and 3 (fast): 2/3 slow, 1/3 fast
    assert np.allclose(gam[2, 2, 2], (2 * ga[0, 0, 0] + ga[5, 0, 0]) / 3)


def _pml_classes(dims, npml):
    """Per point: along each axis 0 (interior), 1 (low face) or 2 (high face)."""
    nx, ny, nz = dims
    ii, jj, kk = _grid(nx, ny, nz)
    out = []
    for q, n, p in ((ii, nx, npml[0]), (jj, ny, npml[1]), (kk, nz, npml[2])):
        out.append(np.where(q < p, 1, np.where(q >= n - p, 2, 0)))
    return np.stack(out, axis=1)


def test_assemble_rows_equals_assemble(w7_table):
    """The row-by-row assembly used on large grids reproduces the whole-matrix
    assembly on a heterogeneous grid whose rows cover the interior, every PML
    face, edge and corner class and the grid boundary (Sec. 2.1 operator,
    built two different ways: Kronecker products of whole 1D matrices versus
    of single rows)."""
    Gs, W7 = w7_table
    dims, npml, f, h = (11, 10, 9), (3, 2, 3), 7.0, 25.0
    c = synth.random_field_model(dims, h, seed=21)
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    w = O.row_weights("GA", idx, W7)
    classes = _pml_classes(dims, npml)
    # every combination of (interior, low, high) per axis occurs
    assert len({tuple(r) for r in classes}) == 27
    rows = np.arange(int(np.prod(dims)))
    for shift in (0.0, 0.7):
        A = O.assemble(c, f, h, npml, w, shift=shift)
        Ar = O.assemble_rows(c, f, h, npml, w[rows], rows, shift=shift)
        diff = abs(A - Ar).max()
        assert diff <= 1e-14 * abs(A).max(), (shift, diff)
        # the same explicit sparsity (no entry missing on either side)
        assert (A != 0).nnz == (Ar != 0).nnz


def _mass_entry_by_entry(c, f, h, npml, w, form):
    """Consistent mass of Sec. 2.1, equation (8), written out entry by entry:
    row i, neighbour j = i + d, class n = number of nonzero components of d,
    entry omega^2 / kappa_m * w_m[n](i) * prod_a s_a, where kappa_m is the bulk
    modulus (c^2, unit density) of the neighbour j in the first form and of
    the collocation point i in the second, and s_a is the coordinate stretch
    at the node (d_a = 0) or at the half node between i and j (d_a = +-1)."""
    nz, ny, nx = c.shape
    omega = 2.0 * math.pi * f
    cr = float(c.astype(np.float64).max())
    prof = [O.pml_profile(n, p, h, omega, cr) for n, p in zip((nx, ny, nz), npml)]
    c64 = c.astype(np.float64).ravel()
    N = nx * ny * nz
    M = np.zeros((N, N), complex)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = i + nx * (j + ny * k)
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            q = (i + dx, j + dy, k + dz)
                            if not (0 <= q[0] < nx and 0 <= q[1] < ny and 0 <= q[2] < nz):
                                continue
                            col = q[0] + nx * (q[1] + ny * q[2])
                            s = 1.0 + 0j
                            for a, (node, d) in enumerate(((i, dx), (j, dy), (k, dz))):
                                xn, xh = prof[a]
                                # half node between node and node + d is xh[node + 1] (d = +1) or xh[node] (d = -1)
                                s *= xn[node] if d == 0 else xh[node + (1 if d > 0 else 0)]
                            n = abs(dx) + abs(dy) + abs(dz)
                            kap = c64[col] ** 2 if form == "a" else c64[r] ** 2
                            M[r, col] += omega ** 2 / kap * w[r, 3 + n] * s
    return M


@pytest.mark.parametrize("form", ["a", "b"])
def test_mass_forms_entry_by_entry_heterogeneous(w7_table, form):
    """Both consistent-mass forms of Sec. 2.1 on a heterogeneous model with
    PML: the assembled matrix minus its stiffness (the same matrix assembled
    with zero mass weights) equals the mass written out entry by entry.  In a
    heterogeneous medium the two forms differ, and a row/column mix-up of the
    bulk modulus fails one of the two cases."""
    Gs, W7 = w7_table
    dims, npml, f, h = (6, 5, 7), (2, 1, 2), 9.0, 25.0
    c = synth.random_field_model(dims, h, seed=5)
    c[3:] *= np.float32(1.35)   # a sharp jump, so neighbouring k^2 differ
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    w = O.row_weights("GA", idx, W7)
    w_stiff = w.copy()
    w_stiff[:, 3:] = 0.0
    A = O.assemble(c, f, h, npml, w, mass_form=form).toarray()
    S = O.assemble(c, f, h, npml, w_stiff, mass_form=form).toarray()
    M = _mass_entry_by_entry(c, f, h, npml, w, form)
    assert np.abs((A - S) - M).max() <= 1e-13 * np.abs(M).max()
    other = _mass_entry_by_entry(c, f, h, npml, w, "b" if form == "a" else "a")
    assert np.abs(other - M).max() > 1e-3 * np.abs(M).max()


def test_attenuation_dst_eigenvalues(w7_table):
    """Constant-Q attenuation: in a uniform PML-free medium the operator is
    still diagonalised by the 3D DST-I, now with eigenvalues of the symbol at
    the complex wavenumber k~ = omega / (c (1 - i/(2Q))).  A conjugated factor
    or a sign error in it moves every eigenvalue's imaginary part."""
    Gs, W7 = w7_table
    nx, ny, nz = 7, 6, 5
    h, f, cv, Q = 20.0, 10.0, 2000.0, 30.0
    c = synth.homogeneous((nx, ny, nz), cv)
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(Gs))
    A = O.assemble(c, f, h, 0, O.row_weights("GA", idx, W7), Q=Q)
    u = synth.random_vectors(nx * ny * nz, 1, 4)[0]
    uh = dstn(u.reshape(nz, ny, nx), type=1, norm="ortho")
    mz, my, mx = np.meshgrid(np.arange(1, nz + 1) * np.pi / (nz + 1),
                             np.arange(1, ny + 1) * np.pi / (ny + 1),
                             np.arange(1, nx + 1) * np.pi / (nx + 1), indexing="ij")
    kt = 2 * math.pi * f / (cv * (1 - 0.5j / Q))
    assert kt.imag > 0   # outgoing waves decay under exp(-i omega t)
    lam = An.symbol(np.stack([mx, my, mz], -1) / h, h, kt, W7[idx.ravel()[0]])
    y_ref = idstn(lam * uh, type=1, norm="ortho").ravel()
    assert np.linalg.norm(A @ u - y_ref) / np.linalg.norm(y_ref) < 1e-14
    # and it reduces to the unattenuated operator as Q grows
    A0 = O.assemble(c, f, h, 0, O.row_weights("GA", idx, W7))
    A9 = O.assemble(c, f, h, 0, O.row_weights("GA", idx, W7), Q=1e9)
    assert abs(A9 - A0).max() <= 1e-8 * abs(A0).max()
