"""Dispersion analysis and the Tikhonov-smoothed G -> weights table (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Follows Sec. 2.2 of the paper:

* the normalised numerical phase velocity of the 27-point stencil in a
  homogeneous medium, as a function of G (grid points per wavelength), the
  plane-wave angles (theta, phi) and the seven weights (equation for v~ with
  the functions A, B, C);
* the five-unknown linear system sum_l H_l w_l = g obtained by asking v~ = 1
  after eliminating w_s3 and the last mass weight;
* the joint least-squares misfit over (G_i, theta_j, phi_k) (fixed "G4" /
  "Gm" weights) and the block-diagonal, Tikhonov-regularised problem
  min ||H w - g||^2 + lambda ||D P w||^2 (adaptive table).

Readings of points the paper leaves open:

* H_2 is printed without the constant term; eliminating w_s3 from v~ = 1 gives
  H_2 = (1 + 3A - 5B/3 + C/3)/2.  The rows here are *derived* from v~ (see
  ``dispersion_rows``) and the printed H_1, H_3..H_5 and g are recovered
  exactly; only H_2 differs, by the constant 1/2.
* Mass weights are per point: the dispersion function J weights each of the
  6 face, 12 edge and 8 corner neighbours by w_m1, w_m2, w_m3, so the
  constraint that makes J = 1 at zero wavenumber is
  w_m0 + 6 w_m1 + 12 w_m2 + 8 w_m3 = 1.  (The normalised form of the
  consistent-mass equation uses 6 w_m1, 12 w_m2, 8 w_m3.)
* Angle grid: theta and phi both take 0, 10, 20, 30, 40 degrees (the figure
  caption's 0-45 degrees by 10), 25 plane waves per G.
* D is the first difference along G with free ends ((N_G-1) x N_G per weight).
* Table axis: the configuration's G-uniform grid, or the paper's own axis
  (figure caption of the dispersion curves: 1/G from 0 to 0.4 by 0.001),
  uniform in s = 1/G.  On the 1/G axis the rows are written in s directly,
  so s = 0 (G infinite) is a regular point where every row vanishes (any
  consistent stencil is exact there) and only the smoothing term fixes the
  weights.
* The fixed-weight problem "G4" (N_G = 1) is rank deficient.  Its
  minimum-norm least-squares solution is a stencil with spurious modes: its
  stiffness symbol changes sign at q h = (pi, pi, 0) and its mass symbol
  goes negative, so a shifted-Laplacian preconditioned Krylov solve of it
  does not converge.  The "G4" of the accuracy comparison is the
  least-squares solution closest to the smoothed table's entry at G = 4
  (identical phase velocities at G = 4, positive symbols, worst error at
  G = 5.5 as the paper states); "Gm" (N_G = 4) is unique.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp

__all__ = [
    "angle_grid", "abc", "complete_weights", "phase_velocity", "dispersion_rows",
    "g_grid", "build_table", "fit_fixed", "table_normal_residual", "dispersion_rows_inv",
]


def angle_grid(step_deg: float = 10.0, max_deg: float = 40.0):
    """Plane-wave angles of the dispersion fit (Sec. 2.2, figure caption of the
    dispersion curves: 0 to 45 degrees by 10).  Returns (theta, phi) in radians,
    flattened over the full tensor grid, theta varying fastest."""
    a = np.deg2rad(np.arange(0.0, max_deg + 1e-9, step_deg))
    th, ph = np.meshgrid(a, a, indexing="xy")  # th varies along axis 1
    return th.ravel(), ph.ravel()


def abc(G, theta, phi):
    """The functions A, B, C of Sec. 2.2 (products / pair sums / sums of the
    three directional cosines cos(2 pi n_a / G))."""
    G = np.asarray(G, dtype=np.float64)
    ca = np.cos(2.0 * np.pi * np.cos(phi) * np.cos(theta) / G)
    cb = np.cos(2.0 * np.pi * np.cos(phi) * np.sin(theta) / G)
    cc = np.cos(2.0 * np.pi * np.sin(phi) / G)
    A = ca * cb * cc
    B = ca * cb + ca * cc + cb * cc
    C = ca + cb + cc
    return A, B, C


def complete_weights(w5):
    """From the five free weights (w_s1, w_s2, w_m0, w_m1, w_m2) to all seven,
    using sum w_s = 1 (Sec. 2.1) and the per-point mass constraint
    w_m0 + 6 w_m1 + 12 w_m2 + 8 w_m3 = 1.  Returns (..., 7) in the order
    (w_s1, w_s2, w_s3, w_m0, w_m1, w_m2, w_m3)."""
    w5 = np.asarray(w5, dtype=np.float64)
    ws1, ws2, wm0, wm1, wm2 = (w5[..., i] for i in range(5))
    ws3 = 1.0 - ws1 - ws2
    wm3 = (1.0 - wm0 - 6.0 * wm1 - 12.0 * wm2) / 8.0
    return np.stack([ws1, ws2, ws3, wm0, wm1, wm2, wm3], axis=-1)


def phase_velocity(G, theta, phi, w7):
    """Normalised numerical phase velocity v~ of the 27-point stencil
    (Sec. 2.2, the v~ equation):

        v~ = G / (sqrt(2 J) pi) * sqrt( w_s1 (3 - C) + w_s2/3 (6 - C - B)
                                        + 2 w_s3/4 (3 - 3A + B - C) )
        J  = w_m0 + 2 w_m1 C + 4 w_m2 B + 8 w_m3 A.
    """
    w7 = np.asarray(w7, dtype=np.float64)
    A, B, C = abc(G, theta, phi)
    ws1, ws2, ws3, wm0, wm1, wm2, wm3 = (w7[..., i] for i in range(7))
    Q = ws1 * (3.0 - C) + ws2 / 3.0 * (6.0 - C - B) + 2.0 * ws3 / 4.0 * (3.0 - 3.0 * A + B - C)
    J = wm0 + 2.0 * wm1 * C + 4.0 * wm2 * B + 8.0 * wm3 * A
    return np.asarray(G, dtype=np.float64) / (np.sqrt(2.0 * J) * np.pi) * np.sqrt(Q)


def dispersion_rows(G, theta, phi):
    """Rows of the linear system sum_l H_l w_l = g (Sec. 2.2), obtained by
    setting v~ = 1, i.e. Q = (2 pi^2 / G^2) J, and eliminating
    w_s3 = 1 - w_s1 - w_s2 and w_m3 = (1 - w_m0 - 6 w_m1 - 12 w_m2) / 8:

        H_1 = (3 + 3A - B - C) / 2
        H_2 = (1 + 3A - 5B/3 + C/3) / 2        (constant 1 restored, see header)
        H_3 = k2 (A - 1),  H_4 = k2 (6A - 2C),  H_5 = k2 (12A - 4B)
        g   = ((4 pi^2 / G^2 + 3) A - B + C - 3) / 2,   k2 = 2 pi^2 / G^2.

    Returns H with shape (..., 5) and g with shape (...)."""
    A, B, C = abc(G, theta, phi)
    k2 = 2.0 * np.pi ** 2 / np.asarray(G, dtype=np.float64) ** 2
    H = np.stack([
        0.5 * (3.0 + 3.0 * A - B - C),
        0.5 * (1.0 + 3.0 * A - 5.0 * B / 3.0 + C / 3.0),
        k2 * (A - 1.0),
        k2 * (6.0 * A - 2.0 * C),
        k2 * (12.0 * A - 4.0 * B),
    ], axis=-1)
    g = 0.5 * ((2.0 * k2 + 3.0) * A - B + C - 3.0)
    return H, g


def dispersion_rows_inv(s, theta, phi):
    """The same rows as ``dispersion_rows`` as functions of s = 1/G (the
    paper's 1/G table axis, Sec. 2.2 figure caption): the phases are
    2 pi s n_a and k2 = 2 pi^2 s^2, so s = 0 gives all-zero rows."""
    s = np.asarray(s, dtype=np.float64)
    ca = np.cos(2.0 * np.pi * np.cos(phi) * np.cos(theta) * s)
    cb = np.cos(2.0 * np.pi * np.cos(phi) * np.sin(theta) * s)
    cc = np.cos(2.0 * np.pi * np.sin(phi) * s)
    A = ca * cb * cc
    B = ca * cb + ca * cc + cb * cc
    C = ca + cb + cc
    k2 = 2.0 * np.pi ** 2 * s ** 2
    H = np.stack([
        0.5 * (3.0 + 3.0 * A - B - C),
        0.5 * (1.0 + 3.0 * A - 5.0 * B / 3.0 + C / 3.0),
        k2 * (A - 1.0),
        k2 * (6.0 * A - 2.0 * C),
        k2 * (12.0 * A - 4.0 * B),
    ], axis=-1)
    g = 0.5 * ((2.0 * k2 + 3.0) * A - B + C - 3.0)
    return H, g


def g_grid(gmin: float, gmax: float, dg: float) -> np.ndarray:
    """Tabulated G values G_i = gmin + i dg, i = 0 .. N_G - 1, with
    N_G = round((gmax - gmin) / dg) + 1 (each computed directly, not as a
    running sum)."""
    n = int(round((gmax - gmin) / dg)) + 1
    return gmin + np.arange(n, dtype=np.float64) * dg


def _stack_H(Gs, theta, phi, spacing="G"):
    """Block-diagonal H (one block of len(theta) rows x 5 per G) and stacked g
    (Sec. 2.2, the block-diagonal H of dimension (N_theta N_phi N_G) x (5 N_G));
    with spacing "invG" the abscissae are s = 1/G."""
    rows = dispersion_rows if spacing == "G" else dispersion_rows_inv
    blocks, gs = [], []
    for Gi in Gs:
        H, g = rows(Gi, theta, phi)
        blocks.append(H)
        gs.append(g)
    return sp.block_diag(blocks, format="csr"), np.concatenate(gs)


def _smoothing_operator(n_g: int, diff: str = "first"):
    """L = D P (Sec. 2.2): P reorders w from G-major ([w^(1); ...; w^(N_G)]) to
    weight-major, D is block diagonal with one difference operator per weight."""
    n = 5 * n_g
    # P: row r = l * n_g + i picks entry i * 5 + l of the G-major vector.
    rows = np.arange(n)
    cols = np.array([(r % n_g) * 5 + (r // n_g) for r in rows])
    P = sp.csr_matrix((np.ones(n), (rows, cols)), shape=(n, n))
    if diff == "first":
        d1 = sp.diags([-np.ones(n_g - 1), np.ones(n_g - 1)], [0, 1], shape=(n_g - 1, n_g))
    elif diff == "second":
        d1 = sp.diags([np.ones(n_g - 2), -2.0 * np.ones(n_g - 2), np.ones(n_g - 2)],
                      [0, 1, 2], shape=(n_g - 2, n_g))
    else:
        raise ValueError(diff)
    D = sp.block_diag([d1] * 5, format="csr")
    return D @ P


def build_table(gmin=3.0, gmax=20.0, dg=0.05, lam=1e-3, theta=None, phi=None,
                diff="first", spacing="G"):
    """Adaptive weight table (Sec. 2.2, Tikhonov-regularised block problem):

        minimize ||H w - g||^2 + lambda ||D P w||^2

    solved as the stacked least-squares problem [H; sqrt(lambda) L] w = [g; 0]
    with a dense LAPACK solver.  spacing "G": abscissae G_i = gmin + i dg;
    spacing "invG": abscissae s_i = gmin + i dg with s = 1/G (then gmin may be
    0).  Returns (abscissae [N_G], W [N_G, 5]) with the columns
    (w_s1, w_s2, w_m0, w_m1, w_m2)."""
    if theta is None:
        theta, phi = angle_grid()
    Gs = g_grid(gmin, gmax, dg)
    if lam == 0:
        # no coupling: every G is its own (rank-deficient) fit
        if spacing != "G":
            raise ValueError("lam = 0 needs the G axis")
        return Gs, np.stack([fit_fixed([G], theta, phi) for G in Gs])
    H, g = _stack_H(Gs, theta, phi, spacing)
    L = _smoothing_operator(len(Gs), diff)
    K = sp.vstack([H, np.sqrt(lam) * L]).toarray()
    rhs = np.concatenate([g, np.zeros(L.shape[0])])
    w, *_ = scipy.linalg.lstsq(K, rhs, lapack_driver="gelsd")
    return Gs, w.reshape(len(Gs), 5)


def table_normal_residual(Gs, W, lam, theta=None, phi=None, diff="first", spacing="G"):
    """Relative residual of the normal equations (H^T H + lambda L^T L) w = H^T g
    for a given table: a property any minimiser of the Tikhonov problem has."""
    if theta is None:
        theta, phi = angle_grid()
    H, g = _stack_H(Gs, theta, phi, spacing)
    L = _smoothing_operator(len(Gs), diff)
    w = np.asarray(W, dtype=np.float64).reshape(-1)
    lhs = H.T @ (H @ w) + lam * (L.T @ (L @ w))
    rhs = H.T @ g
    return float(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))


def fit_fixed(G_list, theta=None, phi=None, near=None):
    """Non-adaptive weights (Sec. 2.2, joint misfit over several G with one
    weight vector): N_G = 1 with G = 4 gives "G4", G = 4, 6, 8, 10 gives "Gm".
    The N_G = 1 problem has rank 3 (two of the five singular values vanish
    for any single G on the 25-direction grid), so its least-squares
    solutions form a plane.
    Without ``near``: the minimum-norm one (the pseudo-inverse with singular
    values below 1e-10 of the largest taken as zero).  With ``near`` (five
    free weights): the least-squares solution closest to it,
    near + pinv(H) (g - H near).  Returns the five free weights."""
    if theta is None:
        theta, phi = angle_grid()
    Hs, gs = [], []
    for Gi in G_list:
        H, g = dispersion_rows(float(Gi), theta, phi)
        Hs.append(H)
        gs.append(g)
    H = np.vstack(Hs)
    g = np.concatenate(gs)
    w0 = np.zeros(5) if near is None else np.asarray(near, dtype=np.float64)
    dw, *_ = scipy.linalg.lstsq(H, g - H @ w0, cond=1e-10, lapack_driver="gelsd")
    return w0 + dw


def worst_phase_error(Gs, W, theta=None, phi=None):
    """max over the grid of |v~ - 1| using each row's own weights."""
    if theta is None:
        theta, phi = angle_grid()
    w7 = complete_weights(W)
    err = 0.0
    for Gi, wi in zip(Gs, w7):
        err = max(err, float(np.max(np.abs(phase_velocity(Gi, theta, phi, wi) - 1.0))))
    return err


def kappa_cond(Gs, lam, theta=None, phi=None, diff="first"):
    """2-norm condition number of the stacked Tikhonov matrix (diagnostic)."""
    if theta is None:
        theta, phi = angle_grid()
    H, _ = _stack_H(Gs, theta, phi)
    L = _smoothing_operator(len(Gs), diff)
    K = sp.vstack([H, math.sqrt(lam) * L]).toarray()
    s = np.linalg.svd(K, compute_uv=False)
    return float(s[0] / s[-1])
