"""Pins of the oracle's dispersion analysis and weight table (CPU only).

Each test checks the oracle against something other than itself: another
equation of the paper, a textbook special case, a property every minimiser of
the regularised problem has, or a qualitative statement the paper makes.
"""
import math

import numpy as np
import pytest

from oracle import table as T


@pytest.fixture(scope="module")
def table():
    Gs, W = T.build_table(3.0, 20.0, 0.05, 1e-3)
    return Gs, W


def test_rows_match_phase_velocity_equation():
    """sum_l H_l w_l - g equals (2 pi^2/G^2) J (v~^2 - 1) for arbitrary weights:
    the linear system of Sec. 2.2 is v~ = 1 rearranged.  A wrong constant in any
    row (as in the printed H_2) breaks it."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        G = rng.uniform(2.5, 40.0)
        th = rng.uniform(0, np.pi / 2)
        ph = rng.uniform(0, np.pi / 4)
        w5 = rng.uniform(-0.5, 1.0, 5)
        w7 = T.complete_weights(w5)
        H, g = T.dispersion_rows(G, th, ph)
        A, B, C = T.abc(G, th, ph)
        J = w7[3] + 2 * w7[4] * C + 4 * w7[5] * B + 8 * w7[6] * A
        if J <= 0:
            continue
        v = T.phase_velocity(G, th, ph, w7)
        lhs = float(H @ w5 - g)
        rhs = 2 * np.pi ** 2 / G ** 2 * J * (v ** 2 - 1.0)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_printed_h2_differs_by_constant_half():
    """The printed H_2 lacks the constant: H_2(derived) - H_2(printed) = 1/2."""
    for G in (3.0, 7.3, 20.0):
        H, _ = T.dispersion_rows(G, 0.3, 0.2)
        A, B, C = T.abc(G, 0.3, 0.2)
        printed = 0.5 * (3 * A - 5 * B / 3 + C / 3)
        assert abs(H[1] - printed - 0.5) < 1e-14


def test_seven_point_textbook_dispersion():
    """w_s1 = 1 with lumped mass (w_m0 = 1) is the classical 7-point stencil;
    along an axis its phase velocity is (G/pi) sin(pi/G) (textbook
    second-order dispersion)."""
    w7 = np.array([1, 0, 0, 1, 0, 0, 0], float)
    for G in (3.0, 4.0, 10.0, 25.0):
        v = T.phase_velocity(G, 0.0, 0.0, w7)
        assert abs(v - G / math.pi * math.sin(math.pi / G)) < 1e-14


def test_consistency_large_G():
    """Any weights obeying the two sum constraints give v~ -> 1 as G -> inf."""
    rng = np.random.default_rng(2)
    w7 = T.complete_weights(rng.uniform(0, 0.5, 5))
    v = T.phase_velocity(1e4, 0.4, 0.3, w7)
    assert abs(v - 1) < 1e-6


def test_table_shape_and_grid(table):
    Gs, W = table
    assert W.shape == (341, 5)
    assert Gs[0] == 3.0 and abs(Gs[-1] - 20.0) < 1e-12
    assert np.all(np.diff(Gs) > 0)


def test_table_normal_equations(table):
    """A minimiser of ||Hw-g||^2 + lambda ||DPw||^2 satisfies the normal
    equations (H^T H + lambda L^T L) w = H^T g."""
    Gs, W = table
    assert T.table_normal_residual(Gs, W, 1e-3) < 1e-9


def test_table_constraints(table):
    """sum w_s = 1 and w_m0 + 6 w_m1 + 12 w_m2 + 8 w_m3 = 1 on every row."""
    _, W = table
    w7 = T.complete_weights(W)
    assert np.allclose(w7[:, :3].sum(1), 1.0, atol=1e-14)
    assert np.allclose(w7[:, 3] + 6 * w7[:, 4] + 12 * w7[:, 5] + 8 * w7[:, 6], 1.0, atol=1e-14)


def test_adaptive_table_is_accurate(table):
    """The adaptive weights reduce dispersion very significantly over the whole
    G range (Sec. 2.2): worst |v~ - 1| over G in [3, 20] and all angles stays
    below 5e-4 (the fixed G4 weights reach ~3e-2 there)."""
    Gs, W = table
    err = T.worst_phase_error(Gs, W)
    assert err < 5e-4
    w4 = T.fit_fixed([4.0])
    err4 = T.worst_phase_error(Gs, np.broadcast_to(w4, W.shape))
    assert err4 > 20 * err


def test_table_is_smooth(table):
    """Tikhonov smoothing: successive rows differ by small amounts."""
    _, W = table
    assert np.max(np.abs(np.diff(W, axis=0))) < 5e-3


def test_lambda_large_limit():
    """lambda -> infinity forces one weight vector for all G."""
    Gs, W = T.build_table(3.0, 6.0, 0.5, 1e8)
    assert np.max(np.ptp(W, axis=0)) < 1e-4


def test_lambda_small_fits_each_G_better():
    """A smaller lambda never increases the data misfit."""
    th, ph = T.angle_grid()

    def misfit(Gs, W):
        return sum(float(np.sum((T.dispersion_rows(g, th, ph)[0] @ w - T.dispersion_rows(g, th, ph)[1]) ** 2))
                   for g, w in zip(Gs, W))

    Gs, Wa = T.build_table(3.0, 8.0, 0.25, 1e-1)
    _, Wb = T.build_table(3.0, 8.0, 0.25, 1e-5)
    assert misfit(Gs, Wb) <= misfit(Gs, Wa) * (1 + 1e-9)


def test_g4_worst_error_near_5p5():
    """Weights fitted for G = 4 only: accurate at 4, worst for G > 4 at
    G ~ 5.5 (Sec. 2.2)."""
    w7 = T.complete_weights(T.fit_fixed([4.0]))
    th, ph = T.angle_grid()
    Gf = np.linspace(4.2, 20.0, 791)
    e = np.array([np.max(np.abs(T.phase_velocity(g, th, ph, w7) - 1)) for g in Gf])
    gworst = Gf[np.argmax(e)]
    assert 5.0 <= gworst <= 6.0
    e4 = np.max(np.abs(T.phase_velocity(4.0, th, ph, w7) - 1))
    assert e4 < 1e-4


def _symbols(w7, n=33):
    """Stiffness bracket Q and mass function J of Sec. 2.2 over the grid's
    wavenumbers q h in [0, pi]^3."""
    q = np.linspace(0.0, np.pi, n)
    ca, cb, cc = np.meshgrid(np.cos(q), np.cos(q), np.cos(q), indexing="ij")
    A, B, C = ca * cb * cc, ca * cb + ca * cc + cb * cc, ca + cb + cc
    ws1, ws2, ws3, wm0, wm1, wm2, wm3 = w7
    Q = ws1 * (3 - C) + ws2 / 3 * (6 - C - B) + 2 * ws3 / 4 * (3 - 3 * A + B - C)
    J = wm0 + 2 * wm1 * C + 4 * wm2 * B + 8 * wm3 * A
    return Q.ravel()[1:], J.ravel()


def test_g4_null_space_and_anchored_solution():
    """The N_G = 1 problem at G = 4 has rank 3: a plane of least-squares
    solutions.  The minimum-norm member has a stiffness symbol
    that changes sign and a negative mass symbol (spurious grid modes); the
    member closest to the smoothed table's entry at G = 4 fits G = 4 exactly
    as well, keeps both symbols positive, and has its worst error for G > 4
    at G ~ 5.5 (Sec. 2.2)."""
    th, ph = T.angle_grid()
    H, g = T.dispersion_rows(4.0, th, ph)
    assert np.linalg.matrix_rank(H, tol=1e-10 * np.linalg.norm(H, 2)) == 3
    Gs, W = T.build_table(3.0, 6.0, 0.05, 1e-3)
    w_min = T.fit_fixed([4.0])
    w_anc = T.fit_fixed([4.0], near=W[20])
    r_min = np.linalg.norm(H @ w_min - g)
    r_anc = np.linalg.norm(H @ w_anc - g)
    assert abs(r_anc - r_min) <= 1e-9 * r_min
    Qm, Jm = _symbols(T.complete_weights(w_min))
    Qa, Ja = _symbols(T.complete_weights(w_anc))
    assert Qm.min() < 0 and Jm.min() < 0
    assert Qa.min() > 0 and Ja.min() > 0
    w7 = T.complete_weights(w_anc)
    Gf = np.linspace(4.2, 20.0, 791)
    e = np.array([np.max(np.abs(T.phase_velocity(x, th, ph, w7) - 1)) for x in Gf])
    assert 5.0 <= Gf[np.argmax(e)] <= 6.0


def test_gm_trades_accuracy_at_g4():
    """Weights fitted jointly for G = 4, 6, 8, 10 are less accurate at G = 4
    than the G4 weights but better balanced over 4..10 (Sec. 2.2)."""
    th, ph = T.angle_grid()
    w4 = T.complete_weights(T.fit_fixed([4.0]))
    wm = T.complete_weights(T.fit_fixed([4.0, 6.0, 8.0, 10.0]))
    err = lambda w, g: np.max(np.abs(T.phase_velocity(g, th, ph, w) - 1))  # noqa: E731
    assert err(wm, 4.0) > err(w4, 4.0)
    Gr = np.linspace(4, 10, 61)
    assert max(err(wm, g) for g in Gr) < max(err(w4, g) for g in Gr)


def test_g_grid_direct():
    Gs = T.g_grid(3.0, 20.0, 0.05)
    assert len(Gs) == 341
    assert Gs[140] == 3.0 + 140 * 0.05


# ---- the paper's own table axis: uniform in s = 1/G (0 to 0.4 by 0.001) ----

@pytest.fixture(scope="module")
def table_inv():
    S, W = T.build_table(0.0, 0.4, 0.001, 1e-3, spacing="invG")
    return S, W


def test_inverse_rows_match_phase_velocity_equation():
    """Rows written in s = 1/G obey the same rearranged v~ = 1 equation:
    sum_l H_l w_l - g = 2 pi^2 s^2 J (v~^2 - 1), with v~ and J evaluated from
    the paper's phase-velocity formula at G = 1/s."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        s = rng.uniform(0.01, 0.45)
        th = rng.uniform(0, np.pi / 2)
        ph = rng.uniform(0, np.pi / 4)
        w7 = T.complete_weights(rng.uniform(-0.5, 1.0, 5))
        H, g = T.dispersion_rows_inv(s, th, ph)
        A, B, C = T.abc(1.0 / s, th, ph)
        J = w7[3] + 2 * w7[4] * C + 4 * w7[5] * B + 8 * w7[6] * A
        if J <= 0:
            continue
        v = T.phase_velocity(1.0 / s, th, ph, w7)
        lhs = float(H @ np.delete(w7, [2, 6]) - g)
        rhs = 2 * np.pi ** 2 * s ** 2 * J * (v ** 2 - 1.0)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


def test_inverse_rows_vanish_at_infinite_G():
    """At s = 0 (G infinite) every stencil satisfying sum w_s = 1 and the mass
    normalisation is exact, so every row and the right-hand side vanish."""
    th, ph = T.angle_grid()
    H, g = T.dispersion_rows_inv(np.zeros_like(th), th, ph)
    assert np.all(H == 0.0) and np.all(g == 0.0)


def test_inverse_table_paper_axis(table_inv):
    """The Tikhonov table on the paper's axis 1/G in [0, 0.4] by 0.001 (401
    entries): it satisfies the normal equations, the consistency constraints,
    and keeps the phase-velocity error small over G >= 2.5 -- about as small
    on G in [3, 20] as the G-axis table of the configuration."""
    S, W = table_inv
    assert len(S) == 401 and S[0] == 0.0 and abs(S[-1] - 0.4) < 1e-15
    assert T.table_normal_residual(S, W, 1e-3, spacing="invG") <= 1e-12
    w7 = T.complete_weights(W)
    assert np.allclose(w7[:, :3].sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(w7[:, 3] + 6 * w7[:, 4] + 12 * w7[:, 5] + 8 * w7[:, 6], 1.0, atol=1e-14)
    th, ph = T.angle_grid()
    err = [float(np.max(np.abs(T.phase_velocity(1.0 / s, th, ph, w) - 1.0))) for s, w in zip(S[1:], w7[1:])]
    assert max(err) <= 2e-3
    band = [e for s, e in zip(S[1:], err) if 1 / 20.0 - 1e-12 <= s <= 1 / 3.0 + 1e-12]
    assert max(band) <= 5e-4


def test_select_index_inverse_is_nearest_entry():
    """Index on the 1/G axis: the nearest tabulated s = (f h)/c, ties upward,
    clamped at both ends (brute force over the table entries)."""
    from oracle import operator as O
    rng = np.random.default_rng(3)
    c = rng.uniform(300.0, 9000.0, 5000).astype(np.float32)
    f, h, s0, ds, n = 7.5, 20.0, 0.0, 0.001, 401
    idx, ncl = O.select_index(c, f, h, s0, ds, n, spacing="invG")
    s_tab = s0 + np.arange(n) * ds
    v = (f * h) / c.astype(np.float64)
    d = np.abs(v[:, None] - s_tab[None, :])
    best = n - 1 - np.argmin(d[:, ::-1], axis=1)   # ties go to the larger index
    assert np.array_equal(idx, best)
    assert ncl == int(np.count_nonzero(v > s_tab[-1] + ds / 2))
