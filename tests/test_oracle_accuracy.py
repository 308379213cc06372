"""Pins of the accuracy metric (Sec. 3.1, equation err) and of the
linear-velocity Green's function (Sec. 3.2) against the mathematics: the PDE
itself by finite differences, the homogeneous limit, reciprocity, the
near-source singularity, and closed forms of the metric and of the point
source's amplitude factor."""
import math

import numpy as np

from oracle import accuracy as Acc
from oracle import analytic as An


def _lap4(fun, x, d):
    """Fourth-order central-difference Laplacian of fun at points x (n, 3)."""
    out = -3 * 30.0 * fun(x)
    for a in range(3):
        e = np.zeros(3)
        e[a] = d
        out = out + 16.0 * (fun(x + e) + fun(x - e)) - (fun(x + 2 * e) + fun(x - 2 * e))
    return out / (12.0 * d * d)


def test_gradient_greens_solves_the_helmholtz_equation():
    """Laplacian(p) + (omega / c(z))^2 p = 0 away from the source, checked by
    a fourth-order finite-difference Laplacian (step 0.5 m, wavelengths of
    300-600 m): relative residual below 1e-6 at points 150-2000 m away."""
    c0, a, omega = 1500.0, 0.7, 2 * math.pi * 5.0
    xs = np.array([1250.0, 1250.0, 275.0])
    rng = np.random.default_rng(11)
    x = xs + rng.uniform(-1200, 1200, (200, 3))
    x[:, 2] = rng.uniform(0.0, 2500.0, 200)
    x = x[np.linalg.norm(x - xs, axis=1) > 150.0]
    f = lambda y: Acc.gradient_greens(y, xs, c0, a, omega)  # noqa: E731
    p = f(x)
    k2 = (omega / (c0 + a * x[:, 2])) ** 2
    res = _lap4(f, x, 0.5) + k2 * p
    assert np.max(np.abs(res) / (k2 * np.abs(p))) < 1e-6


def test_gradient_greens_sign_convention_and_homogeneous_limit():
    """As the gradient vanishes the solution tends to the homogeneous
    -exp(i k r) / (4 pi r) (outgoing, the same convention as the oracle's
    homogeneous Green's function): with a = 1e-7 1/s over 2 km the two agree
    to 1e-5."""
    c0, omega = 2000.0, 2 * math.pi * 6.0
    xs = np.array([0.0, 0.0, 500.0])
    rng = np.random.default_rng(2)
    x = rng.uniform(-1000, 1000, (100, 3)) + np.array([0, 0, 1000.0])
    g = An.greens(np.linalg.norm(x - xs, axis=1), omega / c0)
    p = Acc.gradient_greens(x, xs, c0, 1e-7, omega)
    assert np.max(np.abs(p - g) / np.abs(g)) < 1e-5


def test_gradient_greens_reciprocity_and_singularity():
    """p(x; x_s) = p(x_s; x), and 4 pi r p -> -1 as r -> 0."""
    c0, a, omega = 1500.0, 0.7, 2 * math.pi * 5.0
    rng = np.random.default_rng(5)
    for _ in range(20):
        x = rng.uniform(0, 2500, 3)
        y = rng.uniform(0, 2500, 3)
        p1 = Acc.gradient_greens(x[None], y, c0, a, omega)[0]
        p2 = Acc.gradient_greens(y[None], x, c0, a, omega)[0]
        assert abs(p1 - p2) <= 1e-13 * abs(p1)
    xs = np.array([100.0, 200.0, 300.0])
    for r in (1e-2, 1e-4):
        p = Acc.gradient_greens((xs + np.array([r, 0, 0]))[None], xs, c0, a, omega)[0]
        assert abs(4 * math.pi * r * p + 1.0) < 20 * r * omega / c0


def test_wavefield_error_definition():
    """Equation err: 0 for the reference itself; 2 eps for u = (1 + eps) u_ref
    (each part contributes eps); the gain weights the samples (a zero gain
    removes a sample); a two-sample case by hand."""
    rng = np.random.default_rng(0)
    u = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    w = rng.uniform(0.5, 2.0, 50)
    assert Acc.wavefield_error(u, u, w) == 0.0
    assert abs(Acc.wavefield_error(u, 1.01 * u, w) - 0.02) < 1e-14
    v = u.copy()
    v[3] += 100.0 + 100.0j
    w0 = w.copy()
    w0[3] = 0.0
    assert Acc.wavefield_error(u, v, w0) == 0.0
    ref = np.array([1.0 + 2.0j, -3.0 + 1.0j])
    got = np.array([1.5 + 2.0j, -3.0 + 0.0j])
    gain = np.array([1.0, 2.0])
    # real: |1*(-0.5)| + 0 over 1 + 6 = 0.5/7; imag: 0 + |2*1| over 2 + 2 = 0.5
    assert abs(Acc.wavefield_error(ref, got, gain) - (0.5 / 7 + 0.5)) < 1e-15


def test_source_amplitude_closed_form_for_the_seven_point_stencil():
    """For the textbook 7-point Laplacian with a lumped mass along a grid
    axis, the symbol is -(2/h^2)(1 - cos qh) + k^2, its root obeys
    cos qh = 1 - (kh)^2 / 2 and the residue factor is qh / sin(qh)."""
    w7 = np.array([1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0])
    for G in (4.0, 6.0, 12.0, 25.0):
        kh = 2 * math.pi / G
        qh = math.acos(1 - kh * kh / 2)
        got = Acc.source_amplitude(G, w7, theta=[0.0], phi=[0.0])
        assert abs(got - qh / math.sin(qh)) < 1e-7
