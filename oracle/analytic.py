"""Closed forms used to pin the oracle (homogeneous medium).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

* Green's function of the Helmholtz equation with the e^{-i omega t}
  convention of the first-order system (Sec. 2.1): Laplacian(p) + k^2 p =
  delta(x - x_s) has the outgoing solution p = -exp(i k r) / (4 pi r).
  The paper validates its homogeneous benchmark against this solution
  (Sec. 3.1 / 3.2).
* Plane-wave symbol of the discrete operator in a homogeneous, unstretched
  medium, from the dispersion analysis of Sec. 2.2: for a wavevector q the
  27-point operator acts on exp(i q.x) as

      P(q) = -(2 / h^2) Q(q h) + k^2 J(q h)

  with Q the bracket under the square root of the phase-velocity equation and
  J its mass function, written with the directional cosines cos(q_a h).
* Far from the source the grid solution of P u = delta / h^3 behaves like
  alpha * (-exp(i k~ r) / (4 pi r)) with k~ the root of P along the direction
  and alpha = 1 / (-dP/d|q|^2) there (the residue of 1/P at its root); for
  the exact operator alpha = 1 and k~ = k.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

__all__ = ["greens", "symbol", "numerical_wavenumber", "amplitude_factor"]


def greens(r, k):
    """-exp(i k r) / (4 pi r)."""
    r = np.asarray(r, dtype=np.float64)
    return -np.exp(1j * k * r) / (4.0 * np.pi * r)


def symbol(q, h, k, w7):
    """P(q) for wavevectors q (..., 3) in rad/m (Sec. 2.2, numerator and J of
    the phase-velocity equation written as an operator symbol)."""
    q = np.asarray(q, dtype=np.float64)
    ca, cb, cc = (np.cos(q[..., a] * h) for a in range(3))
    A = ca * cb * cc
    B = ca * cb + ca * cc + cb * cc
    C = ca + cb + cc
    ws1, ws2, ws3, wm0, wm1, wm2, wm3 = w7
    Q = ws1 * (3 - C) + ws2 / 3 * (6 - C - B) + 2 * ws3 / 4 * (3 - 3 * A + B - C)
    J = wm0 + 2 * wm1 * C + 4 * wm2 * B + 8 * wm3 * A
    return -(2.0 / h ** 2) * Q + k ** 2 * J


def numerical_wavenumber(direction, h, k, w7):
    """Root |q| = k~ of P(|q| n) = 0 along the unit vector n (bracketed
    around k)."""
    n = np.asarray(direction, dtype=np.float64)
    n = n / np.linalg.norm(n)
    f = lambda s: symbol(s * n, h, k, w7)  # noqa: E731
    return brentq(f, 0.5 * k, 1.5 * k, xtol=1e-15 * k, rtol=1e-15)


def amplitude_factor(direction, h, k, w7):
    """alpha = 1 / (-dP/d(s^2)) at s = k~ along the direction (central
    difference in s)."""
    n = np.asarray(direction, dtype=np.float64)
    n = n / np.linalg.norm(n)
    kt = numerical_wavenumber(n, h, k, w7)
    ds = 1e-5 * kt
    dP = (symbol((kt + ds) * n, h, k, w7) - symbol((kt - ds) * n, h, k, w7)) / (2 * ds)
    return 1.0 / (-dP / (2.0 * kt)), kt
