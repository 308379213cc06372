"""Accuracy of a wavefield against a reference (Sec. 3.1) and the closed-form
reference of the linear-velocity benchmark (Sec. 3.2).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

* ``wavefield_error``: the paper's accuracy metric (Sec. 3.1, equation err):
  the l1 norm of the gained real part of the difference over that of the
  reference, plus the same for the imaginary parts.  The gain W is diagonal
  and grows linearly with the distance from the source (it balances the
  geometrical spreading); here W_ii = r_i.
* ``gradient_greens``: the outgoing Green's function of
  Laplacian(p) + (omega / c(z))^2 p = delta(x - x_s) for c(z) = c0 + a z
  (the paper's linear model, whose analytic solution it takes from the
  literature).  Written out from the following derivation, not copied:
  with z' = z + c0 / a, c = a z' and kappa = omega / a the equation reads
  z'^2 Laplacian(p) + kappa^2 p = z'^2 delta.  Substituting p = z'^(-1/2) v
  gives z'^2 Laplacian(v) - z' dv/dz' + (3/4 + kappa^2) v, i.e. the
  Laplace-Beltrami operator of hyperbolic space in the upper half-space
  model (metric |dx|^2 / z'^2) plus (3/4 + kappa^2).  In that space the
  radial Green's function of Laplacian + 1 + nu^2 is -exp(i nu rho) /
  (4 pi sinh rho), rho the hyperbolic distance,
  cosh rho = 1 + |x - x_s|^2 / (2 z' z'_s).  With nu^2 = kappa^2 - 1/4 and
  the hyperbolic delta z'^3 delta:

      p = -exp(i nu rho) / (4 pi sinh(rho) sqrt(z' z'_s)).

  As a -> 0 it tends to -exp(i k r) / (4 pi r) with k = omega / c0.
* ``source_amplitude``: the far-field amplitude factor of a grid point
  source for a stencil's weights (the residue of the inverse symbol,
  ``analytic.amplitude_factor``), averaged over the plane-wave directions of
  the dispersion analysis.  The paper does not state how its point source
  is normalised; comparing a grid delta with the continuous Green's function
  needs this factor (1.27 at G = 4, 1.02 at G = 12 for every consistent
  stencil), and each stencil's own factor at the source point is used.
"""
from __future__ import annotations

import numpy as np

from . import analytic as An
from . import table as T

__all__ = ["wavefield_error", "gradient_greens", "source_amplitude"]


def wavefield_error(u_ref, u, gain):
    """Sec. 3.1, equation err: ||W Re(u_ref - u)||_1 / ||W Re(u_ref)||_1 +
    ||W Im(u_ref - u)||_1 / ||W Im(u_ref)||_1 with W = diag(gain)."""
    u_ref = np.asarray(u_ref, dtype=np.complex128).ravel()
    u = np.asarray(u, dtype=np.complex128).ravel()
    w = np.asarray(gain, dtype=np.float64).ravel()
    d = u_ref - u
    re = np.sum(np.abs(w * d.real)) / np.sum(np.abs(w * u_ref.real))
    im = np.sum(np.abs(w * d.imag)) / np.sum(np.abs(w * u_ref.imag))
    return float(re + im)


def gradient_greens(x, xs, c0, a, omega):
    """Outgoing solution of Laplacian(p) + (omega / (c0 + a z))^2 p =
    delta(x - xs) (same sign convention as ``analytic.greens``).  x: (..., 3)
    in metres, z the third coordinate; xs: (3,).  Requires c0 + a z > 0."""
    x = np.asarray(x, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    z0 = c0 / a
    zp = x[..., 2] + z0
    zs = xs[2] + z0
    r2 = np.sum((x - xs) ** 2, axis=-1)
    q = r2 / (2.0 * zp * zs)                       # cosh(rho) - 1
    rho = np.log1p(q + np.sqrt(q * (q + 2.0)))     # arccosh(1 + q), accurate for small q
    kappa = omega / a
    nu = np.sqrt(kappa * kappa - 0.25 + 0j)
    return -np.exp(1j * nu * rho) / (4.0 * np.pi * np.sinh(rho) * np.sqrt(zp * zs))


def source_amplitude(G, w7, theta=None, phi=None):
    """Mean over the dispersion analysis' plane-wave directions of the point
    source's far-field amplitude factor for weights w7 at G points per
    wavelength (unit grid step)."""
    if theta is None:
        theta, phi = T.angle_grid()
    k = 2.0 * np.pi / G
    vals = []
    for th, ph in zip(theta, phi):
        n = (np.cos(ph) * np.cos(th), np.cos(ph) * np.sin(th), np.sin(ph))
        vals.append(An.amplitude_factor(n, 1.0, k, w7)[0])
    return float(np.mean(vals))
