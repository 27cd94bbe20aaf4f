"""Analytic solutions of the paper's validation problems (test references).

TEST INFRASTRUCTURE ONLY, like the rest of the package.

Hohlraum (Sec. 5.1): vacuum, c given, isotropic intensity I = 1 entering
through the x = 0 and y = 0 boundaries from t = 0, both of infinite extent.
The mean intensity J = (1/4 pi) int I dOmega at (x, y) and time t is the
solid-angle fraction of the directions whose backward ray leaves the
quadrant through one of the two walls within a path length c t.  Sec. 5.1
gives it in closed form as J = J_left + J_bottom, with

    J_left = 1/2 - (pi - eta_x) x / (2 pi c t)
                 - asin(x sin(eta_x) / sqrt(x^2 + y^2)) / (2 pi)   if x < c t,
    eta_x = acos(min(y / sqrt((c t)^2 - x^2), 1)),

J_left = 0 for x >= c t, and J_bottom the same with x and y exchanged.

Line source (Sec. 5.4): a pulse U0 delta(x, y) of radiation energy in
vacuum spreads as E(t, r) = U0 H(c t - r) / (2 pi c t sqrt((c t)^2 - r^2)),
whose integral over the plane is U0 at every t (total energy is conserved);
the smoothed initial condition is the Gaussian of width omega.
"""
import numpy as np


def _hohlraum_wall(t, a, b, c):
    """Contribution of the wall at a = 0 (distance a to it, b along it)."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    ct = c * t
    out = np.zeros(np.broadcast(a, b).shape)
    a, b = np.broadcast_to(a, out.shape), np.broadcast_to(b, out.shape)
    m = a < ct
    am, bm = a[m], b[m]
    eta = np.arccos(np.minimum(bm / np.sqrt(ct * ct - am * am), 1.0))
    r = np.sqrt(am * am + bm * bm)
    out[m] = (0.5 - (np.pi - eta) * am / (2.0 * np.pi * ct)
              - np.arcsin(am * np.sin(eta) / r) / (2.0 * np.pi))
    return out


def hohlraum_J(t, x, y, c=1.0):
    """Analytic mean intensity of the hohlraum problem (Sec. 5.1)."""
    return _hohlraum_wall(t, x, y, c) + _hohlraum_wall(t, y, x, c)


def line_source_E(t, r, U0=1.0, c=1.0):
    """Energy density of the vacuum line source from a delta pulse (Sec. 5.4);
    zero outside the front r >= c t (the front itself is singular)."""
    r = np.asarray(r, dtype=float)
    ct = c * t
    out = np.zeros(r.shape)
    m = r < ct
    out[m] = U0 / (2.0 * np.pi * ct * np.sqrt(ct * ct - r[m] ** 2))
    return out
