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
the smoothed initial condition is the Gaussian of width omega,
G(r) = U0 / (2 pi omega^2) exp(-r^2 / (2 omega^2)), and its solution the
plane convolution of the two (line_source_smoothed_E).
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


def line_source_smoothed_E(t, r, U0=1.0, omega=0.03, c=1.0, n=20000):
    """Energy density of the line source from the Gaussian pulse of width
    omega (Sec. 5.4): the plane convolution of the delta-pulse solution with
    the normalised Gaussian.  In polar coordinates about the point, the
    angular integral of the Gaussian over a circle of radius s about a point
    at distance r from its centre is 2 pi exp(-(r^2 + s^2) / (2 omega^2))
    I_0(r s / omega^2), so

        E(t, r) = U0 / (2 pi omega^2 c t) int_0^{c t} s exp(-(r - s)^2 / (2 omega^2))
                  i0e(r s / omega^2) / sqrt((c t)^2 - s^2) ds,

    with i0e(z) = exp(-z) I_0(z).  The substitution s = c t sin(phi) removes
    the front's inverse square root; the phi integral over [0, pi/2] is
    taken by the midpoint rule on n points."""
    from scipy.special import i0e
    r = np.atleast_1d(np.asarray(r, dtype=float))
    ct = c * t
    h = 0.5 * np.pi / n
    s = ct * np.sin((np.arange(n) + 0.5) * h)
    w2 = omega * omega
    out = np.empty(r.shape)
    for k0 in range(0, r.size, 256):
        rr = r.reshape(-1)[k0:k0 + 256, None]
        f = s[None, :] * np.exp(-(rr - s[None, :]) ** 2 / (2 * w2)) * i0e(rr * s[None, :] / w2)
        out.reshape(-1)[k0:k0 + 256] = f.sum(axis=1) * h
    return U0 / (2 * np.pi * w2 * ct) * out
