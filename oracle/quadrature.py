"""Latitude-longitude product quadrature (paper Sec. 3, Sec. 4.1 Integration).

The paper's angular grid samples cos(theta) and phi uniformly, is a 2-D
tensor-product grid, and its solid angles sum to 4 pi.  Reading used here:
midpoint cells in mu = cos(theta) in [-1, 1] and phi in [0, 2 pi), so that
w_l = 2/N_theta, v_p = 2 pi/N_phi and Delta Omega_{lp} = w_l v_p sums to
4 pi exactly.  With N_theta even and N_phi a multiple of 4 no ordinate has
a zero direction cosine.
"""
import numpy as np


def ordinates(ntheta, nphi):
    """Return (mu, w, phi, v): polar cosines and weights, azimuths and weights."""
    mu = -1.0 + (np.arange(ntheta) + 0.5) * (2.0 / ntheta)
    w = np.full(ntheta, 2.0 / ntheta)
    phi = (np.arange(nphi) + 0.5) * (2.0 * np.pi / nphi)
    v = np.full(nphi, 2.0 * np.pi / nphi)
    return mu, w, phi, v


def direction_cosines(ntheta, nphi):
    """n = [sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)] (Sec. 3).

    Returned as rank-1 factors: (sin_theta, cos_phi, sin_phi, mu), so that
    n_x = sin_theta (x) cos_phi, n_y = sin_theta (x) sin_phi and
    n_z = mu (x) 1 (Sec. 4.3).
    """
    mu, _, phi, _ = ordinates(ntheta, nphi)
    sin_t = np.sqrt(1.0 - mu * mu)
    return sin_t, np.cos(phi), np.sin(phi), mu


def solid_angles(ntheta, nphi):
    """Delta Omega_{lp} = w_l v_p as an (N_theta, N_phi) array."""
    _, w, _, v = ordinates(ntheta, nphi)
    return np.outer(w, v)
