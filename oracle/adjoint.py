"""Discrete adjoint of the full-grid step and finite differences.

Loss: radiation energy in a detector patch at the final time,
    L = sum_i det_i E_i^N Delta V,   E_i = (1/c) sum_{lp} I_ilp dOmega_lp.
Frozen temperature: the step is I^{m+1} = d (S I^m + b) + s, with S the
linear part of the upwind transport (zero ghosts), b its inflow part,
d = 1/(1 + c dt rho kappa) and s = d c dt rho kappa (c/4pi) a_r T^4, so
    dd/dkappa = -c dt rho d^2,   ds/dkappa = c dt rho (c/4pi) a_r T^4 d^2.
Reverse sweep: kbar += sum_lp Ibar^{m+1} (dd/dkappa I* + ds/dkappa),
Ibar* = d Ibar^{m+1}, Ibar^m = S^T Ibar*, where S^T swaps the roles of the
backward and forward neighbours (the transposed stencil).
"""
import numpy as np

from . import full
from .setup import PERIODIC, UPWIND


def _shift_zero(J, setup, axis, direction):
    ax = 2 - axis
    S = np.roll(J, -direction, axis=ax)
    if setup.bc_lo[axis] != PERIODIC:
        sl = [slice(None)] * J.ndim
        sl[ax] = 0 if direction < 0 else -1
        S[tuple(sl)] = 0.0
    return S


def transport_linear(I, setup):
    """S I: the upwind update with zero (or periodic) ghosts, no inflow."""
    out = I.copy()
    for a in range(setup.dim):
        tf, pf = setup.cosine_factors(a)
        n = np.outer(tf, pf)
        npos, nneg = np.maximum(n, 0.0), np.minimum(n, 0.0)
        Im = _shift_zero(I, setup, a, -1)
        Ip = _shift_zero(I, setup, a, +1)
        out -= setup.lam[a] * (npos * (I - Im) + nneg * (Ip - I))
    return out


def transport_adjoint(J, setup):
    """S^T J (transposed stencil)."""
    out = J.copy()
    for a in range(setup.dim):
        tf, pf = setup.cosine_factors(a)
        n = np.outer(tf, pf)
        npos, nneg = np.maximum(n, 0.0), np.minimum(n, 0.0)
        Jp = _shift_zero(J, setup, a, +1)
        Jm = _shift_zero(J, setup, a, -1)
        out -= setup.lam[a] * (npos * (J - Jp) + nneg * (Jm - J))
    return out


def loss_full(setup, kappa, nsteps, detector):
    s2 = _with_kappa(setup, kappa)
    I, _ = full.run(s2, nsteps)
    E = full.energy(I, s2)
    return float(np.sum(detector * E) * s2.cell_volume)


def _with_kappa(setup, kappa):
    import copy
    s2 = copy.copy(setup)
    s2.kappa = np.asarray(kappa, float).copy()
    return s2


def grad_full(setup, nsteps, detector):
    """(L, dL/dkappa) by the discrete adjoint (frozen temperature, upwind
    flux: with the HLL flux kappa would also enter the face weights)."""
    assert setup.material == 0
    assert setup.flux == UPWIND
    c, dt, a_r = setup.c, setup.dt, setup.a_r
    shp = setup.grid_shape() + (1, 1)
    I = full.initial_intensity(setup)
    T = setup.T0
    rk = setup.rho * setup.kappa
    d = 1.0 / (1.0 + c * dt * rk)
    s = d * c * dt * rk * (c / (4 * np.pi)) * a_r * T ** 4
    dd = -c * dt * setup.rho * d * d
    ds = c * dt * setup.rho * (c / (4 * np.pi)) * a_r * T ** 4 * d * d
    stars = []
    for _ in range(nsteps):
        Istar = full.transport(I, setup)
        stars.append(Istar)
        I = d.reshape(shp) * Istar + s.reshape(shp)
    E = full.energy(I, setup)
    L = float(np.sum(detector * E) * setup.cell_volume)
    Ibar = (detector * setup.cell_volume / c).reshape(shp) * setup.domega[None, None, None]
    kbar = np.zeros(setup.ns)
    for m in range(nsteps - 1, -1, -1):
        Istar = stars[m]
        kbar += (np.sum(Ibar * Istar, axis=(3, 4)).reshape(-1) * dd
                 + np.sum(Ibar, axis=(3, 4)).reshape(-1) * ds)
        Ibar = transport_adjoint(d.reshape(shp) * Ibar, setup)
    return L, kbar


def grad_fd(loss, kappa, cells, rel_step=1e-4):
    """Central differences of ``loss(kappa)`` at the given cells."""
    g = np.zeros(len(cells))
    for j, i in enumerate(cells):
        h = rel_step * kappa[i]
        kp = kappa.copy(); kp[i] += h
        km = kappa.copy(); km[i] -= h
        g[j] = (loss(kp) - loss(km)) / (2 * h)
    return g
