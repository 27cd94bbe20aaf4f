"""Full-grid ("traditional") S_N step: the plain definition of the method.

The intensity is a dense array I[nz, ny, nx, N_theta, N_phi].

Transport (Sec. 3.1, eq. lhs, applied per axis in multi-D), with the
interface flux of the workload:
  upwind (eq. upwind): F_{i+1/2} = c n I_i if n >= 0, else c n I_{i+1}, so
    I*_i = I_i - sum_a lam_a [ n_a^+ (I_i - I_{i-e_a}) + n_a^- (I_{i+e_a} - I_i) ];
  Rusanov (eq. rusanov_flux_toro): F_{i+1/2} = (c n / 2)(I_i + I_{i+1})
    - (S+ / 2)(I_{i+1} - I_i), so
    I*_i = I_i - sum_a lam_a [ (n_a / 2)(I_{i+e_a} - I_{i-e_a})
                              - (S+ / 2c)(I_{i+e_a} - 2 I_i + I_{i-e_a}) ],
  HLL (eq. hll with the wavespeeds of Sec. 3.1 and tau_c of eq. tauc):
    F_{i+1/2} = c n (alpha I_i + beta I_{i+1}) with per-face weights (see
    Setup.hll_weights), I*_i = I_i - sum_a lam_a (F_{i+1/2} - F_{i-1/2}) / c,
lam_a = c dt / Delta_a, n^+ = max(n, 0), n^- = min(n, 0).  Ghost values
(Sec. 4.5): vacuum 0, periodic wrap, inflow (Dirichlet) a prescribed value
g = face_w (x) theta_w (x) phi_w on the face, outflow the adjacent interior
cell.

Energy density (Sec. 3, discrete form): E_i = (1/c) sum_{lp} I_ilp dOmega_lp.

Source step: I^{m+1} = d I* + s (see ``material``).
"""
import numpy as np

from . import material as mat
from .setup import PERIODIC, INFLOW, OUTFLOW, RUSANOV, HLL


def _ghost(setup, face, like_slice):
    """Dirichlet ghost values on ``face`` shaped like a boundary slice."""
    g = np.zeros_like(like_slice)
    for (f, fw, tw, pw) in setup.inflow:
        if f == face:
            axis = f // 2
            nx, ny, nz = setup.nx, setup.ny, setup.nz
            shp = {0: (nz, ny), 1: (nz, nx), 2: (ny, nx)}[axis]
            g += fw.reshape(shp)[:, :, None, None] * tw[None, None, :, None] * pw[None, None, None, :]
    return g


def neighbours(I, setup, axis):
    """(I_{i-e_a}, I_{i+e_a}) with the boundary ghosts of ``axis``."""
    ax = 2 - axis  # array axis of spatial axis a in (nz, ny, nx, ...)
    Im = np.roll(I, 1, axis=ax)
    Ip = np.roll(I, -1, axis=ax)
    lo = [slice(None)] * I.ndim
    hi = [slice(None)] * I.ndim
    lo[ax] = 0
    hi[ax] = -1
    lo, hi = tuple(lo), tuple(hi)
    bl, bh = setup.bc_lo[axis], setup.bc_hi[axis]
    if bl != PERIODIC:
        Im[lo] = (_ghost(setup, 2 * axis, Im[lo]) if bl == INFLOW
                  else I[lo] if bl == OUTFLOW else 0.0)
    if bh != PERIODIC:
        Ip[hi] = (_ghost(setup, 2 * axis + 1, Ip[hi]) if bh == INFLOW
                  else I[hi] if bh == OUTFLOW else 0.0)
    return Im, Ip


def transport(I, setup):
    """One explicit transport update (eq. lhs with the workload's flux)."""
    out = I.copy()
    for a in range(setup.dim):
        tf, pf = setup.cosine_factors(a)
        n = np.outer(tf, pf)
        Im, Ip = neighbours(I, setup, a)
        if setup.flux == RUSANOV:
            out -= setup.lam[a] * (0.5 * n * (Ip - Im)
                                   - 0.5 * setup.s_plus * (Ip - 2.0 * I + Im))
        elif setup.flux == HLL:
            # eq. hll: F_{i+1/2} / c = n (alpha U_i + beta U_{i+1}), weights per
            # sign of n from the face's optical depth (Setup.hll_weights)
            shp = setup.grid_shape() + (1, 1)
            hi, lo = setup.hll_face_weights(a)
            ap, bp, am, bm = (w.reshape(shp) for w in hi)
            apl, bpl, aml, bml = (w.reshape(shp) for w in lo)
            npos, nneg = np.maximum(n, 0.0), np.minimum(n, 0.0)
            f_hi = npos * (ap * I + bp * Ip) + nneg * (am * I + bm * Ip)
            f_lo = npos * (apl * Im + bpl * I) + nneg * (aml * Im + bml * I)
            out -= setup.lam[a] * (f_hi - f_lo)
        else:
            npos, nneg = np.maximum(n, 0.0), np.minimum(n, 0.0)
            out -= setup.lam[a] * (npos * (I - Im) + nneg * (Ip - I))
    return out


def energy(I, setup):
    """E_i = (1/c) sum_{l,p} I_{ilp} w_l v_p, flattened over cells."""
    return np.einsum("zyxlp,lp->zyx", I, setup.domega).reshape(-1) / setup.c


def initial_intensity(setup):
    p = setup.p
    X, Th, Ph = (np.asarray(p[k], float) for k in ("X0", "Th0", "Ph0"))
    I = np.einsum("ia,alb,bp->ilp", X, Th, Ph)
    return I.reshape(setup.nz, setup.ny, setup.nx, setup.nt, setup.np_)


def step(I, T, setup):
    """One full-grid step; returns (I_new, T_new, info)."""
    Istar = transport(I, setup)
    Estar = energy(Istar, setup)
    d, s, Tdag = mat.source_coefficients(Estar, T, setup)
    shp = setup.grid_shape() + (1, 1)
    Inew = d.reshape(shp) * Istar + s.reshape(shp)
    Enew = energy(Inew, setup)
    Tnew = mat.temperature_update(T, Estar, Enew, setup)
    return Inew, Tnew, dict(Estar=Estar, Enew=Enew, d=d, s=s, Tdag=Tdag)


def run(setup, nsteps, I=None, T=None):
    I = initial_intensity(setup) if I is None else I
    T = setup.T0.copy() if T is None else T
    for _ in range(nsteps):
        I, T, _ = step(I, T, setup)
    return I, T
