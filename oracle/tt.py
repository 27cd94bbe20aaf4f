"""One step-then-truncate time step in TT form (paper Sec. 4).

Transport (Sec. 4.3).  n_x = sin(theta) (x) cos(phi),
n_y = sin(theta) (x) sin(phi) and n_z = mu (x) 1 are rank 1, and so are the
upwind masks, so the explicit update of eq. lhs is a sum of TTs.

Upwind flux, one block per axis and sign (reading of Sec. 4.3):
    I* = I + sum_a [ (D_a^- X) (tf_a^+ Theta) (-lam_a pf_a^+ Phi)
                   + (D_a^+ X) (tf_a^- Theta) (-lam_a pf_a^- Phi) ]
with D_a^- X = X_i - X_{i-e_a}, D_a^+ X = X_{i+e_a} - X_i, and for x/y:
tf^+ = tf^- = sin(theta), pf^+ = max(cos or sin, 0), pf^- = min(cos or
sin, 0); for z (3-D): tf^+ = max(mu, 0), tf^- = min(mu, 0), pf = 1.

Rusanov flux (eq. rusanov_flux_toro; Sec. 4.3 Rusanov), one central block
and one diffusion block per axis (the latter dropped when S+ = 0):
    I* = I + sum_a [ (D_a^0 X) (tf_a Theta) (-lam_a pf_a Phi)
                   + (D_a^2 X) Theta ((lam_a S+ / 2c) Phi) ]
with D^0 X = (X_{i+e_a} - X_{i-e_a}) / 2, D^2 X = X_{i+e_a} - 2 X_i + X_{i-e_a}.

Ghost rows of the stencils (Sec. 4.5): zero (vacuum, and inflow, whose
ghost value enters as rank-1 blocks), wrapped (periodic), or the adjacent
interior row (outflow).  A Dirichlet ghost value g = face_w (x) theta_w (x)
phi_w adds what the stencils miss at the face: upwind, on a lo face
e_face (x) tf^+ theta_w (x) lam pf^+ phi_w and on a hi face
e_face (x) tf^- theta_w (x) (-lam) pf^- phi_w; Rusanov,
e_face (x) tf theta_w (x) (+-lam/2) pf phi_w (+ on lo, - on hi) plus
e_face (x) theta_w (x) (lam S+/2c) phi_w.

Source (Sec. 4.4): every X-block row i is scaled by d_i and the isotropic
source block s (x) 1 (x) 1 (emission and scattering) is appended (omitted
when the temperature is frozen at zero and there is no scattering).

TT sum (Sec. 4.1 Addition): cores concatenated, middle core block-diagonal.
Block order: base, then per axis (minus, plus) or (central, diffusion),
then inflow entries in input order, then the source block.

Rounding: Gram-SVD (``rounding.round_gram``), once after the fused
transport + source sum by default; schedule "twice" also rounds after the
transport sum, as the paper does after each transport and each split update
(Sec. 4.2).
"""
import numpy as np

from . import material as mat
from . import rounding
from .setup import PERIODIC, OUTFLOW, RUSANOV, HLL


def shift(X, setup, axis, direction):
    """Rows X_{i + direction*e_a} with the ghost rows of the face crossed:
    zero, wrapped (periodic) or the row itself (outflow)."""
    r = X.shape[1]
    G = X.reshape(setup.grid_shape() + (r,))
    ax = 2 - axis
    S = np.roll(G, -direction, axis=ax)
    bc = setup.bc_lo[axis] if direction < 0 else setup.bc_hi[axis]
    if bc != PERIODIC:
        sl = [slice(None)] * 4
        sl[ax] = 0 if direction < 0 else -1
        S[tuple(sl)] = G[tuple(sl)] if bc == OUTFLOW else 0.0
    return S.reshape(-1, r)


def _signed_factors(tf, pf, a):
    """(theta, phi) factors of n^+ = max(n, 0) and n^- = min(n, 0) on axis a:
    for x and y the sign is the phi factor's (sin(theta) >= 0), for z the
    theta factor's (mu)."""
    if a < 2:
        return (tf, np.maximum(pf, 0.0)), (tf, np.minimum(pf, 0.0))
    return (np.maximum(tf, 0.0), pf), (np.minimum(tf, 0.0), pf)


def transport_blocks(X, Th, Ph, setup):
    blocks = [(X, Th, Ph)]
    rus = setup.flux == RUSANOV
    hll = setup.flux == HLL
    for a in range(setup.dim):
        tf, pf = setup.cosine_factors(a)
        lam = setup.lam[a]
        Xm, Xp = shift(X, setup, a, -1), shift(X, setup, a, +1)
        if hll:
            # one block per sign of n: the variable-weight stencil
            # (alpha_hi - beta_lo) X_i + beta_hi X_{i+1} - alpha_lo X_{i-1}
            (ap, bp, am, bm), (apl, bpl, aml, bml) = setup.hll_face_weights(a)
            for (al_hi, be_hi, al_lo, be_lo), (ts, ps) in zip(
                    ((ap, bp, apl, bpl), (am, bm, aml, bml)), _signed_factors(tf, pf, a)):
                Y = (al_hi - be_lo)[:, None] * X + be_hi[:, None] * Xp - al_lo[:, None] * Xm
                blocks.append((Y, Th * ts[None, :, None], Ph * (-lam * ps)[None, :]))
            continue
        if rus:
            blocks.append((0.5 * (Xp - Xm), Th * tf[None, :, None], Ph * (-lam * pf)[None, :]))
            if setup.s_plus != 0.0:
                blocks.append((Xp - 2.0 * X + Xm, Th, Ph * (0.5 * lam * setup.s_plus)))
            continue
        if a < 2:
            tpos = tneg = tf
            ppos, pneg = np.maximum(pf, 0.0), np.minimum(pf, 0.0)
        else:
            tpos, tneg = np.maximum(tf, 0.0), np.minimum(tf, 0.0)
            ppos = pneg = pf
        blocks.append((X - Xm, Th * tpos[None, :, None], Ph * (-lam * ppos)[None, :]))
        blocks.append((Xp - X, Th * tneg[None, :, None], Ph * (-lam * pneg)[None, :]))
    for (f, fw, tw, pw) in setup.inflow:
        a, hi = divmod(f, 2)
        tf, pf = setup.cosine_factors(a)
        lam = setup.lam[a]
        e = np.zeros(setup.ns)
        e[setup.face_cells(f)] = fw
        if hll:
            # the ghost value g enters F at the face: + lam n alpha_lo g on a lo
            # face, - lam n beta_hi g on a hi face, one block per sign of n
            (ap, bp, am, bm), (apl, bpl, aml, bml) = setup.hll_face_weights(a)
            wts = (bp, bm) if hi else (apl, aml)
            for w, (ts, ps) in zip(wts, _signed_factors(tf, pf, a)):
                blocks.append(((e * w)[:, None], (ts * tw)[None, :, None],
                               ((-lam if hi else lam) * ps * pw)[None, :]))
            continue
        if rus:
            sgn = -1.0 if hi else 1.0
            blocks.append((e[:, None], (tf * tw)[None, :, None], (sgn * 0.5 * lam * pf * pw)[None, :]))
            if setup.s_plus != 0.0:
                blocks.append((e[:, None], tw[None, :, None], (0.5 * lam * setup.s_plus * pw)[None, :]))
            continue
        if a < 2:
            tpart = tf * tw
            ppart = (lam * np.maximum(pf, 0.0) if not hi else -lam * np.minimum(pf, 0.0)) * pw
        else:
            tpart = (np.maximum(tf, 0.0) if not hi else np.minimum(tf, 0.0)) * tw
            ppart = (lam if not hi else -lam) * pf * pw
        blocks.append((e[:, None], tpart[None, :, None], ppart[None, :]))
    return blocks


def concat(blocks):
    """TT sum by core concatenation (Sec. 4.1 Addition)."""
    Xc = np.concatenate([b[0] for b in blocks], axis=1)
    R1 = Xc.shape[1]
    R2 = sum(b[2].shape[0] for b in blocks)
    nt = blocks[0][1].shape[1]
    Thc = np.zeros((R1, nt, R2))
    o1 = o2 = 0
    for (_, Th, Ph) in blocks:
        a, _, b = Th.shape
        Thc[o1:o1 + a, :, o2:o2 + b] = Th
        o1 += a
        o2 += b
    Phc = np.concatenate([b[2] for b in blocks], axis=0)
    return Xc, Thc, Phc


def energy(X, Th, Ph, setup):
    """E_i = (1/c) X_i (sum_l Theta_l w_l)(sum_p Phi_p v_p)  (eq. tt_energy_density)."""
    th = np.einsum("alb,l->ab", Th, setup.w)
    ph = Ph @ setup.v
    return X @ (th @ ph) / setup.c


def source_blocks(blocks, d, s, setup):
    out = [(d[:, None] * Xb, Thb, Phb) for (Xb, Thb, Phb) in blocks]
    if setup.n_em:
        out.append((s[:, None], np.ones((1, setup.nt, 1)), np.ones((1, setup.np_))))
    return out


def step(X, Th, Ph, T, setup, tol, rmax, schedule="once", ranks=None, perturb=None):
    """One TT step.  Returns ((X, Th, Ph), T_new, info).

    ``ranks``: replayed ranks, a pair (r1, r2) for "once" or a pair of
    pairs for "twice"; None uses the rank rule.  ``perturb`` (tests only):
    see ``rounding.gram_truncate``.
    """
    blocks = transport_blocks(X, Th, Ph, setup)
    infos = []
    rk_last = ranks
    if schedule == "twice":
        Xc, Thc, Phc = concat(blocks)
        rk = None if ranks is None else ranks[0]
        rk_last = None if ranks is None else ranks[1]
        (X1, Th1, Ph1), inf = rounding.round_gram(Xc, Thc, Phc, tol, rmax, rk, perturb=perturb)
        infos.append(inf)
        blocks = [(X1, Th1, Ph1)]
    Estar = sum(energy(*b, setup) for b in blocks)
    d, s, Tdag = mat.source_coefficients(Estar, T, setup)
    cat = concat(source_blocks(blocks, d, s, setup))
    (Xn, Thn, Phn), inf = rounding.round_gram(*cat, tol, rmax, rk_last, perturb=perturb)
    infos.append(inf)
    Enew = energy(Xn, Thn, Phn, setup)
    Tnew = mat.temperature_update(T, Estar, Enew, setup)
    return (Xn, Thn, Phn), Tnew, dict(Estar=Estar, Enew=Enew, d=d, s=s,
                                       round=infos, R=(cat[0].shape[1], cat[2].shape[0]))


def step_untruncated(X, Th, Ph, T, setup):
    """The same step without rounding: concatenated cores (ranks R1, R2)."""
    blocks = transport_blocks(X, Th, Ph, setup)
    Estar = sum(energy(*b, setup) for b in blocks)
    d, s, Tdag = mat.source_coefficients(Estar, T, setup)
    cat = concat(source_blocks(blocks, d, s, setup))
    Enew = energy(*cat, setup)
    return cat, mat.temperature_update(T, Estar, Enew, setup), dict(Estar=Estar, Enew=Enew, Tdag=Tdag)


def run(setup, nsteps, tol=None, rmax=None, schedule="once", cores=None, T=None,
        rank_schedule=None, callback=None):
    p = setup.p
    tol = p["tol"] if tol is None else tol
    rmax = p["rmax"] if rmax is None else rmax
    X, Th, Ph = cores if cores is not None else (np.asarray(p["X0"], float),
                                                  np.asarray(p["Th0"], float),
                                                  np.asarray(p["Ph0"], float))
    T = setup.T0.copy() if T is None else T
    history = []
    for m in range(nsteps):
        rk = None if rank_schedule is None else rank_schedule[m]
        (X, Th, Ph), T, info = step(X, Th, Ph, T, setup, tol, rmax, schedule, rk)
        history.append((X.shape[1], Ph.shape[0]))
        if callback is not None:
            callback(m, (X, Th, Ph), T, info)
    return (X, Th, Ph), T, history
