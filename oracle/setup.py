"""Problem set-up shared by the full-grid and TT forms of the oracle.

Holds the grid, the quadrature, the time step and the per-cell fields of a
workload dict (see the ``workloads`` package).  Time step: the paper bounds
Delta t by CFL * Delta x / c (Sec. 3.1, below eq. lhs); the reading used is
Delta t = CFL * min(Delta x, Delta y[, Delta z]) / c.

Optional workload keys: ``flux`` ("upwind", the default, or "rusanov",
Sec. 3.1), ``s_plus`` (the Rusanov wavespeed S+ in units of c, default 1),
``kappa_s`` (per-cell scattering opacity, default 0, Sec. 3.2).  Boundary
codes: vacuum, periodic, inflow (Dirichlet) and outflow (ghost cell = the
adjacent interior cell, Sec. 4.5).
"""
import numpy as np

from . import quadrature

VACUUM, PERIODIC, INFLOW, OUTFLOW = 0, 1, 2, 3
UPWIND, RUSANOV, HLL = "upwind", "rusanov", "hll"
FROZEN, COUPLED = 0, 1


class Setup:
    def __init__(self, p):
        self.p = p
        self.dim = int(p["dim"])
        self.nx, self.ny = int(p["nx"]), int(p["ny"])
        self.nz = int(p["nz"]) if self.dim == 3 else 1
        self.ns = self.nx * self.ny * self.nz
        self.nt, self.np_ = int(p["ntheta"]), int(p["nphi"])
        self.c = float(p["c"])
        self.a_r = float(p["a_r"])
        self.dx = p["lx"] / self.nx
        self.dy = p["ly"] / self.ny
        self.dz = p["lz"] / self.nz if self.dim == 3 else np.inf
        self.spacing = [self.dx, self.dy, self.dz][: self.dim]
        self.dt = float(p.get("dt", 0.0)) or p["cfl"] * min(self.spacing) / self.c
        self.lam = [self.c * self.dt / h for h in self.spacing]
        self.bc_lo = list(p["bc_lo"])[:3]
        self.bc_hi = list(p["bc_hi"])[:3]
        for a in range(self.dim):
            if (self.bc_lo[a] == PERIODIC) != (self.bc_hi[a] == PERIODIC):
                raise ValueError("periodic boundaries must be paired")
        self.material = int(p["material"])
        self.kappa = np.asarray(p["kappa"], dtype=np.float64).copy()
        self.rho = np.asarray(p["rho"], dtype=np.float64).copy()
        self.cv = np.asarray(p["cv"], dtype=np.float64).copy()
        self.T0 = np.asarray(p["T0"], dtype=np.float64).copy()
        self.kappa_s = np.asarray(p.get("kappa_s", np.zeros(self.ns)), dtype=np.float64).copy()
        self.flux = p.get("flux", UPWIND)
        if self.flux not in (UPWIND, RUSANOV, HLL):
            raise ValueError("flux must be 'upwind', 'rusanov' or 'hll'")
        self.s_plus = float(p.get("s_plus", 1.0))
        self.hll_beta = float(p.get("hll_beta", 1.0))
        self.hll_threshold = float(p.get("hll_tau_threshold", 1e-2))
        if self.flux == HLL and not (0 < self.hll_beta < 1e300 and 0 < self.hll_threshold < 1e300):
            raise ValueError("hll_beta and hll_tau_threshold must be finite and > 0")
        self.inflow = [(int(f), np.asarray(fw, float), np.asarray(tw, float),
                        np.asarray(pw, float)) for (f, fw, tw, pw) in p["inflow"]]
        self.mu, self.w, self.phi, self.v = quadrature.ordinates(self.nt, self.np_)
        self.sin_t, self.cos_p, self.sin_p, _ = quadrature.direction_cosines(self.nt, self.np_)
        self.domega = np.outer(self.w, self.v)
        self.cell_volume = float(np.prod(self.spacing))
        # isotropic source block (emission and scattering) present unless the
        # temperature is frozen at zero and there is no scattering
        self.scatter = bool(np.any(self.kappa_s != 0.0))
        self.n_em = 0 if (self.material == FROZEN and not np.any(self.T0 != 0.0)
                          and not self.scatter) else 1

    # direction-cosine factors per axis: (theta factor, phi factor) of n_a
    def cosine_factors(self, axis):
        if axis == 0:
            return self.sin_t, self.cos_p
        if axis == 1:
            return self.sin_t, self.sin_p
        return self.mu, np.ones(self.np_)

    def grid_shape(self):
        return (self.nz, self.ny, self.nx)

    def face_cells(self, face):
        nx, ny, nz = self.nx, self.ny, self.nz
        ix = np.arange(nx); iy = np.arange(ny); iz = np.arange(nz)
        axis, hi = divmod(face, 2)
        if axis == 0:
            x = nx - 1 if hi else 0
            return (x + nx * (iy[None, :] + ny * iz[:, None])).reshape(-1)
        if axis == 1:
            y = ny - 1 if hi else 0
            return (ix[None, :] + nx * (y + ny * iz[:, None])).reshape(-1)
        z = nz - 1 if hi else 0
        return (ix[None, :] + nx * (iy[:, None] + ny * z)).reshape(-1)

    # ---- HLL flux (Sec. 3.1, eqs. hll and tauc) --------------------------
    def hll_tau(self, axis):
        """Optical depth tau_c at the hi face (i + 1/2 along ``axis``) of every
        cell, flattened: 2 beta Delta / (1/(rho k)_i + 1/(rho k)_{i+1}) with k
        the absorption plus scattering opacity (eq. tauc; reading: the second
        term is cell i+1's, the printed rho_i in both taken as a slip).  A
        face on a non-periodic boundary takes the interior cell's extinction
        on both sides (beta Delta (rho k)_i); zero extinction gives tau = 0."""
        ext = (self.rho * (self.kappa + self.kappa_s)).reshape(self.grid_shape())
        ax = 2 - axis
        nxt = np.roll(ext, -1, axis=ax)
        if self.bc_hi[axis] != PERIODIC:
            sl = [slice(None)] * 3
            sl[ax] = -1
            nxt[tuple(sl)] = ext[tuple(sl)]
        with np.errstate(divide="ignore"):
            inv = 1.0 / ext + 1.0 / nxt
        tau = np.where(np.isfinite(inv), 2.0 * self.hll_beta * self.spacing[axis] / inv, 0.0)
        return tau.reshape(-1)

    def hll_weights(self, tau):
        """Weights of the HLL face flux F = c n (alpha U_L + beta U_R) for n >= 0
        (alpha_p, beta_p) and n < 0 (alpha_m, beta_m).  With the wavespeeds of
        Sec. 3.1 written S_R = c n A, S_L = -c n B for n >= 0 and S_R = -c n B,
        S_L = c n A for n < 0, where A = sqrt((1 - exp(-tau^2)) / tau^2) and
        B = sqrt((1 - exp(-tau^4)) / tau^2) (their expansions sqrt(1 - tau^2/2)
        and tau below the threshold), eq. hll with F_{L,R} = c n U_{L,R} gives
        alpha_p = A (1 + B) / (A + B), beta_p = B (1 - A) / (A + B), and the
        n < 0 pair swapped: alpha_m = beta_p, beta_m = alpha_p.  tau -> 0 is
        the upwind flux (alpha_p = beta_m = 1); large tau the Rusanov flux
        with S+ = c |n| / tau."""
        tau = np.asarray(tau, dtype=float)
        small = tau < self.hll_threshold
        with np.errstate(divide="ignore", invalid="ignore"):
            A = np.where(small, np.sqrt(np.maximum(1.0 - 0.5 * tau * tau, 0.0)),
                         np.sqrt((1.0 - np.exp(-tau * tau)) / (tau * tau)))
            B = np.where(small, tau, np.sqrt((1.0 - np.exp(-tau ** 4)) / (tau * tau)))
        ap = A * (1.0 + B) / (A + B)
        bp = B * (1.0 - A) / (A + B)
        return ap, bp, bp, ap

    def hll_face_weights(self, axis):
        """(alpha_p, beta_p, alpha_m, beta_m) at every cell's hi face and at its
        lo face (the hi face of the cell before it, or the boundary face),
        flattened over cells."""
        hi = self.hll_weights(self.hll_tau(axis))
        ax = 2 - axis
        lo = []
        # the lo face of a cell: the previous cell's hi face; at a
        # non-periodic lo boundary the face takes the cell's own extinction
        ext = (self.rho * (self.kappa + self.kappa_s)).reshape(self.grid_shape())
        tb = (self.hll_beta * self.spacing[axis] * ext).reshape(-1)
        wb = self.hll_weights(tb)
        for h, b in zip(hi, wb):
            g = np.roll(h.reshape(self.grid_shape()), 1, axis=ax)
            if self.bc_lo[axis] != PERIODIC:
                sl = [slice(None)] * 3
                sl[ax] = 0
                g[tuple(sl)] = b.reshape(self.grid_shape())[tuple(sl)]
            lo.append(g.reshape(-1))
        return hi, tuple(lo)

