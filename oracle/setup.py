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
UPWIND, RUSANOV = "upwind", "rusanov"
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
        if self.flux not in (UPWIND, RUSANOV):
            raise ValueError("flux must be 'upwind' or 'rusanov'")
        self.s_plus = float(p.get("s_plus", 1.0))
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
