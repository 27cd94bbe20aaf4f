"""Seeded synthetic workloads for the tensor-train S_N step.

This module only *describes* problems: grid and angle counts, physical
constants, boundary codes, per-cell material fields, initial TT cores and
inflow beam profiles.  It holds none of the method's arithmetic (no
quadrature, no transport, no rounding); both the CPU oracle and the HIP
library read the arrays produced here, so they see bit-identical inputs.

Every generator returns a plain ``dict``:

========== ==============================================================
key        meaning
========== ==============================================================
dim        2 or 3
nx,ny,nz   cells per axis (nz = 1 when dim == 2)
ntheta     polar ordinates (uniform in cos(theta)); even
nphi       azimuthal ordinates; multiple of 4
lx,ly,lz   domain extents (cell size = l/n)
c, a_r     speed of light, radiation constant
cfl        time step = cfl * min cell size / c
tol        relative Frobenius rounding tolerance
rmax       rank cap (<= 0: none)
bc_lo/hi   per axis: 0 vacuum, 1 periodic, 2 inflow, 3 outflow
material   0 frozen temperature, 1 coupled (backward-Euler material)
kappa,rho,cv,T0  per-cell float64 arrays of length N_s = nx*ny*nz
X0,Th0,Ph0 initial cores, shapes (N_s,r1), (r1,ntheta,r2), (r2,nphi)
inflow     list of (face, face_w, theta_w, phi_w); face 0..5 =
           x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; face_w is indexed by the
           face's own 2-D cell index (see ``face_cells``)
steps      number of steps of the workload
flux       optional: "upwind" (default), "rusanov" or "hll"
s_plus     optional: Rusanov wavespeed S+ in units of c (default 1)
hll_beta   optional: HLL optical-depth factor beta (default 1)
hll_tau_threshold  optional: HLL wavespeed series threshold (default 1e-2)
kappa_s    optional: per-cell scattering opacity (default 0)
========== ==============================================================

Spatial cells are flattened as ``i = ix + nx*(iy + ny*iz)``.
"""
from __future__ import annotations

import numpy as np

VACUUM, PERIODIC, INFLOW, OUTFLOW = 0, 1, 2, 3
FROZEN, COUPLED = 0, 1


def _cell_centres(n, l):
    return (np.arange(n) + 0.5) * (l / n)


def _base(dim, nx, ny, nz, ntheta, nphi, *, tol, rmax, steps, l=1.0):
    ns = nx * ny * nz
    return dict(dim=dim, nx=nx, ny=ny, nz=nz, ntheta=ntheta, nphi=nphi,
                lx=l, ly=l, lz=(l if dim == 3 else 1.0), c=1.0, a_r=1.0,
                cfl=0.5, tol=tol, rmax=rmax, steps=steps,
                bc_lo=[VACUUM] * 3, bc_hi=[VACUUM] * 3, material=FROZEN,
                kappa=np.ones(ns), rho=np.ones(ns), cv=np.ones(ns),
                T0=np.ones(ns), inflow=[])


def gaussian_pulse_cores(p, sigma=0.05, U0=1.0):
    """Isotropic Gaussian pulse centred in the unit square/cube, rank (1,1).

    Intensity (c/4pi) * U0/(2 pi sigma^2) * exp(-|x-xc|^2/(2 sigma^2)),
    sampled at cell centres, carried entirely by the spatial core.
    """
    xs = _cell_centres(p["nx"], p["lx"]) - 0.5 * p["lx"]
    ys = _cell_centres(p["ny"], p["ly"]) - 0.5 * p["ly"]
    r2 = xs[None, :] ** 2 + ys[:, None] ** 2
    if p["dim"] == 3:
        zs = _cell_centres(p["nz"], p["lz"]) - 0.5 * p["lz"]
        r2 = r2[None, :, :] + zs[:, None, None] ** 2
    amp = p["c"] / (4 * np.pi) * U0 / (2 * np.pi * sigma ** 2)
    X0 = (amp * np.exp(-r2 / (2 * sigma ** 2))).reshape(-1, 1)
    return X0, np.ones((1, p["ntheta"], 1)), np.ones((1, p["nphi"]))


def zero_cores(p):
    ns = p["nx"] * p["ny"] * p["nz"]
    return np.zeros((ns, 1)), np.ones((1, p["ntheta"], 1)), np.ones((1, p["nphi"]))


def face_cells(p, face):
    """Flattened spatial indices of the cells on ``face``, in face order.

    x-faces are indexed by iy + ny*iz, y-faces by ix + nx*iz, z-faces by
    ix + nx*iy.
    """
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
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


def _beam_profile(t):
    """Collimation profile in units of one ordinate spacing, cut at 3."""
    b = np.exp(-0.5 * t ** 2)
    b[np.abs(t) > 3.0] = 0.0
    return b


def crossing_beams(p, width=8, L=1.0):
    """Two collimated beams entering through the x-lo and y-lo faces.

    The profiles are expressed in ordinate-index units (one ordinate
    spacing = 1): polar offset from the equator (cos theta = 0) is
    ``l + 1/2 - ntheta/2``; azimuthal offset from the beam axis is
    ``p + 1/2 - p_axis`` wrapped to [-nphi/2, nphi/2), with p_axis = 0
    for +x and nphi/4 for +y.
    """
    nt, npf = p["ntheta"], p["nphi"]
    theta_w = _beam_profile(np.arange(nt) + 0.5 - nt / 2)

    def phi_prof(axis_index):
        t = np.arange(npf) + 0.5 - axis_index
        t = (t + npf / 2) % npf - npf / 2
        return _beam_profile(t)

    beams = []
    # x-lo face: rows iy in the central band
    fw = np.zeros(p["ny"] * p["nz"])
    band = np.arange(p["ny"] // 2 - width // 2, p["ny"] // 2 + width // 2)
    for iz in range(p["nz"]):
        fw[band + p["ny"] * iz] = L
    beams.append((0, fw, theta_w.copy(), phi_prof(0.0)))
    # y-lo face: columns ix in the central band
    fw = np.zeros(p["nx"] * p["nz"])
    band = np.arange(p["nx"] // 2 - width // 2, p["nx"] // 2 + width // 2)
    for iz in range(p["nz"]):
        fw[band + p["nx"] * iz] = L
    beams.append((2, fw, theta_w.copy(), phi_prof(npf / 4)))
    return beams


def gaussian_random_field(n, corr_len, seed, l=1.0):
    """Stationary Gaussian random field on the periodic n x n grid.

    White noise from ``default_rng(seed)`` filtered in Fourier space by the
    square root of the spectral density of the covariance
    exp(-r^2 / (2 corr_len^2)), then standardised to sample mean 0, std 1.
    """
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((n, n))
    k = 2 * np.pi * np.fft.fftfreq(n, d=l / n)
    k2 = k[None, :] ** 2 + k[:, None] ** 2
    filt = np.exp(-0.25 * k2 * corr_len ** 2)
    f = np.real(np.fft.ifft2(np.fft.fft2(xi) * filt))
    return (f - f.mean()) / f.std()


# --------------------------------------------------------------------------
# The named workloads
# --------------------------------------------------------------------------

def c1():
    """2-D parity case: 32^2, 8x16 ordinates, kappa = 1, T = 1 frozen,
    centred Gaussian pulse, vacuum, CFL 0.5, 10 steps, tolerance 1e-8."""
    p = _base(2, 32, 32, 1, 8, 16, tol=1e-8, rmax=0, steps=10)
    p["X0"], p["Th0"], p["Ph0"] = gaussian_pulse_cores(p)
    p["name"] = "c1_pulse_32sq_8x16"
    return p


def c2(steps=400):
    """Optically thin crossing beams: 256^2, 32x64 ordinates, kappa = 1e-3,
    cold medium (T = 0), two inflow beams, tolerance 1e-6, rank cap 64."""
    p = _base(2, 256, 256, 1, 32, 64, tol=1e-6, rmax=64, steps=steps)
    p["kappa"][:] = 1e-3
    p["T0"][:] = 0.0
    p["bc_lo"] = [INFLOW, INFLOW, VACUUM]
    p["inflow"] = crossing_beams(p)
    p["X0"], p["Th0"], p["Ph0"] = zero_cores(p)
    p["name"] = "c2_beams_256sq_32x64"
    return p


def c4(n=128, steps=200):
    """Optically thick two-region 3-D medium, coupled material (cv = 1)."""
    p = _base(3, n, n, n, 32, 64, tol=1e-6, rmax=128, steps=steps)
    xc = _cell_centres(n, 1.0)
    inside = (xc >= 0.25) & (xc <= 0.75)
    cube = inside[None, None, :] & inside[None, :, None] & inside[:, None, None]
    p["kappa"] = np.where(cube.reshape(-1), 1e3, 1.0)
    rng = np.random.default_rng(0)
    xi = rng.standard_normal(n ** 3)
    p["T0"] = np.clip(0.75 * (1 + 0.05 * xi), 0.5, 1.0)
    p["material"] = COUPLED
    ns = n ** 3
    p["X0"] = (p["c"] / (4 * np.pi) * p["a_r"] * p["T0"] ** 4).reshape(ns, 1)
    p["Th0"] = np.ones((1, 32, 1))
    p["Ph0"] = np.ones((1, 64))
    p["name"] = f"c4_thick_{n}cube_32x64"
    return p


def c5(n=128, steps=50):
    """Differentiation case: 128^2, 16x32, kappa = exp(GRF), pulse, T = 1."""
    p = _base(2, n, n, 1, 16, 32, tol=1e-6, rmax=128, steps=steps)
    p["kappa"] = np.exp(gaussian_random_field(n, 0.1, seed=0)).reshape(-1)
    p["X0"], p["Th0"], p["Ph0"] = gaussian_pulse_cores(p)
    p["ckpt_every"] = 10
    det = np.zeros((n, n))
    det[56 * n // 128:72 * n // 128, 72 * n // 128:88 * n // 128] = 1.0  # [iy, ix]
    p["detector"] = det.reshape(-1)
    p["name"] = f"c5_grad_{n}sq_16x32"
    return p


def relaxation(kappa=1.0, ntheta=8, nphi=16, steps=300):
    """Thermal relaxation, four cells (here 4 x 1 in 2-D, periodic)."""
    p = _base(2, 4, 1, 1, ntheta, nphi, tol=1e-6, rmax=0, steps=steps, l=4.0)
    p["ly"] = 1.0
    p["bc_lo"] = [PERIODIC, PERIODIC, VACUUM]
    p["bc_hi"] = [PERIODIC, PERIODIC, VACUUM]
    p["material"] = COUPLED
    p["kappa"][:] = kappa
    p["cv"][:] = 8.0
    p["T0"][:] = 2.0
    Er = 1.0  # a_r * T_r^4 with T_r = 1
    p["X0"] = np.full((4, 1), p["c"] * Er / (4 * np.pi))
    p["Th0"] = np.ones((1, ntheta, 1))
    p["Ph0"] = np.ones((1, nphi))
    p["name"] = f"relaxation_kappa{kappa:g}"
    return p


def random_tt(ns, ntheta, nphi, r1, r2, seed, decay=None):
    """Random TT cores (seeded); optional geometric decay of the bond-1
    spectrum ``decay**k`` imposed through the middle core."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ns, r1))
    Th = rng.standard_normal((r1, ntheta, r2))
    Ph = rng.standard_normal((r2, nphi))
    if decay is not None:
        Th *= (decay ** np.arange(r1))[:, None, None]
    return X, Th, Ph


def small_random(dim=2, nx=6, ny=5, nz=1, ntheta=4, nphi=8, r1=3, r2=2,
                 seed=0, bc="vacuum", material=FROZEN, tol=1e-6, rmax=0,
                 flux="upwind", s_plus=1.0, scatter=False, hll_beta=1.0):
    """Small seeded problem for parity tests: random positive material
    fields and random cores; ``bc`` in {vacuum, periodic, inflow, outflow,
    mixed} (mixed: inflow on x-lo, outflow on x-hi, vacuum on y-lo, outflow
    on y-hi, periodic along z); ``scatter`` adds a random positive
    scattering opacity."""
    rng = np.random.default_rng(seed)
    p = _base(dim, nx, ny, nz if dim == 3 else 1, ntheta, nphi, tol=tol,
              rmax=rmax, steps=3)
    ns = p["nx"] * p["ny"] * p["nz"]
    p["kappa"] = np.exp(rng.standard_normal(ns))
    p["rho"] = 0.5 + rng.random(ns)
    p["cv"] = 0.5 + rng.random(ns)
    p["T0"] = 0.5 + 0.5 * rng.random(ns)
    p["material"] = material
    X, Th, Ph = random_tt(ns, ntheta, nphi, r1, r2, seed + 1000)
    p["X0"], p["Th0"], p["Ph0"] = np.abs(X), np.abs(Th), np.abs(Ph)
    if bc == "periodic":
        p["bc_lo"] = [PERIODIC] * 3
        p["bc_hi"] = [PERIODIC] * 3
    elif bc == "inflow":
        p["bc_lo"] = [INFLOW, INFLOW, INFLOW if dim == 3 else VACUUM]
        p["bc_hi"] = [VACUUM, INFLOW, VACUUM]
        faces = [0, 2, 3] + ([4] if dim == 3 else [])
        for f in faces:
            nface = {0: ny * p["nz"], 2: nx * p["nz"], 3: nx * p["nz"],
                     4: nx * ny}[f]
            p["inflow"].append((f, rng.random(nface), rng.random(ntheta),
                                rng.random(nphi)))
    elif bc == "outflow":
        p["bc_lo"] = [OUTFLOW] * 3
        p["bc_hi"] = [OUTFLOW] * 3
    elif bc == "mixed":
        p["bc_lo"] = [INFLOW, VACUUM, PERIODIC]
        p["bc_hi"] = [OUTFLOW, OUTFLOW, PERIODIC]
        p["inflow"].append((0, rng.random(ny * p["nz"]), rng.random(ntheta), rng.random(nphi)))
    p["flux"] = flux
    p["s_plus"] = float(s_plus)
    p["hll_beta"] = float(hll_beta)
    if scatter:
        p["kappa_s"] = np.exp(rng.standard_normal(ns))
    p["name"] = f"small_{dim}d_{bc}_{flux}{'_scat' if scatter else ''}_s{seed}"
    return p


def gaussian_diffusion(n=64, ntheta=8, nphi=16, steps=200, t0=200.0, rho_kappa_s=1e3, A=1.0,
                       tol=1e-4):
    """Diffusion of a Gaussian pulse by isotropic scattering (reduced size).

    Domain [0, 5]^2 with the pulse at its centre, outflow boundaries,
    rho kappa_s = 1e3, no absorption, Rusanov flux with S+ = 0.  Initial
    intensity I = c E(0) / (4 pi), isotropic, with the diffusion solution
    E(t) = A / (4 pi D (t0 + t)) exp(-r^2 / (4 D (t0 + t))), D = c / (3 rho kappa_s)
    at t = 0 (rank (1, 1)).  Frozen temperature at zero."""
    p = _base(2, n, n, 1, ntheta, nphi, tol=tol, rmax=0, steps=steps, l=5.0)
    p["bc_lo"] = [OUTFLOW, OUTFLOW, VACUUM]
    p["bc_hi"] = [OUTFLOW, OUTFLOW, VACUUM]
    ns = n * n
    p["kappa"][:] = 0.0
    p["kappa_s"] = np.full(ns, rho_kappa_s)
    p["T0"][:] = 0.0
    p["flux"] = "rusanov"
    p["s_plus"] = 0.0
    D = p["c"] / (3.0 * rho_kappa_s)
    xs = _cell_centres(n, 5.0) - 2.5
    r2 = xs[None, :] ** 2 + xs[:, None] ** 2
    E0 = A / (4 * np.pi * D * t0) * np.exp(-r2 / (4 * D * t0))
    p["X0"] = (p["c"] * E0 / (4 * np.pi)).reshape(ns, 1)
    p["Th0"] = np.ones((1, ntheta, 1))
    p["Ph0"] = np.ones((1, nphi))
    p["diffusion"] = dict(D=D, t0=t0, A=A)
    p["name"] = f"gaussian_diffusion_{n}sq_{ntheta}x{nphi}"
    return p


def hohlraum(n=64, ntheta=16, nphi=32, tol=1e-4, rmax=0, t_end=0.75):
    """Hohlraum (Sec. 5.1) at reduced size: domain [0, 2]^2, vacuum (no
    opacity, no emission), isotropic intensity I = 1 entering through the
    x-lo and y-lo faces (Dirichlet inflow g = 1 for every ordinate; the
    upwind stencil reads it only for entering directions), the other faces
    vacuum.  Zero initial state; CFL 0.5, so Delta t = 1/n and the run has
    t_end n steps (n a multiple of 4 for t_end = 0.75)."""
    steps = int(round(t_end * n))
    p = _base(2, n, n, 1, ntheta, nphi, tol=tol, rmax=rmax, steps=steps, l=2.0)
    p["bc_lo"] = [INFLOW, INFLOW, VACUUM]
    p["bc_hi"] = [VACUUM, VACUUM, VACUUM]
    ns = n * n
    p["kappa"][:] = 0.0
    p["T0"][:] = 0.0
    p["X0"], p["Th0"], p["Ph0"] = zero_cores(p)
    p["inflow"] = [(0, np.ones(n), np.ones(ntheta), np.ones(nphi)),
                   (2, np.ones(n), np.ones(ntheta), np.ones(nphi))]
    p["hohlraum"] = dict(t=steps * p["cfl"] * (2.0 / n) / p["c"])
    p["name"] = f"hohlraum_{n}sq_{ntheta}x{nphi}"
    return p


def line_source(n=64, ntheta=16, nphi=32, tol=1e-4, rmax=200, t_end=0.5, omega=0.03, U0=1.0):
    """Line source (Sec. 5.4) at reduced size: domain [-1.1, 1.1]^2 (extent
    2.2, the pulse at its centre), vacuum everywhere, no opacity or emission,
    CFL 0.4, an isotropic Gaussian pulse of width omega carrying U0 (rank
    (1, 1)).  t_end = 0.5 keeps the front (and the upwind scheme's smearing
    of it) inside the domain, so the energy leaves only through truncation."""
    p = _base(2, n, n, 1, ntheta, nphi, tol=tol, rmax=rmax, steps=0, l=2.2)
    p["cfl"] = 0.4
    p["kappa"][:] = 0.0
    p["T0"][:] = 0.0
    p["X0"], p["Th0"], p["Ph0"] = gaussian_pulse_cores(p, sigma=omega, U0=U0)
    dt = p["cfl"] * (2.2 / n) / p["c"]
    p["steps"] = int(round(t_end / dt))
    p["line_source"] = dict(U0=U0, omega=omega, t=p["steps"] * dt)
    p["name"] = f"line_source_{n}sq_{ntheta}x{nphi}"
    return p


def rounding_bench_cores(p, r1=64, r2=12, seed=2, decades_per_8=1.0):
    """Seeded synthetic state on the crossing-beam shape for the rounding
    benchmark: orthonormal X (N_s x r1), orthonormal Phi rows (r2 x N_phi)
    and a middle core whose bond-1 unfolding is diag(s) Q with Q having
    orthonormal rows, so the bond-1 singular values are s_k = 10^(-k/8)
    (k = 0 .. r1-1).  One step of the crossing-beam workload from this state
    concatenates it to ranks (5 r1 + 2, 5 r2 + 2) = (322, 62) before
    rounding."""
    rng = np.random.default_rng(seed)
    ns = p["nx"] * p["ny"] * p["nz"]
    nt, npf = p["ntheta"], p["nphi"]
    X = np.linalg.qr(rng.standard_normal((ns, r1)))[0]
    Ph = np.linalg.qr(rng.standard_normal((npf, r2)))[0].T
    Q = np.linalg.qr(rng.standard_normal((nt * r2, r1)))[0].T  # r1 x (nt r2), orthonormal rows
    s = 10.0 ** (-np.arange(r1) * decades_per_8 / 8.0)
    Th = (s[:, None] * Q).reshape(r1, nt, r2)
    return X, Th, Ph


def gaussian_test_matrices(ntheta, nphi, r1t, r2t, seed):
    """Seeded standard Gaussian test matrices for randomized rounding: Omega_1
    of shape (ntheta nphi, r1t) and Omega_2 of shape (nphi, r2t)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ntheta * nphi, r1t)), rng.standard_normal((nphi, r2t))

