"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to a closed form, an invariant, a value
printed in the paper, or a library routine (SVD / QR / ODE integrator), so
that a dropped term, wrong sign, wrong neighbour or transposed operand in
the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, full, tt, rounding, metrics, material, adjoint, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("nt,npf", [(2, 4), (8, 16), (32, 64)])
def test_quadrature_closed_forms(nt, npf):
    mu, w, phi, v = quadrature.ordinates(nt, npf)
    dom = quadrature.solid_angles(nt, npf)
    assert abs(dom.sum() - 4 * np.pi) < 1e-13          # sum dOmega = 4 pi (Sec. 3)
    st, cp, sp, mu2 = quadrature.direction_cosines(nt, npf)
    for n in (np.outer(st, cp), np.outer(st, sp), np.outer(mu2, np.ones(npf))):
        assert abs((dom * n).sum()) < 1e-13            # no net flux direction
    # midpoint rule on int mu^2 dmu over [-1,1]: 2/3 (1 - 1/Nt^2) exactly
    assert abs(w @ mu ** 2 - 2.0 / 3.0 * (1 - 1.0 / nt ** 2)) < 1e-14
    # midpoint rule over a full period is exact for cos^2: pi
    assert abs(v @ np.cos(phi) ** 2 - np.pi) < 1e-13
    assert np.all(np.abs(np.outer(st, cp)) > 0) and np.all(np.abs(mu2) > 0)


# ------------------------------------------------------------ full transport
def _line_problem(nx=16, nt=4, npf=8, bc="periodic", kappa=0.0):
    p = wl._base(2, nx, 1, 1, nt, npf, tol=0.0, rmax=0, steps=1)
    p["ly"] = p["lx"] / nx
    p["bc_lo"] = [wl.PERIODIC if bc == "periodic" else wl.INFLOW, wl.PERIODIC, 0]
    p["bc_hi"] = [wl.PERIODIC if bc == "periodic" else wl.VACUUM, wl.PERIODIC, 0]
    p["kappa"][:] = kappa
    p["T0"][:] = 0.0
    return p


def test_upwind_fourier_amplification():
    """Upwind scheme on a periodic line: a Fourier mode evolves by the
    textbook amplification factor g = 1 - nu (1 - e^{-ih}) (nu >= 0) or
    g = 1 - nu (e^{ih} - 1) (nu < 0), nu = lam n_x; checked over 5 steps."""
    p = _line_problem()
    s = Setup(p)
    k = 3
    x = (np.arange(s.nx) + 0.5) * s.dx
    theta = 2 * np.pi * k * x
    h = 2 * np.pi * k * s.dx
    I = np.broadcast_to(np.cos(theta)[None, None, :, None, None],
                        (1, 1, s.nx, s.nt, s.np_)).copy()
    m = 5
    for _ in range(m):
        I = full.transport(I, s)
    nu = s.lam[0] * np.outer(s.sin_t, s.cos_p)
    g = np.where(nu >= 0, 1 - nu * (1 - np.exp(-1j * h)), 1 - nu * (np.exp(1j * h) - 1))
    expect = np.real(g[None, :, :] ** m * np.exp(1j * theta)[:, None, None])
    assert np.max(np.abs(I[0, 0] - expect)) < 1e-13


def test_upwind_inflow_steady_state():
    """Constant inflow g on the x-lo face, absorption d: the scheme's steady
    state is I_i = q^{i+1} g with q = d nu / (1 - d (1 - nu)) for n_x > 0 and
    zero for n_x < 0 (vacuum on the far face)."""
    nx, nt, npf = 6, 4, 8
    p = _line_problem(nx=nx, nt=nt, npf=npf, bc="inflow", kappa=0.7)
    p["inflow"] = [(0, np.array([1.3]), np.ones(nt), np.ones(npf))]
    p["cfl"] = 0.9
    s = Setup(p)
    I = np.zeros((1, 1, nx, nt, npf))
    for _ in range(4000):
        I, _, _ = full.step(I, s.T0, s)
    nu = s.lam[0] * np.outer(s.sin_t, s.cos_p)
    d = 1.0 / (1.0 + s.c * s.dt * 0.7)
    q = d * nu / (1 - d * (1 - nu))
    i = np.arange(nx)[:, None, None]
    expect = np.where(nu[None] > 0, 1.3 * q[None] ** (i + 1), 0.0)
    assert np.max(np.abs(I[0, 0] - expect)) < 1e-12


def test_transport_conserves_per_ordinate_and_stays_positive():
    p = wl.small_random(bc="periodic", seed=7)
    p["kappa"][:] = 0.0
    s = Setup(p)
    I = full.initial_intensity(s)
    I1 = full.transport(I, s)
    assert np.allclose(I1.sum(axis=(0, 1, 2)), I.sum(axis=(0, 1, 2)), rtol=1e-14, atol=0)
    assert I1.min() >= 0 and I1.max() <= I.max() * (1 + 1e-15)  # convex combination (CFL)


def test_energy_of_isotropic_field():
    p = wl.small_random(seed=3)
    s = Setup(p)
    I = np.full(s.grid_shape() + (s.nt, s.np_), 2.5)
    assert np.allclose(full.energy(I, s), 4 * np.pi * 2.5 / s.c, rtol=1e-14)


# ------------------------------------------------------------------ material
def test_newton_root_and_identity():
    p = wl.small_random(material=wl.COUPLED, seed=11)
    s = Setup(p)
    rng = np.random.default_rng(5)
    Estar = rng.random(s.ns) * 3
    d, sv, Tdag = material.source_coefficients(Estar, s.T0, s)
    g = s.c * s.dt * s.kappa / s.cv / (1 + s.c * s.dt * s.rho * s.kappa)
    f = Tdag - s.T0 + g * (s.a_r * Tdag ** 4 - Estar)
    assert np.max(np.abs(f)) < 1e-14 * np.max(Tdag)
    # untruncated step: T^{m+1} = T_dag exactly (energy-conserving update)
    cat, T1, info = tt.step_untruncated(p["X0"], p["Th0"], p["Ph0"], s.T0, s)
    assert np.allclose(T1, info["Tdag"], rtol=1e-12, atol=1e-13)


def _relaxation_run(kappa, steps, dt=0.01):
    p = wl.relaxation(kappa=kappa, steps=steps)
    p["dt"] = dt
    s = Setup(p)
    Ts, Es, ranks = [], [], []

    def cb(m, cores, T, info):
        Ts.append(T.copy()); Es.append(info["Enew"].copy())
        ranks.append((cores[0].shape[1], cores[2].shape[0]))
    tt.run(s, steps, callback=cb)
    return np.array(Ts), np.array(Es), ranks


def test_relaxation_paper_example():
    """Thermal relaxation (Sec. 5.2): rho c_v T + a_r T_r^4 is conserved,
    kappa = 1e6 equilibrates in one step to the root of 8T + T^4 = 17,
    ranks stay (1, 1), and kappa = 1 converges to the ODE solution at first
    order in dt (backward Euler) when going from 300 to 600 steps to t = 3."""
    Ts, Es, ranks = _relaxation_run(1e6, 3)
    roots = np.roots([1, 0, 0, 8, -17])
    Teq = float(np.real(roots[(np.abs(roots.imag) < 1e-12) & (roots.real > 0)][0]))
    assert abs(Teq - 1.497) < 1e-3
    assert np.allclose(Ts[0], Teq, rtol=1e-3)
    assert np.allclose(8 * Ts + Es, 17.0, rtol=1e-12)
    assert all(r == (1, 1) for r in ranks)
    from scipy.integrate import solve_ivp

    def rhs(t, y):
        T, E = y
        q = 1.0 * (T ** 4 - E)
        return [-q / 8.0, q]
    sol = solve_ivp(rhs, (0, 3), [2.0, 1.0], rtol=1e-12, atol=1e-14, dense_output=True)
    errs = []
    for steps in (300, 600):
        Ts, Es, ranks = _relaxation_run(1.0, steps, dt=3.0 / steps)
        assert all(r == (1, 1) for r in ranks)
        assert np.allclose(8 * Ts + Es, 17.0, rtol=1e-12)
        Tode = sol.sol(3.0 / steps * np.arange(1, steps + 1))[0]
        errs.append(np.max(np.abs(Ts[:, 0] - Tode)))
    assert errs[0] < 5e-3
    assert 1.8 < errs[0] / errs[1] < 2.2


# ------------------------------------------------------------------ rounding
def _orth(n, r, rng):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _spectrum_tt(ns, nt, npf, s, rng):
    """Orthonormal X, orthonormal Phi rows and Theta_{a,l,b} = s_a d_ab
    d_{l, a mod nt}: both bond unfoldings have singular values s."""
    r = s.size
    X = _orth(ns, r, rng)
    Ph = _orth(npf, r, rng).T
    Th = np.zeros((r, nt, r))
    for a in range(r):
        Th[a, a % nt, a] = s[a]
    return X, Th, Ph


def test_gram_svd_recovers_constructed_spectrum_and_ranks():
    rng = np.random.default_rng(0)
    s = 10.0 ** (-np.arange(10) / 1.5)
    X, Th, Ph = _spectrum_tt(60, 5, 16, s, rng)
    tol = 1e-4
    (Xn, Thn, Phn), (i1, i2) = rounding.round_gram(X, Th, Ph, tol, 0)
    assert np.allclose(i1["sigma"][:s.size], s, rtol=1e-10, atol=1e-12)
    delta2 = tol ** 2 * np.sum(s ** 2) / 2
    tail = np.array([np.sum(s[k:] ** 2) for k in range(s.size + 1)])
    expect = int(np.argmax(tail <= delta2))
    assert Xn.shape[1] == expect and Phn.shape[0] == expect
    assert np.allclose(i2["sigma"][:expect], s[:expect], rtol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gram_svd_equals_dense_and_ttsvd(seed):
    """Gram-SVD, TT-SVD (QR) and dense SVD truncate the same unfoldings, so
    they agree up to rounding where the spectrum has a gap at the cut."""
    rng = np.random.default_rng(seed)
    X, Th, Ph = wl.random_tt(40, 6, 12, 8, 5, seed, decay=0.15)
    T = metrics.reconstruct(X, Th, Ph)
    tol = 1e-5
    g = rounding.round_gram(X, Th, Ph, tol, 0)[0]
    d = rounding.round_dense(T, tol, 0)
    q = rounding.round_ttsvd(X, Th, Ph, tol, 0)
    assert g[0].shape[1] == d[0].shape[1] == q[0].shape[1]
    assert g[2].shape[0] == d[2].shape[0] == q[2].shape[0]
    assert metrics.rel_diff(g, d) < 1e-9
    assert metrics.rel_diff(q, d) < 1e-11
    # error bound of the tolerance split, and orthonormal left factor
    assert np.linalg.norm(metrics.reconstruct(*g) - T) <= tol * np.linalg.norm(T) * (1 + 1e-6)
    assert np.allclose(g[0].T @ g[0], np.eye(g[0].shape[1]), atol=1e-10)


def test_rank_one_exact_self_sum_and_zero():
    p = wl.c1()
    X, Th, Ph = p["X0"], p["Th0"], p["Ph0"]
    (Xn, Thn, Phn), _ = rounding.round_gram(X, Th, Ph, 1e-8, 0)
    assert (Xn.shape[1], Phn.shape[0]) == (1, 1)
    T = metrics.reconstruct(X, Th, Ph)
    assert np.linalg.norm(metrics.reconstruct(Xn, Thn, Phn) - T) < 1e-14 * np.linalg.norm(T)
    # T + T by concatenation rounds back to rank(T), values 2T
    A = wl.random_tt(30, 4, 8, 3, 2, 9)
    cat = tt.concat([A, A])
    (Xs, Ts, Ps), _ = rounding.round_gram(*cat, 1e-10, 0)
    assert (Xs.shape[1], Ps.shape[0]) == (3, 2)
    TA = metrics.reconstruct(*A)
    assert np.linalg.norm(metrics.reconstruct(Xs, Ts, Ps) - 2 * TA) < 1e-12 * np.linalg.norm(TA)
    # zero tensor -> rank (1,1), zero cores
    (Xz, Tz, Pz), _ = rounding.round_gram(np.zeros((20, 3)), np.ones((3, 4, 2)), np.ones((2, 8)), 1e-6, 0)
    assert (Xz.shape[1], Pz.shape[0]) == (1, 1) and not Xz.any()


def test_cluster_and_cap_rules():
    sig = np.array([3.0, 2.0, 2.0, 1.0, 1e-9])
    # tolerance would cut inside the degenerate pair: extended to the end
    assert rounding.select_rank(sig, 1.5, 0) == 3
    # cap inside the pair: cut before it
    assert rounding.select_rank(sig, 1e-30, 2) == 1
    assert rounding.select_rank(sig, 1e-30, 4) == 4
    assert rounding.select_rank(np.zeros(3), 0.0, 0) == 1
    # a pair split only at the Gram resolution (R u sigma_1^2 / sigma) is a cluster
    pair = np.array([1.0, 1e-3, 1e-6 + 4e-11, 1e-6, 1e-9])
    d2 = 1.01 * (1e-6 ** 2 + 1e-18)
    assert rounding.select_rank(pair, d2, 0) == 3
    assert rounding.select_rank(pair, d2, 0, noise=42 * rounding.U) == 4
    # a chain of ties is not followed below the resolution sqrt(noise) sigma_1:
    # with noise 1e-10 the floor is 1e-5, the tail rule keeps 2, the tie with
    # 1.1e-5 (resolved) adds one, and the tie with 9e-6 (unresolved) stops it
    chain = np.array([1.0, 1.3e-5, 1.1e-5, 9e-6, 7e-6, 5e-6])
    assert rounding.select_rank(chain, 3e-10, 0) == 2
    assert rounding.select_rank(chain, 3e-10, 0, noise=1e-10) == 3
    # closest comparisons: tail(2) at 0.92 delta^2 and the two resolution tests at 0.9, 1.1 floor
    assert abs(rounding.rank_margin(chain, 3e-10, 0, noise=1e-10) - 0.08) < 1e-12


# ---------------------------------------------------------------- TT vs full
@pytest.mark.parametrize("kw", [dict(seed=1), dict(bc="periodic", seed=2),
                                dict(bc="inflow", seed=3, material=wl.COUPLED),
                                dict(dim=3, nx=4, ny=3, nz=5, bc="inflow", seed=4, material=wl.COUPLED),
                                dict(dim=3, nx=4, ny=3, nz=4, bc="periodic", seed=5)])
def test_tt_step_without_truncation_is_the_full_grid_step(kw):
    p = wl.small_random(**kw)
    s = Setup(p)
    I1, T1, _ = full.step(full.initial_intensity(s), s.T0, s)
    cat, T1t, _ = tt.step_untruncated(p["X0"], p["Th0"], p["Ph0"], s.T0, s)
    F = metrics.reconstruct(*cat).reshape(I1.shape)
    assert np.linalg.norm(F - I1) < 1e-13 * np.linalg.norm(I1)
    (Xn, Thn, Phn), T2, _ = tt.step(p["X0"], p["Th0"], p["Ph0"], s.T0, s, 0.0, 0)
    F2 = metrics.reconstruct(Xn, Thn, Phn).reshape(I1.shape)
    assert np.linalg.norm(F2 - I1) < 1e-12 * np.linalg.norm(I1)


def test_conservation_periodic_no_absorption():
    p = wl.small_random(bc="periodic", seed=12, nx=8, ny=6)
    p["kappa"][:] = 0.0
    p["T0"][:] = 0.0
    s = Setup(p)
    X, Th, Ph = p["X0"], p["Th0"], p["Ph0"]
    tol = 1e-6
    E0 = tt.energy(X, Th, Ph, s).sum()
    for _ in range(5):
        cat, _, info = tt.step_untruncated(X, Th, Ph, s.T0, s)
        assert abs(info["Enew"].sum() - E0) < 1e-14 * abs(E0) * 10
        nrm = metrics.tt_norm(*cat)
        (X, Th, Ph), _ = rounding.round_gram(*cat, tol, 0)
        E1 = tt.energy(X, Th, Ph, s).sum()
        bound = tol * nrm * np.sqrt(s.ns) * 4 * np.pi / np.sqrt(s.nt * s.np_) / s.c
        assert abs(E1 - E0) <= bound
        E0 = E1


def test_c1_symmetry_of_the_square():
    """C1 (square, centred pulse, symmetric quadrature): E is invariant under
    the 8 symmetries of the square up to the truncation level."""
    p = wl.c1()
    p["tol"] = 1e-6
    s = Setup(p)
    (X, Th, Ph), _, hist = tt.run(s, 6)
    E = tt.energy(X, Th, Ph, s).reshape(32, 32)
    ref = np.abs(E).max()
    for img in (E.T, E[::-1], E[:, ::-1], E[::-1, ::-1], E.T[::-1], E.T[:, ::-1], E.T[::-1, ::-1]):
        assert np.max(np.abs(img - E)) < 1e-5 * ref


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("kw", [dict(seed=1), dict(bc="periodic", seed=2),
                                dict(dim=3, nx=3, ny=4, nz=3, seed=3)])
def test_transport_adjoint_dot_product(kw):
    s = Setup(wl.small_random(**kw))
    rng = np.random.default_rng(1)
    shp = s.grid_shape() + (s.nt, s.np_)
    x, y = rng.standard_normal(shp), rng.standard_normal(shp)
    lhs = np.sum(adjoint.transport_linear(x, s) * y)
    rhs = np.sum(x * adjoint.transport_adjoint(y, s))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_full_grid_gradient_matches_finite_differences():
    p = wl.small_random(nx=7, ny=6, seed=21)
    p["material"] = wl.FROZEN
    s = Setup(p)
    det = np.zeros(s.ns); det[[10, 11, 17, 18]] = 1.0
    L, g = adjoint.grad_full(s, 4, det)
    cells = [3, 10, 17, 25, 40]
    gfd = adjoint.grad_fd(lambda k: adjoint.loss_full(s, k, 4, det), s.kappa, cells)
    assert np.allclose(g[cells], gfd, rtol=1e-6, atol=1e-10 * np.abs(g).max())


# ------------------------------------------------------------------ metrics
def test_compression_reproduces_printed_values():
    with open(os.path.join(GOLDEN, "compression_pins.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        C = metrics.compression(c["ns"], c["nt"], c["np"], c["r1"], c["r2"])
        assert abs(C - c["printed"]) <= c["rel"] * c["printed"], c["what"]


def test_tt_difference_norm_matches_dense():
    A = wl.random_tt(50, 4, 6, 3, 2, 1)
    B = wl.random_tt(50, 4, 6, 2, 3, 2)
    dn = np.linalg.norm(metrics.reconstruct(*A) - metrics.reconstruct(*B))
    assert abs(metrics.tt_diff_norm(A, B) - dn) < 1e-12 * dn
    assert abs(metrics.rel_diff(A, B, dense_limit=0) - metrics.rel_diff(A, B)) < 1e-12


def test_rank_margin_flags_boundary_decisions():
    """rank_margin is small exactly when a comparison of the rank rule sits
    on its threshold: tail(k) = delta^2, or a tie test at its threshold."""
    sig = np.array([1.0, 0.5, 0.1, 0.01])
    # tail(2) = 0.0101 exactly on delta^2 -> margin 0
    assert rounding.rank_margin(sig, 0.0101, 0) < 1e-12
    # far from every threshold
    m = rounding.rank_margin(sig, 0.02, 0)
    assert m > 0.4
    # a tie test sitting on eta sigma_1: sigma_2 - sigma_3 = eta sigma_1
    sig2 = np.array([1.0, 0.5, 0.5 - 1e-12, 1e-3])
    assert rounding.rank_margin(sig2, 0.3, 0) < 1e-3  # r = 2 before the tie test


# ------------------------------------------------- clip to the row rank (Q11)
def _noisy(scale, seed):
    """A symmetric perturbation of ``scale`` unit roundoffs of max|G| (a
    stand-in for the rounding error of another summation order)."""
    r = np.random.default_rng(seed)

    def pert(G):
        E = r.uniform(-1.0, 1.0, G.shape)
        return G + scale * rounding.U * np.abs(G).max() * 0.5 * (E + E.T)
    return pert


@pytest.mark.parametrize("scale", [0, 30, 300])
def test_kept_eigenpairs_never_exceed_the_row_rank(scale):
    """G_B at bond 2 is Phi Phi^T of order r2 = 20 built from N_phi = 8
    columns, so it has rank <= 8 and every further eigenpair is rounding
    noise.  Under Gram noise of up to 300 u max|G| the kept counts stay
    within the row ranks, the TT ranks within the mode bounds (r2 <= N_phi,
    r1 <= min(N_s, N_theta N_phi)), and the result is the dense-SVD rounding
    of the same tensor (App. A.2 vs. the SVD of the unfoldings).  Without
    the cut to the row rank the noise pairs are kept and r2 exceeds N_phi."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 6))
    Th = rng.standard_normal((6, 4, 20))
    Ph = rng.standard_normal((20, 8))
    T = metrics.reconstruct(X, Th, Ph)
    (Xg, Tg, Pg), (i1, i2) = rounding.round_gram(X, Th, Ph, 1e-8, 0,
                                                 perturb=_noisy(scale, 1) if scale else None)
    assert i1["kA"] <= 40 and i1["kB"] <= 4 * 8
    assert i2["kA"] <= Xg.shape[1] * 4 and i2["kB"] <= 8
    assert Xg.shape[1] <= min(40, 32) and Pg.shape[0] <= 8
    d = rounding.round_dense(T, 1e-8, 0)
    assert (Xg.shape[1], Pg.shape[0]) == (d[0].shape[1], d[2].shape[0])
    assert metrics.rel_diff((Xg, Tg, Pg), d) < 1e-12


def test_c1_bond2_gram_beyond_its_row_rank():
    """C1 after three steps: the concatenated angular core has R2 > N_phi =
    16 rows, so G_R3 = Phi_cat Phi_cat^T is singular beyond rank 16.  The
    kept count of its side is at most 16 and the step's rounding equals the
    dense-SVD rounding of the untruncated step."""
    p = wl.c1()
    p["tol"] = 1e-6
    s = Setup(p)
    (X, Th, Ph), _, _ = tt.run(s, 3)
    cat, _, _ = tt.step_untruncated(X, Th, Ph, s.T0, s)
    assert cat[2].shape[0] > 16
    (Xg, Tg, Pg), (i1, i2) = rounding.round_gram(*cat, p["tol"], 0)
    assert i2["kB"] <= 16 and Pg.shape[0] <= 16
    d = rounding.round_dense(metrics.reconstruct(*cat), p["tol"], 0)
    assert (Xg.shape[1], Pg.shape[0]) == (d[0].shape[1], d[2].shape[0])
    assert metrics.rel_diff((Xg, Tg, Pg), d) < 1e-9


# --------------------------------------------- the two-rounding schedule (Sec. 4.2)
@pytest.mark.parametrize("kw", [dict(seed=1), dict(bc="inflow", seed=3, material=wl.COUPLED),
                                dict(dim=3, nx=4, ny=3, nz=4, bc="periodic", seed=5)])
def test_twice_schedule_without_truncation_is_the_full_grid_step(kw):
    """Rounding after the transport sum and again after the source update
    (Sec. 4.2) changes nothing when nothing is truncated: with tol = 0 the
    two-rounding step equals the full-grid step and the one-rounding step,
    temperature included."""
    p = wl.small_random(**kw)
    s = Setup(p)
    I1, T1, _ = full.step(full.initial_intensity(s), s.T0, s)
    X0, Th0, Ph0 = p["X0"], p["Th0"], p["Ph0"]
    tw, Tt, info = tt.step(X0, Th0, Ph0, s.T0, s, 0.0, 0, schedule="twice")
    on, To, _ = tt.step(X0, Th0, Ph0, s.T0, s, 0.0, 0, schedule="once")
    assert len(info["round"]) == 2
    F = metrics.reconstruct(*tw).reshape(I1.shape)
    assert np.linalg.norm(F - I1) < 1e-12 * np.linalg.norm(I1)
    assert metrics.rel_diff(tw, on) < 1e-12
    assert np.max(np.abs(Tt - T1)) < 1e-12 * np.max(np.abs(T1))
    assert np.max(np.abs(Tt - To)) < 1e-12 * np.max(np.abs(T1))


def test_twice_schedule_error_bound():
    """With truncation, each of the two roundings moves its tensor by at most
    tol times that tensor's norm (App. A note on rank truncation), and the
    source update scales by d <= 1: the two-rounding step is within
    tol (max d ||I*|| + ||I^{m+1}||) of the full-grid step, and its first
    rounding sees only the transport blocks (ranks B r + n_bc)."""
    p = wl.small_random(nx=8, ny=7, ntheta=6, nphi=12, r1=4, r2=3, seed=9, bc="inflow")
    s = Setup(p)
    tol = 1e-3
    I0 = full.initial_intensity(s)
    Istar = full.transport(I0, s)
    I1, _, _ = full.step(I0, s.T0, s)
    tw, _, info = tt.step(p["X0"], p["Th0"], p["Ph0"], s.T0, s, tol, 0, schedule="twice")
    R1 = info["round"][0][0]["R"]
    assert R1 == 5 * 4 + len(p["inflow"])
    err = np.linalg.norm(metrics.reconstruct(*tw).reshape(I1.shape) - I1)
    dmax = np.max(1.0 / (1.0 + s.c * s.dt * s.rho * s.kappa))
    assert err <= tol * (dmax * np.linalg.norm(Istar) + np.linalg.norm(I1)) * (1 + 1e-9)


# --------------------------------------- Rusanov flux, outflow, scattering
def test_rusanov_fourier_amplification():
    """Rusanov flux on a periodic line (eq. rusanov_flux_toro with piecewise
    constant states): a Fourier mode evolves by the textbook factor
    g = 1 - i nu sin h - lam s (1 - cos h), nu = lam n_x, s = S+ / c."""
    for s_plus in (1.0, 0.3, 0.0):
        p = _line_problem()
        p["flux"], p["s_plus"] = "rusanov", s_plus
        s = Setup(p)
        k = 3
        x = (np.arange(s.nx) + 0.5) * s.dx
        theta = 2 * np.pi * k * x
        h = 2 * np.pi * k * s.dx
        I = np.broadcast_to(np.cos(theta)[None, None, :, None, None],
                            (1, 1, s.nx, s.nt, s.np_)).copy()
        m = 4
        for _ in range(m):
            I = full.transport(I, s)
        lam = s.lam[0]
        nu = lam * np.outer(s.sin_t, s.cos_p)
        g = 1 - 1j * nu * np.sin(h) - lam * s_plus * (1 - np.cos(h))
        expect = np.real(g[None, :, :] ** m * np.exp(1j * theta)[:, None, None])
        assert np.max(np.abs(I[0, 0] - expect)) < 1e-13


@pytest.mark.parametrize("flux", ["upwind", "rusanov"])
def test_outflow_boundaries(flux):
    """Outflow ghost cells copy the adjacent interior cell (Sec. 4.5): a
    uniform field with outflow on every face is a steady state of the
    transport step.  With outflow on x-lo and vacuum on x-hi (periodic in
    y), upwind changes only the last column, and there only the directions
    entering through the vacuum face (n_x < 0), by the factor 1 + lam n_x."""
    p = _line_problem(nx=7)
    p["flux"] = flux
    p["bc_lo"] = [wl.OUTFLOW, wl.OUTFLOW, 0]
    p["bc_hi"] = [wl.OUTFLOW, wl.OUTFLOW, 0]
    s = Setup(p)
    I = np.full((1, 1, s.nx, s.nt, s.np_), 1.7)
    assert np.max(np.abs(full.transport(I, s) - I)) < 1e-15
    if flux == "upwind":
        p["bc_hi"] = [wl.VACUUM, wl.OUTFLOW, 0]
        p["bc_lo"] = [wl.OUTFLOW, wl.OUTFLOW, 0]
        s = Setup(p)
        I1 = full.transport(I, s)
        nx_ = np.outer(s.sin_t, s.cos_p)
        assert np.max(np.abs(I1[0, 0, :-1] - 1.7)) < 1e-15
        expect = np.where(nx_ < 0, 1.7 * (1 + s.lam[0] * nx_), 1.7)
        assert np.max(np.abs(I1[0, 0, -1] - expect)) < 1e-15


def test_scattering_relaxes_to_isotropy():
    """Pure isotropic scattering (kappa_a = 0) in a uniform medium, eq.
    couple_a: J^{m+1} = J*, so I^{m+1} = d I* + (1 - d) J* with
    d = 1 / (1 + c dt rho kappa_s): the mean intensity is kept and the
    anisotropic part decays by d per step."""
    p = _line_problem(nx=4, bc="periodic", kappa=0.0)
    p["kappa_s"] = np.full(4, 2.5)
    s = Setup(p)
    rng = np.random.default_rng(0)
    ang = rng.random((s.nt, s.np_))
    I = np.broadcast_to(ang[None, None, None], (1, 1, 4, s.nt, s.np_)).copy()
    J0 = np.sum(ang * s.domega) / (4 * np.pi)
    d = 1.0 / (1.0 + s.c * s.dt * 2.5)
    for m in range(1, 4):
        I, _, _ = full.step(I, s.T0, s)
        expect = J0 + d ** m * (ang - J0)
        assert np.max(np.abs(I[0, 0] - expect[None])) < 1e-14


def test_scattering_conserves_energy_and_keeps_the_temperature_equation():
    """Scattering moves no energy between radiation and material: with
    kappa_a = 0, periodic boundaries, the total radiation energy of a step
    is constant; with absorption and coupled material, adding kappa_s leaves
    T_dag unchanged (eq. couple_b after eliminating J^{m+1}) and total energy
    is conserved."""
    p = wl.small_random(bc="periodic", seed=13, scatter=True)
    p["kappa"][:] = 0.0
    s = Setup(p)
    I = full.initial_intensity(s)
    E0 = full.energy(I, s).sum()
    for _ in range(3):
        I, _, _ = full.step(I, s.T0, s)
        assert abs(full.energy(I, s).sum() - E0) < 1e-13 * E0
    q = wl.small_random(bc="periodic", seed=14, material=wl.COUPLED, scatter=True)
    sq = Setup(q)
    q0 = dict(q)
    q0["kappa_s"] = np.zeros_like(q["kappa_s"])
    s0 = Setup(q0)
    I = full.initial_intensity(sq)
    _, T1, info = full.step(I, sq.T0, sq)
    _, _, info0 = full.step(I, s0.T0, s0)
    assert np.max(np.abs(info["Tdag"] - info0["Tdag"])) < 1e-14 * np.max(info0["Tdag"])
    tot0 = full.energy(I, sq).sum() + np.sum(sq.rho * sq.cv * sq.T0)
    I1, T1, _ = full.step(I, sq.T0, sq)
    tot1 = full.energy(I1, sq).sum() + np.sum(sq.rho * sq.cv * T1)
    assert abs(tot1 - tot0) < 1e-13 * tot0


NEW_OPERATOR_CASES = [dict(bc="outflow", seed=31), dict(bc="mixed", seed=32),
                      dict(flux="rusanov", bc="periodic", seed=33),
                      dict(flux="rusanov", s_plus=0.0, bc="outflow", seed=34, scatter=True),
                      dict(flux="rusanov", s_plus=0.4, bc="inflow", seed=35),
                      dict(flux="rusanov", bc="mixed", seed=36, material=wl.COUPLED, scatter=True),
                      dict(bc="inflow", seed=37, scatter=True),
                      dict(dim=3, nx=4, ny=3, nz=4, bc="mixed", seed=38, scatter=True),
                      dict(dim=3, nx=3, ny=4, nz=4, flux="rusanov", bc="inflow", seed=39)]


@pytest.mark.parametrize("kw", NEW_OPERATOR_CASES, ids=[f"op{i}" for i in range(len(NEW_OPERATOR_CASES))])
def test_new_operators_tt_without_truncation_is_the_full_grid_step(kw):
    """Rusanov blocks, outflow ghost rows, the two-term Rusanov inflow and
    the scattering source in TT form reconstruct the full-grid step exactly
    when nothing is truncated (the TT form is an exact rewrite, Sec. 4)."""
    p = wl.small_random(**kw)
    s = Setup(p)
    I1, T1, _ = full.step(full.initial_intensity(s), s.T0, s)
    cat, T1t, _ = tt.step_untruncated(p["X0"], p["Th0"], p["Ph0"], s.T0, s)
    F = metrics.reconstruct(*cat).reshape(I1.shape)
    assert np.linalg.norm(F - I1) < 1e-13 * np.linalg.norm(I1)
    assert np.max(np.abs(T1t - T1)) < 1e-13 * np.max(np.abs(T1))
    (Xn, Thn, Phn), T2, _ = tt.step(p["X0"], p["Th0"], p["Ph0"], s.T0, s, 0.0, 0)
    F2 = metrics.reconstruct(Xn, Thn, Phn).reshape(I1.shape)
    assert np.linalg.norm(F2 - I1) < 1e-12 * np.linalg.norm(I1)


def test_gaussian_diffusion_ranks_and_analytic_solution():
    """Gaussian diffusion by isotropic scattering (Sec. 5.3), at reduced
    size (64^2 cells on [0,5]^2, 8x16 ordinates, rho kappa_s = 1e3, outflow,
    Rusanov with S+ = 0, tolerance 1e-4): the ranks stay at the (3, 3) the
    paper prints throughout (the isotropic part and the two first-order
    anisotropic terms n_x dJ/dx, n_y dJ/dy), the energy density follows
    the diffusion solution A / (4 pi D (t0 + t)) exp(-r^2 / (4 D (t0 + t))),
    D = c / (3 rho kappa_s), to well within the distance it travels, and the
    total energy stays at A."""
    p = wl.gaussian_diffusion(n=64, steps=300)
    s = Setup(p)
    (X, Th, Ph), _, hist = tt.run(s, 300)
    assert set(hist) == {(3, 3)}
    dif = p["diffusion"]
    t = 300 * s.dt
    xs = (np.arange(64) + 0.5) * 5.0 / 64 - 2.5
    r2 = xs[None, :] ** 2 + xs[:, None] ** 2

    def Ea(tt_):
        return dif["A"] / (4 * np.pi * dif["D"] * (dif["t0"] + tt_)) * np.exp(-r2 / (4 * dif["D"] * (dif["t0"] + tt_)))
    E = tt.energy(X, Th, Ph, s).reshape(64, 64)
    err = np.linalg.norm(E - Ea(t)) / np.linalg.norm(Ea(t))
    moved = np.linalg.norm(Ea(0.0) - Ea(t)) / np.linalg.norm(Ea(t))
    assert moved > 0.03 and err < 0.1 * moved
    assert abs(E.sum() * s.cell_volume - dif["A"]) < 1e-6


def test_gram_summation_is_not_the_fp64_parity_floor(monkeypatch):
    """Reading of the FP64 parity bar (App. A.4, Gram conditioning).  On C1
    states 3-5 (kept singular values down to 1e-7 sigma_1), replacing the
    plain FP64 Gram G_A = A^T A by one accumulated in 64-bit-mantissa
    arithmetic (correctly rounded to FP64) moves the oracle's step by less
    than 1e-11, while a symmetric change of one unit roundoff of lambda_max
    -- the norm-wise backward error of any backward-stable FP64 eigensolver
    -- moves it by more than 1e-10.  So compensated Gram sums cannot bring
    two independent FP64 Gram-SVD implementations closer than the
    eigensolvers' backward error allows; that spread is the bar of an
    'unpinned' comparison."""
    p = wl.c1()
    s = Setup(p)
    states = [(p["X0"], p["Th0"], p["Ph0"])]
    tt.run(s, 5, callback=lambda m, c, T, i: states.append(c))
    orig = rounding.gram_truncate

    def exact_first(A, GB, **kw):
        AL = np.asarray(A, dtype=np.longdouble)
        GAe = (AL.T @ AL).astype(np.float64)
        calls = [0]

        def pert(G):
            calls[0] += 1
            return GAe if calls[0] == 1 else G
        kw = dict(kw)
        kw["perturb"] = pert
        return orig(A, GB, **kw)
    worst_spread = 0.0
    for m in (3, 4, 5):
        Xs, Ts, Ps = states[m]
        ref, _, _ = tt.step(Xs, Ts, Ps, s.T0, s, p["tol"], p["rmax"])
        ranks = (ref[0].shape[1], ref[2].shape[0])
        monkeypatch.setattr(rounding, "gram_truncate", exact_first)
        ex, _, _ = tt.step(Xs, Ts, Ps, s.T0, s, p["tol"], p["rmax"], ranks=ranks)
        monkeypatch.setattr(rounding, "gram_truncate", orig)
        assert metrics.rel_diff(ex, ref) < 1e-11
        r = np.random.default_rng(1000 + m)

        def pert(G):
            E = r.uniform(-1.0, 1.0, G.shape)
            return G + rounding.U * np.abs(G).max() * 0.5 * (E + E.T)
        b, _, _ = tt.step(Xs, Ts, Ps, s.T0, s, p["tol"], p["rmax"], ranks=ranks, perturb=pert)
        worst_spread = max(worst_spread, metrics.rel_diff(b, ref))
    assert worst_spread > 1e-10


# ------------------------------------------------------------------ hohlraum
def _hohlraum_J_by_quadrature(t, x, y, c=1.0, nth=1000, nph=2000):
    """Mean intensity as the solid-angle fraction (midpoint rule in theta,
    phi) of directions whose backward ray from (x, y) leaves the quadrant
    x, y > 0 through a wall within path length c t (Sec. 5.1's set-up)."""
    th = (np.arange(nth) + 0.5) * np.pi / nth
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    st = np.sin(TH)
    hx, hy = st * np.cos(PH), st * np.sin(PH)
    with np.errstate(divide="ignore", invalid="ignore"):
        sx = np.where(hx > 0, x / hx, np.inf)
        sy = np.where(hy > 0, y / hy, np.inf)
    w = st * (np.pi / nth) * (2 * np.pi / nph)
    return float((w * (np.minimum(sx, sy) <= c * t)).sum() / (4 * np.pi))


def test_hohlraum_analytic_matches_quadrature():
    """The closed form of Sec. 5.1 (J_left + J_bottom) against a direct
    solid-angle quadrature of the same set-up, on both sides of the fronts
    x = c t and y = c t."""
    from oracle.analytic import hohlraum_J
    for (x, y) in [(0.1, 0.2), (0.5, 0.3), (0.2, 0.9), (0.74, 0.01), (0.05, 0.7), (0.8, 0.3),
                   (0.9, 0.9)]:
        a = float(hohlraum_J(0.75, x, y))
        q = _hohlraum_J_by_quadrature(0.75, x, y)
        assert abs(a - q) < 1e-4, (x, y, a, q)
    # symmetric in x and y; a half-space's 1/2 at a wall far from the corner
    assert abs(float(hohlraum_J(0.75, 0.3, 0.6)) - float(hohlraum_J(0.75, 0.6, 0.3))) < 1e-15
    assert abs(float(hohlraum_J(0.5, 1e-12, 0.9)) - 0.5) < 1e-9


def test_hohlraum_full_grid_first_order():
    """The full-grid S_N solution of the reduced hohlraum (16 x 32 ordinates)
    against the analytic J over [0, 1]^2: the area-weighted L1 error is below
    2e-2 at 32^2 cells and falls at first order in the cell size."""
    from oracle.analytic import hohlraum_J
    errs = []
    for n in (32, 64):
        p = wl.hohlraum(n=n, ntheta=16, nphi=32)
        s = Setup(p)
        I, _ = full.run(s, p["steps"])
        J = s.c * full.energy(I, s).reshape(n, n) / (4 * np.pi)
        xc = (np.arange(n) + 0.5) * 2.0 / n
        Ja = hohlraum_J(p["hohlraum"]["t"], xc[None, :], xc[:, None])
        m = n // 2
        errs.append(np.abs(J[:m, :m] - Ja[:m, :m]).sum() * (2.0 / n) ** 2)
    assert errs[0] < 2e-2
    assert errs[1] < 0.65 * errs[0]


# --------------------------------------------------------------- line source
def test_line_source_analytic_integrates_to_U0():
    """The delta-pulse solution of Sec. 5.4 carries U0 at every time: its
    integral over the plane, 2 pi int_0^{ct} E r dr, by a substitution that
    removes the front's singularity (r = c t sin(a))."""
    from oracle.analytic import line_source_E
    for t, U0 in ((0.3, 1.0), (1.0, 2.5)):
        a = (np.arange(20000) + 0.5) * (0.5 * np.pi / 20000)
        r = t * np.sin(a)
        integrand = 2 * np.pi * line_source_E(t, r, U0) * r * t * np.cos(a)
        assert abs(integrand.sum() * (0.5 * np.pi / 20000) - U0) < 1e-8 * U0
    assert line_source_E(0.5, 0.6) == 0.0


def test_line_source_full_grid_conserves_energy():
    """The upwind finite-volume step moves energy between cells only: with the
    pulse and its front inside the domain (vacuum, no opacity), the full-grid
    oracle keeps sum_i E_i dA to rounding, and the TT oracle at a tolerance
    far below the state's spectrum does too."""
    p = wl.line_source(n=32, ntheta=8, nphi=16, t_end=0.25, tol=1e-13, rmax=0)
    s = Setup(p)
    dA = (p["lx"] / p["nx"]) ** 2
    I0 = full.initial_intensity(s)
    E0 = full.energy(I0, s).sum() * dA
    I, _ = full.run(s, p["steps"], I=I0)
    assert abs(full.energy(I, s).sum() * dA - E0) < 1e-12 * E0
    (X, Th, Ph), _, _ = tt.run(s, p["steps"])
    assert abs(tt.energy(X, Th, Ph, s).sum() * dA - E0) < 1e-10 * E0


# ------------------------------------------------------- randomized rounding
def test_randomized_rounding_exact_on_low_rank():
    """A TT whose bond ranks exceed the tensor's (the concatenation of a
    rank-(3, 2) TT with twice itself: ranks (6, 4), tensor 3 X Theta Phi) is
    reproduced to rounding by randomized rounding at the true ranks (App. A.3),
    and both left factors come out with orthonormal columns."""
    rng = np.random.default_rng(11)
    ns, nt, npf = 40, 6, 8
    X = rng.standard_normal((ns, 3))
    Th = rng.standard_normal((3, nt, 2))
    Ph = rng.standard_normal((2, npf))
    Xc = np.hstack([X, 2.0 * X])
    Thc = np.zeros((6, nt, 4))
    Thc[:3, :, :2] = Th
    Thc[3:, :, 2:] = Th
    Phc = np.vstack([Ph, Ph])
    T = 3.0 * metrics.reconstruct(X, Th, Ph)
    Xr, Thr, Phr = rounding.round_randomized(Xc, Thc, Phc, wl.gaussian_test_matrices(nt, npf, 3, 2, 5))
    assert Xr.shape == (ns, 3) and Thr.shape == (3, nt, 2) and Phr.shape == (2, npf)
    R = metrics.reconstruct(Xr, Thr, Phr)
    assert np.linalg.norm(R - T) < 1e-12 * np.linalg.norm(T)
    assert np.abs(Xr.T @ Xr - np.eye(3)).max() < 1e-13
    A2 = Thr.reshape(3 * nt, 2)
    assert np.abs(A2.T @ A2 - np.eye(2)).max() < 1e-13


@pytest.mark.parametrize("decay_in", ["X", "Theta"])
def test_randomized_rounding_expected_error_bound(decay_in):
    """Bond 1 with oversampling (target k + p, k = 6, p = 4; bond 2 kept at
    its full rank, which the sketch reproduces exactly): over 40 seeds the
    mean Frobenius error is within the expected-error bound of a Gaussian
    sketch, sqrt(1 + k / (p - 1)) times the optimal rank-k error (Halko,
    Martinsson and Tropp, SIAM Review 2011, Thm. 10.5), and no trial beats
    the optimal rank-(k + p) error (Eckart-Young).  The spectrum's decay is
    put in X or in Theta: with it in Theta, a sketch of X alone (without
    B^T Omega) would miss the dominant directions."""
    rng = np.random.default_rng(12)
    ns, nt, npf, r1, r2 = 60, 8, 16, 24, 4
    U, _ = np.linalg.qr(rng.standard_normal((ns, r1)))
    s = 0.7 ** np.arange(r1)
    # Theta unfolded (r1 x nt r2) and Phi with orthonormal rows, and the
    # weights s on X's columns or on Theta's rows: the bond-1 singular values
    # of the tensor are exactly s either way
    Qt, _ = np.linalg.qr(rng.standard_normal((nt * r2, r1)))
    if decay_in == "X":
        X = U * s
        Th = Qt.T.reshape(r1, nt, r2)
    else:
        X = U
        Th = (s[:, None] * Qt.T).reshape(r1, nt, r2)
    Qp, _ = np.linalg.qr(rng.standard_normal((npf, r2)))
    Ph = Qp.T
    T1 = metrics.reconstruct(X, Th, Ph).reshape(ns, nt * npf)
    assert np.allclose(np.linalg.svd(T1, compute_uv=False)[:r1], s, rtol=0, atol=1e-13)
    k, p = 6, 4
    tail = lambda j: np.sqrt(np.sum(s[j:] ** 2))
    errs = []
    for seed in range(40):
        Xr, Thr, Phr = rounding.round_randomized(X, Th, Ph,
                                                 wl.gaussian_test_matrices(nt, npf, k + p, r2, 100 + seed))
        errs.append(np.linalg.norm(metrics.reconstruct(Xr, Thr, Phr).reshape(ns, -1) - T1))
    errs = np.array(errs)
    assert errs.mean() <= np.sqrt(1 + k / (p - 1)) * tail(k)
    assert errs.min() >= tail(k + p) * (1 - 1e-10)


# ------------------------------------------------------------------ HLL flux
def _hll_speeds(n, tau, c, thr):
    """(S_L, S_R) of Sec. 3.1, case by case as printed."""
    if tau >= thr:
        a = np.sqrt((1.0 - np.exp(-tau ** 2)) / tau ** 2)
        b = np.sqrt((1.0 - np.exp(-tau ** 4)) / tau ** 2)
    else:
        a = np.sqrt(1.0 - tau ** 2 / 2.0)
        b = tau
    if n >= 0:
        return -c * n * b, c * n * a
    return c * n * a, -c * n * b


def test_hll_step_brute_force_from_the_wavespeeds():
    """eq. hll evaluated face by face in plain loops, with the four-case
    wavespeeds of Sec. 3.1 and the harmonic-mean tau_c of eq. tauc (cell
    i+1's extinction in the second term), on a periodic line whose random
    extinction puts faces on both sides of tau_threshold."""
    rng = np.random.default_rng(7)
    nx, beta = 10, 1.7
    p = _line_problem(nx=nx)
    p["flux"], p["hll_beta"] = "hll", beta
    s0 = Setup(p)
    p["rho"][:] = 0.5 + rng.random(nx)
    p["kappa"][:] = 10.0 ** rng.uniform(-4.0, 1.8, nx) / (beta * s0.dx * p["rho"])
    s = Setup(p)
    ext = s.rho * (s.kappa + s.kappa_s)
    taus = [2 * beta * s.dx / (1 / ext[i] + 1 / ext[(i + 1) % nx]) for i in range(nx)]
    assert min(taus) < s.hll_threshold < max(taus) and max(taus) > 2
    I = rng.random((1, 1, nx, s.nt, s.np_))
    c = s.c

    def flux(i, l, q):                      # F at face i + 1/2
        j = (i + 1) % nx
        n = s.sin_t[l] * s.cos_p[q]
        sl, sr = _hll_speeds(n, taus[i], c, s.hll_threshold)
        ul, ur = I[0, 0, i, l, q], I[0, 0, j, l, q]
        return (sr * c * n * ul - sl * c * n * ur + sl * sr * (ur - ul)) / (sr - sl)

    expect = np.empty_like(I)
    for i in range(nx):
        for l in range(s.nt):
            for q in range(s.np_):
                expect[0, 0, i, l, q] = I[0, 0, i, l, q] - s.dt / s.dx * (
                    flux(i, l, q) - flux((i - 1) % nx, l, q))
    assert np.max(np.abs(full.transport(I, s) - expect)) < 1e-13


def test_hll_zero_optical_depth_is_upwind():
    """tau -> 0 recovers the upwind flux (Sec. 3.1): exactly at zero
    extinction (inflow, outflow and vacuum faces included), and to O(tau^2)
    below the threshold."""
    p = wl.small_random(bc="mixed", seed=61)
    p["kappa"][:] = 0.0
    s_up = Setup(p)
    I = full.initial_intensity(s_up)
    Iu = full.transport(I, s_up)
    p["flux"] = "hll"
    assert np.max(np.abs(full.transport(I, Setup(p)) - Iu)) < 1e-15 * np.max(np.abs(Iu))
    p["kappa"][:] = 1e-4
    s = Setup(p)
    tmax = max(s.hll_tau(a).max() for a in range(s.dim))
    assert 0 < tmax < s.hll_threshold
    assert np.max(np.abs(full.transport(I, s) - Iu)) < 4 * tmax ** 2 * np.max(np.abs(I))


@pytest.mark.parametrize("tau", [12.0, 6.0])
def test_hll_thick_limit_is_rusanov_fourier(tau):
    """Large tau_c: the HLL flux is the Rusanov flux with S+ = c |n_x| / tau_c
    (Sec. 3.1), up to terms of order exp(-tau^2); on a periodic line of
    uniform extinction a Fourier mode evolves by
    g = 1 - i nu sin h - lam (|n_x| / tau)(1 - cos h), nu = lam n_x."""
    p = _line_problem()
    p["flux"] = "hll"
    s0 = Setup(p)
    p["kappa"][:] = tau / (s0.dx * p["rho"])
    s = Setup(p)
    assert np.allclose(s.hll_tau(0), tau, rtol=1e-14)
    k = 3
    x = (np.arange(s.nx) + 0.5) * s.dx
    theta = 2 * np.pi * k * x
    h = 2 * np.pi * k * s.dx
    I = np.broadcast_to(np.cos(theta)[None, None, :, None, None], (1, 1, s.nx, s.nt, s.np_)).copy()
    m = 4
    for _ in range(m):
        I = full.transport(I, s)
    lam = s.lam[0]
    n = np.outer(s.sin_t, s.cos_p)
    g = 1 - 1j * lam * n * np.sin(h) - lam * (np.abs(n) / tau) * (1 - np.cos(h))
    expect = np.real(g[None, :, :] ** m * np.exp(1j * theta)[:, None, None])
    assert np.max(np.abs(I[0, 0] - expect)) < 1e-13 + 10 * np.exp(-tau ** 2)


def test_hll_flux_form_conservation_and_outflow_steady_state():
    """The HLL update is in flux form with alpha + beta = 1 at every face: on
    a periodic grid with random extinction each direction's total is kept,
    and with outflow on every face a uniform field is steady."""
    p = wl.small_random(bc="periodic", seed=62, flux="hll", hll_beta=3.0, scatter=True)
    s = Setup(p)
    I = full.initial_intensity(s)
    I1 = full.transport(I, s)
    tot0, tot1 = I.sum(axis=(0, 1, 2)), I1.sum(axis=(0, 1, 2))
    assert np.max(np.abs(tot1 - tot0)) < 1e-13 * np.max(np.abs(tot0))
    p = wl.small_random(bc="outflow", seed=63, flux="hll", hll_beta=0.3)
    s = Setup(p)
    U = np.full(s.grid_shape() + (s.nt, s.np_), 1.7)
    assert np.max(np.abs(full.transport(U, s) - U)) < 1e-14


HLL_CASES = [dict(flux="hll", bc="periodic", seed=41),
             dict(flux="hll", hll_beta=2.5, bc="inflow", seed=42, scatter=True),
             dict(flux="hll", bc="mixed", seed=43, material=wl.COUPLED),
             dict(flux="hll", hll_beta=0.01, bc="outflow", seed=44),
             dict(dim=3, nx=4, ny=3, nz=4, flux="hll", hll_beta=0.05, bc="mixed", seed=45,
                  scatter=True),
             dict(dim=3, nx=3, ny=4, nz=4, flux="hll", bc="inflow", seed=46)]


@pytest.mark.parametrize("kw", HLL_CASES, ids=[f"hll{i}" for i in range(len(HLL_CASES))])
def test_hll_tt_without_truncation_is_the_full_grid_step(kw):
    """The HLL flux in TT form (one variable-weight stencil block per axis
    and sign of n, the inflow ghost as rank-1 blocks per sign; Sec. 4.3)
    reconstructs the full-grid step exactly when nothing is truncated."""
    p = wl.small_random(**kw)
    s = Setup(p)
    I1, T1, _ = full.step(full.initial_intensity(s), s.T0, s)
    cat, T1t, _ = tt.step_untruncated(p["X0"], p["Th0"], p["Ph0"], s.T0, s)
    F = metrics.reconstruct(*cat).reshape(I1.shape)
    assert np.linalg.norm(F - I1) < 1e-13 * np.linalg.norm(I1)
    assert np.max(np.abs(T1t - T1)) < 1e-13 * np.max(np.abs(T1))


def test_line_source_smoothed_solution():
    """The Gaussian-smoothed line source (Sec. 5.4): its plane integral is
    U0 at every t, it tends to the initial Gaussian as c t / omega -> 0, and
    at four radii (inside, near and past the front) it equals the plane
    convolution of the delta-pulse solution with the Gaussian taken by brute
    force over the circle (no Bessel reduction)."""
    from oracle import analytic as an
    om = 0.03
    for t in (0.25, 0.5, 1.0):
        r = np.linspace(0.0, t + 12 * om, 6001)
        tot = 2 * np.pi * np.trapezoid(an.line_source_smoothed_E(t, r, U0=1.3, omega=om, n=6000) * r, r)
        assert abs(tot - 1.3) < 1e-7
    r = np.linspace(0.0, 0.1, 11)
    G = np.exp(-r ** 2 / (2 * om ** 2)) / (2 * np.pi * om ** 2)
    assert np.max(np.abs(an.line_source_smoothed_E(1e-4, r, omega=om) - G)) < 1e-5 * G.max()
    t = ct = 0.5
    nphi, npsi = 4000, 1024
    rho = ct * np.sin((np.arange(nphi) + 0.5) * (0.5 * np.pi / nphi))
    psi = (np.arange(npsi) + 0.5) * (2 * np.pi / npsi)
    for rp in (0.1, 0.3, 0.48, 0.52):
        d2 = rp ** 2 + rho[:, None] ** 2 - 2 * rp * rho[:, None] * np.cos(psi[None, :])
        G = np.exp(-d2 / (2 * om ** 2)) / (2 * np.pi * om ** 2)
        # E_delta(rho) rho drho = rho dphi / (2 pi c t) with rho = c t sin(phi)
        brute = np.sum(rho[:, None] * G) * (0.5 * np.pi / nphi) * (2 * np.pi / npsi) / (2 * np.pi * ct)
        assert abs(an.line_source_smoothed_E(t, rp, omega=om)[0] - brute) < 1e-7 * brute
