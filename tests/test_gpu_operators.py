"""Parity of the library's transport-operator options and two-rounding
schedule with the CPU oracle, through the C ABI.

- Rusanov flux (Sec. 3.1 eq. rusanov_flux_toro; Sec. 4.3), with S+ > 0 and
  S+ = 0, outflow ghost cells (Sec. 4.5), mixed faces, and isotropic
  scattering with implicit J^{m+1} (Sec. 3.2 eq. couple_a): one step from
  the same state to 1e-10 and three free-running steps to 1e-8 with identical
  ranks, the temperature to 1e-10 (small seeded cases whose spectra have
  gaps at the cut).
- The two-rounding schedule (Sec. 4.2): the same bars, both precisions for
  the FP32-mixed form at the mixed bar, and rank replay consuming two
  schedule entries per step.
- Reduced Gaussian diffusion (Sec. 5.3): ranks (3, 3) at every step, as the
  paper prints, and the oracle's trajectory.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, tt

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _state(p, **kw):
    from paper_2503_18056_amd import TTState
    return TTState(p, device=0, **kw)


OPS = [dict(bc="outflow", seed=31), dict(bc="mixed", seed=32),
       dict(flux="rusanov", bc="periodic", seed=33),
       dict(flux="rusanov", s_plus=0.0, bc="outflow", seed=34, scatter=True),
       dict(flux="rusanov", s_plus=0.4, bc="inflow", seed=35),
       dict(flux="rusanov", bc="mixed", seed=36, material=wl.COUPLED, scatter=True),
       dict(bc="inflow", seed=37, scatter=True),
       dict(bc="vacuum", seed=40, material=wl.COUPLED, scatter=True),
       dict(dim=3, nx=4, ny=3, nz=4, bc="mixed", seed=38, scatter=True),
       dict(dim=3, nx=3, ny=4, nz=4, flux="rusanov", bc="inflow", seed=39),
       dict(nx=33, ny=17, ntheta=8, nphi=16, r1=5, r2=3, seed=41, bc="mixed", flux="rusanov",
            s_plus=0.5, scatter=True)]


def _compare(p, st, nsteps, schedule="once", bar1=1e-10, barn=1e-8, tbar=1e-10):
    s = Setup(p)
    st.step(1)
    (X1, T1c, P1), T1, _ = tt.run(s, 1, schedule=schedule)
    err1 = metrics.rel_diff(st.cores(), (X1, T1c, P1))
    st.step(nsteps - 1)
    hist_gpu = st.tt_get_rank_history()
    (X, Th, Ph), T, hist = tt.run(s, nsteps, schedule=schedule)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    Tg = st.tt_get_temperature()
    terr = np.max(np.abs(Tg - T)) / max(np.max(np.abs(T)), 1e-300)
    _log(f"{p['name']} [{schedule}]: ranks gpu={hist_gpu} oracle={hist} step1 err={err1:.2e} "
         f"step{nsteps} err={err:.2e} Terr={terr:.2e}")
    assert hist_gpu == hist
    assert err1 < bar1
    assert err < barn
    assert terr < tbar


@pytest.mark.parametrize("kw", OPS, ids=[f"op{i}" for i in range(len(OPS))])
def test_operator_parity(kw):
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    _compare(p, _state(p, max_steps=3), 3)


@pytest.mark.parametrize("kw", [dict(seed=1), dict(bc="inflow", seed=3, material=wl.COUPLED),
                                dict(bc="periodic", seed=2, scatter=True),
                                dict(flux="rusanov", bc="mixed", seed=36, material=wl.COUPLED,
                                     scatter=True),
                                dict(dim=3, nx=4, ny=3, nz=5, bc="inflow", seed=4,
                                     material=wl.COUPLED)],
                         ids=["vac", "inflow_coupled", "periodic_scat", "rusanov_mixed", "3d"])
def test_twice_schedule_parity(kw):
    from paper_2503_18056_amd import TT_ROUND_TWICE
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    _compare(p, _state(p, max_steps=3, schedule=TT_ROUND_TWICE), 3, schedule="twice")


def test_twice_schedule_mixed_precision_and_replay():
    """FP32-mixed form with two roundings per step against the FP64 oracle
    (1e-6 over three steps, the mixed bar of the one-rounding schedule); rank
    replay takes two schedule entries per step and reproduces the oracle's
    rank pairs."""
    from paper_2503_18056_amd import TT_FP32_MIXED, TT_RANK_REPLAY, TT_ROUND_TWICE
    p = wl.small_random(bc="inflow", seed=3, material=wl.COUPLED)
    p["tol"] = 1e-6
    s = Setup(p)
    st = _state(p, max_steps=3, schedule=TT_ROUND_TWICE, precision=TT_FP32_MIXED)
    st.step(3)
    infos = []
    (X, Th, Ph), T, hist = tt.run(s, 3, schedule="twice", callback=lambda m, c, T, i: infos.append(i))
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    _log(f"twice mixed: ranks gpu={st.tt_get_rank_history()} oracle={hist} err={err:.2e}")
    assert st.tt_get_rank_history() == hist
    assert err < 1e-6
    pairs = []
    for i in infos:
        for (b1, b2) in i["round"]:
            pairs.append((b1["rank"], b2["rank"]))
    assert len(pairs) == 6
    sr = _state(p, max_steps=3, schedule=TT_ROUND_TWICE, rank_mode=TT_RANK_REPLAY)
    sr.tt_set_rank_schedule(pairs)
    sr.step(3)
    assert sr.tt_get_rank_history() == hist
    assert metrics.rel_diff(sr.cores(), (X, Th, Ph)) < 1e-8


def test_gaussian_diffusion_reduced():
    """Sec. 5.3 at reduced size (64^2, 8x16, rho kappa_s = 1e3, outflow,
    Rusanov S+ = 0, tolerance 1e-4): ranks (3, 3) at all 300 steps, the
    oracle's end state to 1e-8, and the analytic diffusion solution to a
    tenth of the distance it moves."""
    p = wl.gaussian_diffusion(n=64, steps=300)
    s = Setup(p)
    st = _state(p, max_steps=300)
    st.step(300)
    hist = st.tt_get_rank_history()
    assert set(hist) == {(3, 3)}, set(hist)
    (X, Th, Ph), _, ohist = tt.run(s, 300)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    E = st.tt_energy()[0].cpu().numpy().reshape(64, 64)
    dif = p["diffusion"]
    xs = (np.arange(64) + 0.5) * 5.0 / 64 - 2.5
    r2 = xs[None, :] ** 2 + xs[:, None] ** 2

    def Ea(t):
        return dif["A"] / (4 * np.pi * dif["D"] * (dif["t0"] + t)) * np.exp(-r2 / (4 * dif["D"] * (dif["t0"] + t)))
    t = 300 * s.dt
    aerr = np.linalg.norm(E - Ea(t)) / np.linalg.norm(Ea(t))
    moved = np.linalg.norm(Ea(0.0) - Ea(t)) / np.linalg.norm(Ea(t))
    _log(f"gaussian diffusion: ranks {set(hist)}, vs oracle {err:.2e}, vs analytic {aerr:.2e} (moved {moved:.2e})")
    assert err < 1e-8
    assert aerr < 0.1 * moved


def test_detector_loss_is_formed_by_the_library():
    """tt_detector_loss: L = dV sum_i w_i E_i of the current state, against
    the oracle's energy density of the same state, and equal to the loss
    tt_grad reports for the same state."""
    p = wl.c5(n=24, steps=4)
    p["ntheta"], p["nphi"] = 8, 16
    p["X0"], p["Th0"], p["Ph0"] = wl.gaussian_pulse_cores(p)
    p["rmax"] = 0
    s = Setup(p)
    det = np.zeros(24 * 24)
    det[::7] = 1.0
    st = _state(p, max_steps=4, ckpt_every=2)
    st.step(4)
    L = st.tt_detector_loss(det)
    (X, Th, Ph), _, _ = tt.run(s, 4)
    Lo = float(det @ tt.energy(X, Th, Ph, s)) * s.cell_volume
    Lg, _ = st.tt_grad(det)
    _log(f"detector loss {L:.15e} oracle {Lo:.15e} tt_grad {Lg:.15e}")
    assert abs(L - Lo) < 1e-10 * abs(Lo)
    assert L == Lg


def test_grad_after_round_is_stale():
    """A rounding is not a recorded step: after tt_step then tt_round, the
    tape no longer ends in the stored state, so tt_grad reports
    TT_ERR_STATE instead of a gradient of some other map."""
    from paper_2503_18056_amd import TTError, _ffi
    p = wl.c5(n=24, steps=3)
    p["ntheta"], p["nphi"] = 8, 16
    p["X0"], p["Th0"], p["Ph0"] = wl.gaussian_pulse_cores(p)
    st = _state(p, max_steps=3, ckpt_every=1)
    st.step(2)
    st.tt_round(1e-3, 0)
    with pytest.raises(TTError) as e:
        st.tt_grad(np.ones(24 * 24))
    assert e.value.status == _ffi.TT_ERR_STATE
    assert "stale" in str(e.value)
    st.tt_set_cores(p["X0"], p["Th0"], p["Ph0"])
    st.step(2)
    L, g = st.tt_grad(np.ones(24 * 24))
    assert np.isfinite(L) and np.all(np.isfinite(g.cpu().numpy()))


def test_jacobi_sweep_cap_reports_non_convergence():
    """The failure path of the SVD of M, forced from the host: with
    tt_set_solver_limits capping the one-sided Jacobi SVD at one sweep (too
    few for the dense M of a step), the step returns TT_ERR_NUMERIC naming
    that solver and the context is poisoned; without the cap the same steps
    run.  The solver's rotations keep every value finite, so every kernel
    exits normally."""
    from paper_2503_18056_amd import TTError
    from paper_2503_18056_amd._ffi import TT_ERR_INVALID_ARG, TT_ERR_NUMERIC, TT_ERR_STATE
    p = wl.small_random(nx=33, ny=17, ntheta=8, nphi=16, r1=5, r2=3, seed=41, bc="mixed")
    p["tol"] = 1e-6
    st = _state(p, max_steps=4)
    with pytest.raises(TTError) as e:
        st.tt_set_solver_limits(-1)
    assert e.value.status == TT_ERR_INVALID_ARG
    st.step(2)
    st.tt_set_solver_limits(1)
    with pytest.raises(TTError) as e:
        st.step(1)
    _log(f"capped Jacobi: {e.value}")
    assert e.value.status == TT_ERR_NUMERIC
    assert "Jacobi SVD did not converge" in str(e.value)
    with pytest.raises(TTError) as e:
        st.step(1)
    assert e.value.status == TT_ERR_STATE
    ok = _state(p, max_steps=4)
    ok.tt_set_solver_limits(0)
    ok.step(3)
