"""Parity of the library's HLL flux (Sec. 3.1 eqs. hll and tauc; Sec. 4.3)
with the CPU oracle, through the C ABI.

- One step from the same state to 1e-10 and three free-running steps to
  1e-8 with identical ranks, the temperature to 1e-10: periodic, inflow,
  outflow and mixed faces, 2-D and 3-D, beta from 0.01 (faces on both sides
  of the series threshold) to 5, scattering (whose opacity enters tau_c, so
  the weights are re-formed by tt_set_scattering) and coupled material.
  The seeded cases have rank-decision margins of at least 0.37 in the
  oracle.
- The two-rounding schedule, and the FP32-mixed form at its 1e-6 bar.
- tt_set_kappa re-forms the face weights: the step after it matches the
  oracle built with the new opacity.
- Zero extinction: the HLL step is the upwind step (tau -> 0 limit).
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


HLL_OPS = [dict(flux="hll", bc="periodic", seed=41),
           dict(flux="hll", hll_beta=2.5, bc="inflow", seed=42, scatter=True),
           dict(flux="hll", bc="mixed", seed=43, material=wl.COUPLED),
           dict(flux="hll", hll_beta=0.01, bc="outflow", seed=44),
           dict(dim=3, nx=4, ny=3, nz=4, flux="hll", hll_beta=0.05, bc="mixed", seed=45,
                scatter=True),
           dict(dim=3, nx=3, ny=4, nz=4, flux="hll", bc="inflow", seed=46),
           dict(nx=33, ny=17, ntheta=8, nphi=16, r1=5, r2=3, seed=47, bc="mixed", flux="hll",
                hll_beta=5.0, scatter=True)]


def _compare(p, st, nsteps, schedule="once", bar1=1e-10, barn=1e-8, tbar=1e-10):
    s = Setup(p)
    st.step(1)
    (X1, T1c, P1), _, _ = tt.run(s, 1, schedule=schedule)
    err1 = metrics.rel_diff(st.cores(), (X1, T1c, P1))
    st.step(nsteps - 1)
    hist_gpu = st.tt_get_rank_history()
    (X, Th, Ph), T, hist = tt.run(s, nsteps, schedule=schedule)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    terr = np.max(np.abs(st.tt_get_temperature() - T)) / max(np.max(np.abs(T)), 1e-300)
    _log(f"{p['name']} beta={p['hll_beta']} [{schedule}]: ranks gpu={hist_gpu} oracle={hist} "
         f"step1 err={err1:.2e} step{nsteps} err={err:.2e} Terr={terr:.2e}")
    assert hist_gpu == hist
    assert err1 < bar1
    assert err < barn
    assert terr < tbar


@pytest.mark.parametrize("kw", HLL_OPS, ids=[f"hll{i}" for i in range(len(HLL_OPS))])
def test_hll_parity(kw):
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    _compare(p, _state(p, max_steps=3), 3)


@pytest.mark.parametrize("kw", [HLL_OPS[1], HLL_OPS[4]], ids=["inflow_scat", "3d_mixed"])
def test_hll_twice_schedule_parity(kw):
    from paper_2503_18056_amd import TT_ROUND_TWICE
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    _compare(p, _state(p, max_steps=3, schedule=TT_ROUND_TWICE), 3, schedule="twice")


def test_hll_mixed_precision():
    from paper_2503_18056_amd import TT_FP32_MIXED
    p = wl.small_random(**HLL_OPS[2])
    p["tol"] = 1e-6
    _compare(p, _state(p, max_steps=3, precision=TT_FP32_MIXED), 3, bar1=1e-6, barn=1e-6, tbar=1e-6)


def test_hll_set_kappa_reforms_the_weights():
    p = wl.small_random(**HLL_OPS[1])
    p["tol"] = 1e-6
    st = _state(p, max_steps=3)
    k2 = p["kappa"] * np.exp(np.random.default_rng(9).standard_normal(p["kappa"].size))
    st.tt_set_kappa(k2)
    q = dict(p, kappa=k2)
    s = Setup(q)
    st.step(2)
    (X, Th, Ph), T, hist = tt.run(s, 2)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    _log(f"set_kappa: ranks gpu={st.tt_get_rank_history()} oracle={hist} err={err:.2e}")
    assert st.tt_get_rank_history() == hist
    assert err < 1e-8


def test_hll_zero_extinction_is_upwind():
    p = wl.small_random(bc="mixed", seed=61, flux="hll")
    p["kappa"][:] = 0.0
    p["tol"] = 1e-6
    a = _state(p, max_steps=2)
    b = _state(dict(p, flux="upwind"), max_steps=2)
    a.step(2)
    b.step(2)
    err = metrics.rel_diff(a.cores(), b.cores())
    _log(f"zero extinction: hll ranks {a.tt_get_rank_history()} upwind {b.tt_get_rank_history()} "
         f"err={err:.2e}")
    assert a.tt_get_rank_history() == b.tt_get_rank_history()
    assert err < 1e-10
