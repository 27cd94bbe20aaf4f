"""The optically thick 3-D workload at full size, through the C ABI, against
the CPU oracle: 128^3 cells, 32 x 64 ordinates, kappa = 1e3 in the central
64^3 cube and 1 outside, coupled material (c_v = 1) with a seeded rough
initial temperature, equilibrium isotropic initial intensity of rank (1, 1),
vacuum boundaries, tolerance 1e-6, rank cap 128.

The first five steps, in which the ranks ramp from (1, 1) up to the cap
(concatenated ranks up to 7 * 128 + 1 = 897 at bond 1), are taken by the
oracle once and by the library in FP64 and in the FP32-mixed form:

- ranks: identical at every step, unless the oracle's decision lies within
  MARGIN of its threshold (then FP64 rounding decides it, on either side,
  and the comparison of ranks stops there);
- FP64: relative Frobenius difference of the five-step state below 1e-8 and
  temperature below 1e-10 relative; with the oracle's rank history replayed,
  the same bars;
- FP32-mixed: state below 1e-5 (the precision target), temperature below
  1e-5 relative (its update differences energies of FP32-stored cores).
"""
import sys
import time

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, tt

pytestmark = pytest.mark.gpu

NSTEPS = 5
MARGIN = 1e-3


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def oracle_run():
    p = wl.c4(steps=NSTEPS)
    s = Setup(p)
    t0 = time.time()
    infos = []

    def cb(m, c, T, info):
        infos.append(info)
        _log(f"  oracle {p['name']} step {m + 1}: ranks ({c[0].shape[1]},{c[2].shape[0]}) "
             f"{time.time() - t0:.1f}s")
    cores, T, hist = tt.run(s, NSTEPS, callback=cb)
    return p, cores, T, hist, infos


def _compare(p, st, oracle, bar, tbar, label):
    _, cores, T, hist, infos = oracle
    hist_gpu = [tuple(h) for h in st.tt_get_rank_history()]
    compared = NSTEPS
    for k, (g, o) in enumerate(zip(hist_gpu, hist)):
        if g != o:
            margin = min(b.get("margin", np.inf) for b in infos[k]["round"][-1])
            _log(f"  {label}: step {k + 1} gpu ranks {g} oracle {o} (oracle's margin {margin:.2e})")
            assert margin < MARGIN, (k + 1, g, o, margin)
            compared = k
            break
    err = metrics.rel_diff(st.cores(), cores)
    terr = float(np.max(np.abs(st.tt_get_temperature() - T)) / np.max(np.abs(T)))
    _log(f"  {label}: ranks gpu {hist_gpu} oracle {hist}; identical for {compared}/{NSTEPS} "
         f"steps; err={err:.2e} Terr={terr:.2e}")
    if compared == NSTEPS:
        assert err < bar
        assert terr < tbar
    return compared


def test_thick3d_fp64_vs_oracle(oracle_run):
    from paper_2503_18056_amd import TT_RANK_REPLAY, TTState
    p, _, _, hist, _ = oracle_run
    st = TTState(p, device=0, max_steps=NSTEPS)
    st.step(NSTEPS)
    compared = _compare(p, st, oracle_run, 1e-8, 1e-10, "fp64 free run")
    st.close()
    sr = TTState(p, device=0, max_steps=NSTEPS, rank_mode=TT_RANK_REPLAY)
    sr.tt_set_rank_schedule(hist)
    sr.step(NSTEPS)
    assert [tuple(h) for h in sr.tt_get_rank_history()] == list(hist)
    assert _compare(p, sr, oracle_run, 1e-8, 1e-10, "fp64 replayed ranks") == NSTEPS
    sr.close()
    assert compared >= 1


def test_thick3d_mixed_vs_oracle(oracle_run):
    from paper_2503_18056_amd import TT_FP32_MIXED, TT_RANK_REPLAY, TTState
    p, _, _, hist, _ = oracle_run
    st = TTState(p, device=0, max_steps=NSTEPS, precision=TT_FP32_MIXED)
    st.step(NSTEPS)
    compared = _compare(p, st, oracle_run, 1e-5, 1e-5, "fp32-mixed free run")
    st.close()
    if compared < NSTEPS:
        sr = TTState(p, device=0, max_steps=NSTEPS, precision=TT_FP32_MIXED,
                     rank_mode=TT_RANK_REPLAY)
        sr.tt_set_rank_schedule(hist)
        sr.step(NSTEPS)
        assert _compare(p, sr, oracle_run, 1e-5, 1e-5, "fp32-mixed replayed ranks") == NSTEPS
        sr.close()
