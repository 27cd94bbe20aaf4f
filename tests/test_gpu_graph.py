"""Graph replay of the step (tt_use_graphs, the default) against eager
stepping, through the C ABI: the two modes launch the same kernels on the
same data, so every step must give the same bits.

Each case runs two contexts of one problem side by side, one replaying the
captured step graph and one launching eagerly, one step at a time.  After
every step the cores, ranks, rank history and temperature are compared for
equality, and between the replays the test does eager work of its own on
the graph context's stream (energy reductions, core reads, torch kernels)
with synchronisations, so that every replay, not only the first, is checked
against the eager result.
"""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(p, **kw):
    from paper_2503_18056_amd import TTState
    g = TTState(p, device=0, **kw)
    e = TTState(p, device=0, **kw)
    e.use_graphs(False)
    return g, e


def _same(g, e, what):
    import torch
    assert g.ranks() == e.ranks(), what
    for a, b, name in zip(g.cores(), e.cores(), ("X", "Theta", "Phi")):
        assert np.array_equal(a, b), f"{what}: {name} differs"
    assert np.array_equal(g.tt_get_temperature(), e.tt_get_temperature()), what
    assert g.tt_get_rank_history() == e.tt_get_rank_history(), what
    # eager work of the test's own on the graph context's stream between replays
    Eg, rad_g, mat_g = g.tt_energy()
    Ee, rad_e, mat_e = e.tt_energy()
    assert torch.equal(Eg, Ee) and rad_g == rad_e and mat_g == mat_e, what
    x = torch.randn(64, 64, dtype=torch.float64, device=g.device)
    (x @ x).sum().item()
    torch.cuda.synchronize()


def _run(g, e, nsteps, name):
    for m in range(nsteps):
        g.step(1)
        e.step(1)
        _same(g, e, f"{name} step {m + 1}")
    _log(f"{name}: {nsteps} steps identical, ranks {g.ranks()}")


CASES = {
    "frozen_vacuum": (dict(seed=1), {}),
    "coupled_inflow": (dict(bc="inflow", seed=3, material=wl.COUPLED), {}),
    "rusanov_scatter_coupled": (dict(flux="rusanov", bc="mixed", seed=36, material=wl.COUPLED,
                                     scatter=True), {}),
    "outflow_3d": (dict(dim=3, nx=4, ny=3, nz=5, bc="outflow", seed=4), {}),
    "hll_inflow_scatter": (dict(flux="hll", hll_beta=2.5, bc="inflow", seed=42, scatter=True), {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_graph_matches_eager(name):
    kw, ctx_kw = CASES[name]
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    g, e = _pair(p, max_steps=8, **ctx_kw)
    _run(g, e, 8, name)


def test_graph_twice_mixed_and_replay():
    """The two-rounding schedule in the FP32-mixed form, then rank replay
    (the schedule position lives on the device, so replays consume it as
    eager steps do)."""
    from paper_2503_18056_amd import TT_FP32_MIXED, TT_RANK_REPLAY, TT_ROUND_TWICE
    p = wl.small_random(bc="inflow", seed=3, material=wl.COUPLED)
    p["tol"] = 1e-6
    g, e = _pair(p, max_steps=6, schedule=TT_ROUND_TWICE, precision=TT_FP32_MIXED)
    _run(g, e, 6, "twice_mixed")
    pairs = [(2, 2), (3, 2), (2, 1), (3, 3), (1, 1), (2, 2), (3, 2), (2, 2)]
    g, e = _pair(p, max_steps=4, schedule=TT_ROUND_TWICE, rank_mode=TT_RANK_REPLAY)
    g.tt_set_rank_schedule(pairs)
    e.tt_set_rank_schedule(pairs)
    _run(g, e, 4, "twice_replay")


def test_graph_modes_switch_and_profile():
    """Switching modes mid-run, event timing (eager steps) between replays,
    a rounding and new cores between replays, and a non-default stream."""
    import torch
    p = wl.small_random(bc="mixed", seed=7, scatter=True)
    p["tol"] = 1e-6
    from paper_2503_18056_amd import TTState
    stream = torch.cuda.Stream(device=0)
    g = TTState(p, device=0, stream=stream, max_steps=20)
    e = TTState(p, device=0, max_steps=20)
    e.use_graphs(False)
    _run(g, e, 3, "switch a")
    g.use_graphs(False)
    _run(g, e, 2, "switch b (both eager)")
    g.use_graphs(True)
    g.tt_profile_enable(True)
    e.tt_profile_enable(True)
    _run(g, e, 2, "switch c (profiled, eager)")
    g.tt_profile_enable(False)
    e.tt_profile_enable(False)
    _run(g, e, 3, "switch d")
    assert g.tt_round(1e-3) == e.tt_round(1e-3)
    _run(g, e, 2, "switch e (after a rounding)")
    X, Th, Ph = wl.random_tt(g.ns, g.nt, g.np_, 3, 2, 99)
    g.tt_set_cores(np.abs(X), np.abs(Th), np.abs(Ph))
    e.tt_set_cores(np.abs(X), np.abs(Th), np.abs(Ph))
    _run(g, e, 3, "switch f (new cores)")


def test_graph_crossing_beams_full_size():
    """The 256^2 x 32 x 64 crossing-beam workload, 30 steps, graph against
    eager (ranks ramp through the rank capacity's early range)."""
    p = wl.c2(steps=30)
    g, e = _pair(p, max_steps=30)
    for m in range(30):
        g.step(1)
        e.step(1)
        if (m + 1) % 10 == 0:
            _same(g, e, f"crossing beams step {m + 1}")
    _log(f"crossing beams: 30 steps identical, ranks {g.ranks()}")
