"""Parity of the HIP library (through its C ABI) with the CPU oracle.

FP64 bar: identical ranks and a relative Frobenius difference of the
reconstructed intensity below 1e-10 for one step from the same state.
Forming Gram matrices squares their conditioning (App. A.4): a change of a
Gram matrix by one unit roundoff of its largest entry -- the norm-wise
backward error of any backward-stable FP64 eigensolver -- can move the
oracle's own step by more than 1e-10 when kept singular values are tiny
against sigma_1 (more accurate Gram sums do not help; a CPU pin shows it).
Each single-step comparison is therefore tagged: "pinned" where that spread
of the oracle is below 1e-11 (bar 1e-10), "unpinned (eigensolver floor)"
elsewhere (bar: four times the spread, printed with the difference).

Multi-step runs: free-running, the ranks must equal the oracle's until the
oracle meets a rank decision within MARGIN of its threshold (there FP64
rounding decides, on either side); with the oracle's rank history replayed,
values must agree over the whole run.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, rounding, tt

pytestmark = pytest.mark.gpu


def _state(p, **kw):
    from paper_2503_18056_amd import TTState
    return TTState(p, device=0, **kw)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ rounding
@pytest.mark.parametrize("seed", [0, 1])
def test_round_random_tt(seed):
    X, Th, Ph = wl.random_tt(300, 6, 12, 8, 5, seed, decay=0.15)
    p = wl.small_random(nx=20, ny=15, ntheta=6, nphi=12, seed=seed)
    st = _state(p, cores=(X, Th, Ph), r1_cap=8, r2_cap=5)
    r = st.tt_round(1e-5, 0)
    (Xo, To, Po), (i1, i2) = rounding.round_gram(X, Th, Ph, 1e-5, 0)
    got = st.cores()
    err = metrics.rel_diff(got, (Xo, To, Po))
    _log(f"round seed={seed} ranks gpu={r} oracle={(Xo.shape[1], Po.shape[0])} err={err:.2e}")
    assert r == (Xo.shape[1], Po.shape[0])
    assert err < 1e-10
    Xg = got[0]
    assert np.allclose(Xg.T @ Xg, np.eye(Xg.shape[1]), atol=1e-10)


def test_round_constructed_spectrum():
    rng = np.random.default_rng(0)
    s = 10.0 ** (-np.arange(10) / 1.5)
    ns, nt, npf = 240, 5, 16
    X = np.linalg.qr(rng.standard_normal((ns, 10)))[0]
    Ph = np.linalg.qr(rng.standard_normal((npf, 10)))[0].T
    Th = np.zeros((10, nt, 10))
    for a in range(10):
        Th[a, a % nt, a] = s[a]
    p = wl.small_random(nx=16, ny=15, ntheta=nt + 1, nphi=npf, seed=0)
    p["ntheta"] = nt + 1  # even ntheta required: pad one zero slice
    Thp = np.zeros((10, nt + 1, 10)); Thp[:, :nt] = Th
    st = _state(p, cores=(X, Thp, Ph), r1_cap=10, r2_cap=10)
    tol = 1e-4
    r = st.tt_round(tol, 0)
    delta2 = tol ** 2 * np.sum(s ** 2) / 2
    tail = np.array([np.sum(s[k:] ** 2) for k in range(11)])
    expect = int(np.argmax(tail <= delta2))
    info = st.tt_get_round_info()
    _log("spectrum ranks", r, "expect", expect, "s1", info["s1"])
    assert r == (expect, expect)
    assert abs(info["s1"] - s[0]) < 1e-12


def test_round_rank_one_and_zero():
    p = wl.c1()
    st = _state(p)
    assert st.tt_round(1e-8, 0) == (1, 1)
    X, Th, Ph = st.cores()
    T0 = metrics.reconstruct(p["X0"], p["Th0"], p["Ph0"])
    assert np.linalg.norm(metrics.reconstruct(X, Th, Ph) - T0) < 1e-14 * np.linalg.norm(T0)
    p2 = wl.small_random(seed=4)
    st2 = _state(p2, cores=(np.zeros((30, 3)), np.ones((3, 4, 2)), np.ones((2, 8))))
    assert st2.tt_round(1e-6, 0) == (1, 1)
    X, Th, Ph = st2.cores()
    assert not np.any(metrics.reconstruct(X, Th, Ph))


# ------------------------------------------------------------------- steps
CASES = [
    dict(seed=1),
    dict(bc="periodic", seed=2),
    dict(bc="inflow", seed=3, material=wl.COUPLED),
    dict(dim=3, nx=4, ny=3, nz=5, bc="inflow", seed=4, material=wl.COUPLED),
    dict(dim=3, nx=5, ny=4, nz=4, bc="periodic", seed=5),
    dict(nx=33, ny=17, ntheta=8, nphi=16, r1=5, r2=3, seed=6, bc="inflow"),
]


@pytest.mark.parametrize("kw", CASES, ids=[f"case{i}" for i in range(len(CASES))])
def test_step_matches_oracle(kw):
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    s = Setup(p)
    nsteps = 3
    st = _state(p, max_steps=nsteps)
    st.step(1)
    (X1, T1c, P1), T1, _ = tt.run(s, 1)
    err1 = metrics.rel_diff(st.cores(), (X1, T1c, P1))
    st.step(nsteps - 1)
    hist_gpu = st.tt_get_rank_history()
    (X, Th, Ph), T, hist = tt.run(s, nsteps)
    got = st.cores()
    err = metrics.rel_diff(got, (X, Th, Ph))
    Tg = st.tt_get_temperature()
    terr = np.max(np.abs(Tg - T)) / np.max(np.abs(T))
    _log(f"{p['name']}: ranks gpu={hist_gpu} oracle={hist} step1 err={err1:.2e} "
         f"step{nsteps} err={err:.2e} Terr={terr:.2e}")
    assert hist_gpu == hist
    assert err1 < 1e-10
    assert err < 1e-8
    assert terr < 1e-10


def test_energy_matches_oracle():
    p = wl.small_random(bc="inflow", seed=8, material=wl.COUPLED)
    s = Setup(p)
    st = _state(p)
    st.step(2)
    E, rad, mat = st.tt_energy()
    (X, Th, Ph), T, _ = tt.run(s, 2)
    Eo = tt.energy(X, Th, Ph, s)
    e = E.cpu().numpy()
    assert np.max(np.abs(e - Eo)) < 1e-10 * np.max(np.abs(Eo))
    assert abs(rad - Eo.sum() * s.cell_volume) < 1e-10 * abs(rad)
    assert abs(mat - np.sum(s.rho * s.cv * T) * s.cell_volume) < 1e-10 * abs(mat)


SPREAD_FACTOR = 4.0
PIN_SPREAD = 1e-11  # the oracle's own spread below which a comparison is pinned at 1e-10
MARGIN = 1e-3  # rank decisions closer than this to their threshold are rounding-determined


def _oracle_spread(X, Th, Ph, s, p, ref, seeds=(0, 1)):
    """Largest relative change of the oracle's step (its ranks replayed) when
    every Gram matrix is moved by a seeded symmetric perturbation of one unit
    roundoff of its largest entry: the norm-wise backward error that any
    backward-stable FP64 eigensolver leaves (its Gram sums are far more
    accurate than that; see the CPU pin of this reading)."""
    worst = 0.0
    ranks = (ref[0].shape[1], ref[2].shape[0])
    for sd in seeds:
        rng = np.random.default_rng(1000 + sd)

        def pert(G):
            E = rng.uniform(-1.0, 1.0, G.shape)
            return G + rounding.U * np.abs(G).max() * 0.5 * (E + E.T)
        b, _, _ = tt.step(X, Th, Ph, s.T0, s, p["tol"], p["rmax"], ranks=ranks, perturb=pert)
        worst = max(worst, metrics.rel_diff(b, ref))
    return worst


def _single_step_parity(p, states, steps_to_check, tol_single=1e-10):
    """One GPU step from the oracle's own state m against the oracle's step
    from the same state.  Every comparison is tagged and printed:

    - pinned: the oracle's own spread (``_oracle_spread``) is below 1e-11,
      so an independent FP64 implementation is held to 1e-10 with identical
      ranks;
    - unpinned (eigensolver floor): the spread is larger; the bar is
      SPREAD_FACTOR times the spread, printed beside the measured difference.

    Where the oracle's own rank decision lies within MARGIN of its threshold
    the ranks may differ; the test checks the margin, replays the oracle's
    ranks and tags the comparison 'rank decision replayed'.  Returns
    (worst pinned difference, number pinned, number unpinned)."""
    from paper_2503_18056_amd import TT_RANK_REPLAY
    s = Setup(p)
    worst_pinned, npin, nun = 0.0, 0, 0
    st = _state(p, max_steps=4)
    for m in steps_to_check:
        X, Th, Ph = states[m]
        st.tt_set_cores(X, Th, Ph)
        st.step(1)
        got = st.cores()
        (Xo, To, Po), _, info = tt.step(X, Th, Ph, s.T0, s, p["tol"], p["rmax"])
        ro = (Xo.shape[1], Po.shape[0])
        note = ""
        if st.ranks() != ro:
            margin = min(b.get("margin", np.inf) for b in info["round"][-1])
            assert margin < MARGIN, (m, st.ranks(), ro, margin)
            note = f", rank decision replayed (gpu {st.ranks()}, oracle margin {margin:.1e})"
            sr = _state(p, max_steps=4, rank_mode=TT_RANK_REPLAY)
            sr.tt_set_cores(X, Th, Ph)
            sr.tt_set_rank_schedule([ro])
            sr.step(1)
            assert sr.ranks() == ro
            got = sr.cores()
            sr.close()
        err = metrics.rel_diff(got, (Xo, To, Po))
        spread = _oracle_spread(X, Th, Ph, s, p, (Xo, To, Po))
        if spread < PIN_SPREAD:
            tag, bar = "pinned", tol_single
            npin += 1
            worst_pinned = max(worst_pinned, err)
        else:
            tag, bar = "unpinned (eigensolver floor)", max(tol_single, SPREAD_FACTOR * spread)
            nun += 1
        _log(f"  {p['name']} state {m}: ranks {ro} err={err:.2e} [{tag}; oracle spread "
             f"{spread:.2e}, bar {bar:.1e}{note}]")
        assert err < bar
    _log(f"  {p['name']}: {npin} pinned (worst {worst_pinned:.2e} < {tol_single:.0e}), "
         f"{nun} unpinned")
    return worst_pinned, npin, nun


def _trajectory(p, nsteps):
    s = Setup(p)
    states = [(np.asarray(p["X0"], float), np.asarray(p["Th0"], float), np.asarray(p["Ph0"], float))]
    infos = []

    def cb(m, c, T, i):
        states.append(c)
        infos.append(i)
    tt.run(s, nsteps, callback=cb)
    return states, infos


def _free_run(p, states, infos, nsteps, bound):
    """The library stepping on its own from the initial state: ranks equal the
    oracle's at every step until the oracle meets a rank decision within
    MARGIN of its threshold (tail vs delta^2 or a tie test), where FP64
    rounding of either side decides it; the end state is within ``bound``."""
    st = _state(p, max_steps=nsteps)
    st.step(nsteps)
    hist_gpu = [tuple(h) for h in st.tt_get_rank_history()]
    hist = [(c[0].shape[1], c[2].shape[0]) for c in states[1:]]
    compared = nsteps
    for k, (g, o) in enumerate(zip(hist_gpu, hist)):
        if g != o:
            margin = min(b.get("margin", np.inf) for b in infos[k]["round"][-1])
            _log(f"  {p['name']}: step {k + 1} gpu ranks {g} oracle {o} (oracle's margin {margin:.2e})")
            assert margin < MARGIN, (k + 1, g, o, margin)
            compared = k
            break
    err = metrics.rel_diff(st.cores(), states[-1])
    _log(f"  {p['name']} free run: ranks identical for {compared}/{nsteps} steps, end err={err:.2e}")
    assert err < bound
    return hist


def _replay_run(p, hist, states, nsteps, bound):
    """The library replaying the oracle's rank history: the same ranks by
    construction, values within ``bound`` after ``nsteps`` steps."""
    from paper_2503_18056_amd import TT_RANK_REPLAY
    st = _state(p, max_steps=nsteps, rank_mode=TT_RANK_REPLAY)
    st.tt_set_rank_schedule(hist)
    st.step(nsteps)
    assert [tuple(h) for h in st.tt_get_rank_history()] == hist
    err = metrics.rel_diff(st.cores(), states[-1])
    _log(f"  {p['name']} replayed ranks: {nsteps}-step err={err:.2e}")
    assert err < bound


def test_c1_parity():
    """C1 (32^2, 8x16, 10 steps, tolerance 1e-8 at the FP64 Gram floor, and
    the same case at 1e-6): every step from the oracle's state matches (see
    _single_step_parity) with identical ranks; the free-running 10-step
    runs keep the oracle's ranks (see _free_run) and, like the runs with the
    oracle's ranks replayed, end within 2e-8 (about ten times the measured
    0.9-1.8e-9)."""
    for tol in (1e-6, 1e-8):
        p = wl.c1()
        p["tol"] = tol
        states, infos = _trajectory(p, 10)
        _single_step_parity(p, states, range(10))
        hist = _free_run(p, states, infos, 10, 2e-8)
        _replay_run(p, hist, states, 10, 2e-8)


def test_c2_parity():
    """C2 (256^2, 32x64, cap 64), first 40 steps: single steps from oracle
    states (see _single_step_parity) with identical ranks; the free run keeps
    the oracle's ranks up to a rounding-determined decision and ends within
    1.5e-6 (about ten times the measured 0.45-1.3e-7, the upper value when a
    rank decision inside MARGIN went the other way); with the oracle's ranks
    replayed the 40-step run agrees to 5e-7 (measured 4.5e-8)."""
    p = wl.c2(steps=40)
    states, infos = _trajectory(p, 40)
    _single_step_parity(p, states, [0, 1, 2, 5, 13, 20, 39])
    hist = _free_run(p, states, infos, 40, 1.5e-6)
    _replay_run(p, hist, states, 40, 5e-7)
