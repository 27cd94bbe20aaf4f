"""FP32-mixed precision form (TT_FP32_MIXED) of the library against the FP64
CPU oracle, through the C ABI.

The mixed form stores the spatial core X and the concatenated core X_cat in
FP32, forms the N_s-long Gram by error-free slicing on FP32 MFMA (exact to
2^-44 of the column scales, so singular values down to the truncation
tolerance keep their meaning) and the core update X_cat P by split products
on FP32 MFMA; the eigensolves, the SVD of M, the rank rule, the inverse
square-root scalings, the angular cores and the energy / temperature update
stay FP64.  Each step therefore rounds the state to FP32 once (relative
2^-24 per entry).

Bars: small cases, 3 steps, relative Frobenius difference from the oracle
below 1e-6 (FP32 storage alone contributes ~1e-7) and temperature within
1e-5 (its update differences two energies of FP32-stored cores); a
standalone rounding below 1e-6; the
crossing-beam workload over its 400 steps at tolerance 1e-6 below 1e-5
(the target), with the rank history compared step by step against the
oracle's.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, rounding, tt

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _mixed(p, **kw):
    from paper_2503_18056_amd import TT_FP32_MIXED, TTState
    return TTState(p, device=0, precision=TT_FP32_MIXED, **kw)


CASES = [
    dict(seed=1),
    dict(bc="periodic", seed=2),
    dict(bc="inflow", seed=3, material=wl.COUPLED),
    dict(dim=3, nx=4, ny=3, nz=5, bc="inflow", seed=4, material=wl.COUPLED),
    dict(nx=33, ny=17, ntheta=8, nphi=16, r1=5, r2=3, seed=6, bc="inflow"),
]


@pytest.mark.parametrize("kw", CASES, ids=[f"case{i}" for i in range(len(CASES))])
def test_mixed_steps_vs_oracle(kw):
    p = wl.small_random(**kw)
    p["tol"] = 1e-6
    s = Setup(p)
    st = _mixed(p, max_steps=3)
    st.step(3)
    hist_gpu = st.tt_get_rank_history()
    (X, Th, Ph), T, hist = tt.run(s, 3)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    terr = np.max(np.abs(st.tt_get_temperature() - T)) / np.max(np.abs(T))
    _log(f"mixed {p['name']}: ranks gpu={hist_gpu} oracle={hist} 3-step err={err:.2e} Terr={terr:.2e}")
    assert err < 1e-6
    # the temperature update is FP64, but it takes the difference E* - E of two
    # energies of FP32-stored cores: ~2^-24 E / (rho c_v) per step
    assert terr < 1e-5


def test_gram_slices():
    """tt_set_gram_slices: 4 slices (the default) give the default's bits;
    every count 1 .. 6 runs; 3 or more (33+ bits, all of FP32's 24) keep the
    3-step result within the default's bar of the oracle; 1 slice (11 bits)
    is worse than 4; counts outside 1 .. 6 are rejected."""
    p = wl.small_random(bc="inflow", seed=3, material=wl.COUPLED)
    p["tol"] = 1e-6
    (X, Th, Ph), _, _ = tt.run(Setup(p), 3)
    base = _mixed(p, max_steps=3)
    base.step(3)
    errs = {}
    for sl in range(1, 7):
        st = _mixed(p, max_steps=3)
        st.tt_set_gram_slices(sl)
        st.step(3)
        if sl == 4:
            for a, b in zip(st.cores(), base.cores()):
                assert np.array_equal(a, b)
        errs[sl] = metrics.rel_diff(st.cores(), (X, Th, Ph))
        assert np.isfinite(errs[sl])
        if sl >= 3:
            assert errs[sl] < 1e-6, (sl, errs[sl])
        if sl == 6:
            for bad in (0, 7):
                with pytest.raises(Exception):
                    st.tt_set_gram_slices(bad)
        st.close()
    _log("gram slices: 3-step err vs oracle " + ", ".join(f"{k}: {v:.2e}" for k, v in errs.items()))
    assert errs[1] > errs[4]


def test_mixed_round_vs_oracle():
    X, Th, Ph = wl.random_tt(300, 6, 12, 8, 5, 0, decay=0.15)
    p = wl.small_random(nx=20, ny=15, ntheta=6, nphi=12, seed=0)
    st = _mixed(p, cores=(X, Th, Ph), r1_cap=8, r2_cap=5)
    r = st.tt_round(1e-5, 0)
    (Xo, To, Po), _ = rounding.round_gram(X, Th, Ph, 1e-5, 0)
    err = metrics.rel_diff(st.cores(), (Xo, To, Po))
    _log(f"mixed round: ranks gpu={r} oracle={(Xo.shape[1], Po.shape[0])} err={err:.2e}")
    assert r == (Xo.shape[1], Po.shape[0])
    assert err < 1e-6


def test_mixed_crossing_beams_400_steps_vs_oracle():
    """The crossing-beam workload (256^2 cells, 32x64 ordinates, tolerance
    1e-6, cap 64) over all 400 steps: the mixed form within 1e-5 of the FP64
    oracle, the FP64 form within 1.5e-6 (about ten times its measured
    1.4e-7)."""
    from paper_2503_18056_amd import TTState
    p = wl.c2(steps=400)
    s = Setup(p)
    hist = []
    (X, Th, Ph), _, _ = tt.run(s, 400, callback=lambda m, c, T, i: hist.append((c[0].shape[1], c[2].shape[0])))
    st = _mixed(p, max_steps=400)
    st.step(400)
    hm = [tuple(h) for h in st.tt_get_rank_history()]
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    s64 = TTState(p, device=0, max_steps=400)
    s64.step(400)
    h64 = [tuple(h) for h in s64.tt_get_rank_history()]
    err64 = metrics.rel_diff(s64.cores(), (X, Th, Ph))
    same = sum(a == b for a, b in zip(hm, hist))
    same64 = sum(a == b for a, b in zip(h64, hist))
    _log(f"crossing beams 400 steps: mixed err={err:.2e} (ranks equal to the oracle's at "
         f"{same}/400 steps, end {hm[-1]} vs {hist[-1]}); fp64 err={err64:.2e} ({same64}/400)")
    assert err < 1e-5
    assert err64 < 1.5e-6
