"""Randomized TT rounding on the GPU (App. A.3, eqs. randfinal and
randprojection) against the oracle's `rounding.round_randomized`, through
the C ABI, with the same seeded Gaussian test matrices.

- A state whose spectra decay geometrically in both bonds, rounded to
  several target-rank pairs (fewer than, and equal to, its ranks): the
  rounded tensor matches the oracle's to 1e-12 relative (the two sides
  orthonormalise the same sketch, the oracle by Householder QR, the library
  by shifted CholeskyQR3; measured 1e-15 to 7e-15), and both left factors
  have orthonormal columns to 1e-13.
- A TT whose bond ranks exceed the tensor's (ranks (6, 4) holding a
  rank-(3, 2) tensor) is reproduced to 1e-12 at the true ranks.
- The rounded state is a valid state: its energy density is the oracle's
  of the same cores, and a step from it matches the oracle's step.
- Sizes outside the contract and FP32-mixed contexts are refused.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, rounding, tt

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _state(p, cores, **kw):
    from paper_2503_18056_amd import TTState
    return TTState(p, device=0, cores=cores, **kw)


def _problem():
    return wl.small_random(nx=24, ny=20, ntheta=8, nphi=16, seed=71)


def _decaying_tt(p, r1, r2, seed, decay=0.55):
    rng = np.random.default_rng(seed)
    ns, nt, npf = p["nx"] * p["ny"], p["ntheta"], p["nphi"]
    X = np.linalg.qr(rng.standard_normal((ns, r1)))[0]
    sc = (decay ** np.arange(r1))[:, None, None] * (decay ** np.arange(r2))[None, None, :]
    Th = rng.standard_normal((r1, nt, r2)) * sc
    Ph = np.linalg.qr(rng.standard_normal((npf, r2)))[0].T
    return X, Th, Ph


def _orth_err(A):
    return float(np.abs(A.T @ A - np.eye(A.shape[1])).max())


@pytest.mark.parametrize("k1,k2", [(16, 8), (10, 5), (24, 12), (7, 12)])
def test_randomized_rounding_matches_the_oracle(k1, k2):
    p = _problem()
    X, Th, Ph = _decaying_tt(p, 24, 12, seed=72)
    om = wl.gaussian_test_matrices(p["ntheta"], p["nphi"], k1, k2, seed=73)
    st = _state(p, (X, Th, Ph))
    assert st.tt_round_randomized(*om) == (k1, k2)
    Xg, Thg, Phg = st.tt_get_cores()
    Xo, Tho, Pho = rounding.round_randomized(X, Th, Ph, om)
    err = metrics.rel_diff((Xg, Thg, Phg), (Xo, Tho, Pho))
    full = metrics.rel_diff((Xg, Thg, Phg), (X, Th, Ph))
    ox, ot = _orth_err(Xg), _orth_err(Thg.reshape(k1 * p["ntheta"], k2))
    _log(f"randomized ({k1}, {k2}): vs oracle {err:.2e}, vs the unrounded TT {full:.2e}, "
         f"orthonormality X {ox:.1e} Theta {ot:.1e}")
    assert err < 1e-12
    assert ox < 1e-13 and ot < 1e-13


def test_randomized_rounding_past_the_numerical_rank():
    """Target ranks beyond the state's numerical ranks (singular values
    0.05^i in both bonds: rounding level past about 12): the sketch is
    numerically rank deficient, the second shifted pass lifts its null
    directions, and the result is the unrounded tensor to rounding with
    orthonormal factors."""
    p = _problem()
    X, Th, Ph = _decaying_tt(p, 24, 12, seed=81, decay=0.05)
    om = wl.gaussian_test_matrices(p["ntheta"], p["nphi"], 20, 12, seed=82)
    st = _state(p, (X, Th, Ph))
    assert st.tt_round_randomized(*om) == (20, 12)
    Xg, Thg, Phg = st.tt_get_cores()
    full = metrics.rel_diff((Xg, Thg, Phg), (X, Th, Ph))
    ox, ot = _orth_err(Xg), _orth_err(Thg.reshape(20 * p["ntheta"], 12))
    _log(f"past the numerical rank: vs the unrounded TT {full:.2e}, orthonormality X {ox:.1e} "
         f"Theta {ot:.1e}")
    assert full < 1e-13
    assert ox < 1e-13 and ot < 1e-13


def test_randomized_rounding_exact_on_padded_low_rank():
    p = _problem()
    rng = np.random.default_rng(74)
    ns, nt, npf = p["nx"] * p["ny"], p["ntheta"], p["nphi"]
    X = rng.standard_normal((ns, 3))
    Th = rng.standard_normal((3, nt, 2))
    Ph = rng.standard_normal((2, npf))
    Thc = np.zeros((6, nt, 4))
    Thc[:3, :, :2] = Th
    Thc[3:, :, 2:] = Th
    st = _state(p, (np.hstack([X, 2.0 * X]), Thc, np.vstack([Ph, Ph])))
    om = wl.gaussian_test_matrices(nt, npf, 3, 2, seed=75)
    assert st.tt_round_randomized(*om) == (3, 2)
    R = metrics.reconstruct(*st.tt_get_cores())
    T = 3.0 * metrics.reconstruct(X, Th, Ph)
    err = np.linalg.norm(R - T) / np.linalg.norm(T)
    _log(f"padded low rank: {err:.2e}")
    assert err < 1e-12


def test_randomized_rounding_leaves_a_valid_state():
    p = _problem()
    p["tol"] = 1e-6
    X, Th, Ph = _decaying_tt(p, 24, 12, seed=76)
    om = wl.gaussian_test_matrices(p["ntheta"], p["nphi"], 16, 8, seed=77)
    st = _state(p, (X, Th, Ph), max_steps=2)
    st.tt_round_randomized(*om)
    Xr, Thr, Phr = st.tt_get_cores()
    s = Setup(p)
    Eg = st.tt_energy()[0].cpu().numpy()
    Eo = tt.energy(Xr, Thr, Phr, s)
    assert np.max(np.abs(Eg - Eo)) < 1e-12 * np.max(np.abs(Eo))
    st.step(1)
    Eg1 = st.tt_energy()[0].cpu().numpy()
    (X1, Th1, Ph1), _, _ = tt.step(Xr, Thr, Phr, s.T0, s, p["tol"], 0)
    Eo1 = tt.energy(X1, Th1, Ph1, s)
    e = np.max(np.abs(Eg1 - Eo1)) / np.max(np.abs(Eo1))
    _log(f"step after randomized rounding: energy density vs oracle {e:.2e}")
    assert e < 1e-6


def test_randomized_rounding_refuses_bad_sizes():
    from paper_2503_18056_amd import TT_FP32_MIXED, TTError
    p = _problem()
    X, Th, Ph = _decaying_tt(p, 24, 12, seed=78)
    st = _state(p, (X, Th, Ph))
    for k1, k2 in ((25, 4), (8, 13), (0, 4)):
        om = wl.gaussian_test_matrices(p["ntheta"], p["nphi"], max(k1, 1), k2, seed=79)
        if k1 == 0:
            om = (om[0][:, :0], om[1])
        with pytest.raises(TTError):
            st.tt_round_randomized(*om)
    assert st.ranks() == (24, 12)
    sm = _state(p, (X, Th, Ph), precision=TT_FP32_MIXED)
    with pytest.raises(TTError):
        sm.tt_round_randomized(*wl.gaussian_test_matrices(p["ntheta"], p["nphi"], 8, 4, seed=80))
