"""Reduced-size analytic validation: the hohlraum (Sec. 5.1) through the C
ABI.

Isotropic inflow I = 1 through the x-lo and y-lo faces into vacuum; the
mean intensity J = c E / (4 pi) at t = 0.75 is compared over the cells of
[0, 1]^2 (causally disconnected from the far faces) with the analytic J of
Sec. 5.1 (`oracle.analytic.hohlraum_J`, itself pinned by direct quadrature
in test_oracle_pins.py), as an area-weighted L1 error.

- 64^2 cells, 16 x 32 ordinates, tolerance 1e-4, rank cap 128 (48 steps;
  the ranks grow to about (107, 24) without reaching the cap, so the
  concatenated rank passes 500 and the wide Gram and the grid reductions
  run): the library's state against the TT oracle's (unpinned, to 1e-6),
  and the same L1 error as the oracle's to 1e-7.
- 64^2, 128^2, 256^2 cells, 32 x 64 ordinates, rank cap 160: the L1 error
  falls at first order in the cell size (the scheme is first order in
  space, Sec. 5.1).
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, tt
from oracle.analytic import hohlraum_J

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _state(p, **kw):
    from paper_2503_18056_amd import TTState
    return TTState(p, device=0, **kw)


def _l1(E, p):
    """Area-weighted L1 error of J = c E / 4 pi over [0, 1]^2."""
    n = p["nx"]
    J = p["c"] * np.asarray(E).reshape(n, n) / (4 * np.pi)
    xc = (np.arange(n) + 0.5) * p["lx"] / n
    Ja = hohlraum_J(p["hohlraum"]["t"], xc[None, :], xc[:, None], p["c"])
    m = int(round(n / p["lx"]))
    return float(np.abs(J[:m, :m] - Ja[:m, :m]).sum() * (p["lx"] / n) ** 2)


def test_hohlraum_reduced_vs_oracle_and_analytic():
    p = wl.hohlraum(n=64, ntheta=16, nphi=32, tol=1e-4, rmax=128)
    nsteps = p["steps"]
    _log(f"hohlraum 64^2 16x32: {nsteps} steps")
    st = _state(p, max_steps=nsteps)
    st.step(nsteps)
    hist_gpu = st.tt_get_rank_history()
    s = Setup(p)
    (X, Th, Ph), _, hist = tt.run(s, nsteps)
    err = metrics.rel_diff(st.cores(), (X, Th, Ph))
    l1_gpu = _l1(st.tt_energy()[0].cpu().numpy(), p)
    l1_or = _l1(tt.energy(X, Th, Ph, s), p)
    same = hist_gpu == hist
    _log(f"hohlraum: ranks gpu {hist_gpu[-1]} oracle {hist[-1]}, identical {same}; state err {err:.2e}; "
         f"L1 gpu {l1_gpu:.6e} oracle {l1_or:.6e}")
    if not same:
        # a near-tie at some cut: replay the oracle's ranks (parity of the map)
        from paper_2503_18056_amd import TT_RANK_REPLAY
        sr = _state(p, max_steps=nsteps, rank_mode=TT_RANK_REPLAY)
        sr.tt_set_rank_schedule(hist)
        sr.step(nsteps)
        err = metrics.rel_diff(sr.cores(), (X, Th, Ph))
        l1_gpu = _l1(sr.tt_energy()[0].cpu().numpy(), p)
        _log(f"hohlraum replayed: state err {err:.2e}, L1 gpu {l1_gpu:.6e}")
    # unpinned (Gram floor): 48 free-running steps at ranks near 100, each
    # rounding resolving the spectrum near its cut only to the Gram route's
    # floor (about sqrt(u) sigma_1); measured 2.7e-7, bar 100 times below the
    # rounding tolerance.  The L1 errors, the physics check, agree to 1e-9.
    assert err < 1e-6
    assert abs(l1_gpu - l1_or) < 1e-7
    assert l1_gpu < 1e-2


def test_hohlraum_first_order_convergence():
    l1 = []
    for n in (64, 128, 256):
        p = wl.hohlraum(n=n, ntheta=32, nphi=64, tol=1e-4, rmax=160)
        _log(f"hohlraum {n}^2 32x64: {p['steps']} steps")
        st = _state(p, max_steps=p["steps"])
        st.step(p["steps"])
        l1.append(_l1(st.tt_energy()[0].cpu().numpy(), p))
        _log(f"  ranks {st.tt_get_rank_history()[-1]}, L1 {l1[-1]:.4e}")
    assert l1[0] < 1e-2
    assert l1[1] < 0.65 * l1[0]
    assert l1[2] < 0.65 * l1[1]
