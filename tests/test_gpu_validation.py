"""Reduced-size analytic validations through the C ABI: the hohlraum
(Sec. 5.1) and the line source's energy conservation and profile (Sec. 5.4).

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

Line source: an isotropic Gaussian pulse (width 0.03, U0 = 1) in vacuum on
[-1.1, 1.1]^2, run to t = 0.5 so that the front stays inside the domain and
the upwind scheme moves energy only between cells: what the total loses is
what the roundings drop.  Sec. 5.4 reports conservation errors of 8e-5 U0
(tolerance 1e-4) and 2e-4 U0 (tolerance 1e-3) for its full run.
- 64^2 cells, 16 x 32 ordinates, both tolerances: the library's total energy
  after every step against the TT oracle's (parity), both under those
  figures.
- 256^2 cells, 16 x 32 ordinates, both tolerances: under those figures.
- The profile (Sec. 5.4 compares azimuthal averages with the exact
  solution): the azimuthal average of E over annuli one cell wide against
  that of the Gaussian-smoothed analytic solution
  (`oracle.analytic.line_source_smoothed_E`, pinned in test_oracle_pins.py),
  as an L1 distance relative to U0, at 64^2 / 8 x 16, 128^2 / 16 x 32 and
  256^2 / 32 x 64 (tolerance 1e-4): it falls with each refinement of space
  and angle together (measured 0.427, 0.287, 0.186; the full-grid oracle
  gives the same first two); the error is the first-order scheme's smearing of the ring and
  the ray effects of the coarse ordinates, as Sec. 5.4 discusses.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import Setup, metrics, tt
from oracle.analytic import hohlraum_J, line_source_smoothed_E

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


def _total(E, p):
    return float(np.sum(E)) * (p["lx"] / p["nx"]) * (p["ly"] / p["ny"])


@pytest.mark.parametrize("tol,paper", [(1e-4, 8e-5), (1e-3, 2e-4)])
def test_line_source_conservation_vs_oracle(tol, paper):
    p = wl.line_source(n=64, ntheta=16, nphi=32, tol=tol, rmax=200)
    nsteps = p["steps"]
    _log(f"line source 64^2 16x32 tol {tol}: {nsteps} steps")
    s = Setup(p)
    E0 = _total(tt.energy(p["X0"], p["Th0"], p["Ph0"], s), p)
    def run_gpu(**kw):
        st = _state(p, max_steps=nsteps, **kw)
        if kw:
            st.tt_set_rank_schedule(hist)
        e = []
        for _ in range(nsteps):
            st.step(1)
            e.append(_total(st.tt_energy()[0].cpu().numpy(), p))
        return st, np.array(e)

    eo = []
    _, _, hist = tt.run(s, nsteps, callback=lambda m, c, T, i: eo.append(_total(tt.energy(*c, s), p)))
    eo = np.array(eo)
    st, eg = run_gpu()
    cg, co = np.max(np.abs(eg - E0)), np.max(np.abs(eo - E0))
    same = st.tt_get_rank_history() == hist
    _log(f"  ranks gpu {st.tt_get_rank_history()[-1]} oracle {hist[-1]} identical {same}; conservation "
         f"error gpu {cg:.3e} oracle {co:.3e}; totals differ by {np.max(np.abs(eg - eo)):.2e}")
    if not same:
        # a near-tie at some cut: the same map with the oracle's ranks replayed
        from paper_2503_18056_amd import TT_RANK_REPLAY
        _, er = run_gpu(rank_mode=TT_RANK_REPLAY)
        _log(f"  replayed ranks: totals differ by {np.max(np.abs(er - eo)):.2e}")
    else:
        er = eg
    # unpinned (Gram floor): each rounding drops, to within the Gram route's
    # floor, the same part of the spectrum on both sides; measured 3.5e-9 of
    # U0 at tolerance 1e-4 against conservation errors near 2e-8
    assert np.max(np.abs(er - eo)) < 1e-7
    assert cg < 10 * co + 1e-8
    assert cg < paper


def test_line_source_256_conservation():
    for tol, paper in ((1e-4, 8e-5), (1e-3, 2e-4)):
        p = wl.line_source(n=256, ntheta=16, nphi=32, tol=tol, rmax=204)
        _log(f"line source 256^2 16x32 tol {tol}: {p['steps']} steps")
        s = Setup(p)
        E0 = _total(tt.energy(p["X0"], p["Th0"], p["Ph0"], s), p)
        st = _state(p, max_steps=p["steps"])
        st.step(p["steps"])
        err = abs(_total(st.tt_energy()[0].cpu().numpy(), p) - E0)
        _log(f"  ranks {st.tt_get_rank_history()[-1]} (cap 204), conservation error {err:.3e} "
             f"(Sec. 5.4: {paper:.0e} for its full run)")
        assert err < paper


def _azimuthal_l1(E, p):
    """L1 distance, relative to U0, between the azimuthal averages of E and
    of the smoothed analytic solution over annuli one cell wide about the
    pulse's centre (each annulus weighted by its cells' area)."""
    n = p["nx"]
    dx = p["lx"] / n
    xs = (np.arange(n) + 0.5) * dx - 0.5 * p["lx"]
    R = np.sqrt(xs[None, :] ** 2 + xs[:, None] ** 2).reshape(-1)
    ls = p["line_source"]
    Ea = line_source_smoothed_E(ls["t"], R, U0=ls["U0"], omega=ls["omega"], c=p["c"])
    b = np.floor(R / dx).astype(int)
    cnt = np.bincount(b)
    Eb = np.bincount(b, np.asarray(E).reshape(-1)) / np.maximum(cnt, 1)
    Ab = np.bincount(b, Ea) / np.maximum(cnt, 1)
    return float(np.sum(np.abs(Eb - Ab) * cnt) * dx * dx / ls["U0"])


def test_line_source_profile_converges_to_the_smoothed_solution():
    errs = []
    for n, nt, npf in ((64, 8, 16), (128, 16, 32), (256, 32, 64)):
        p = wl.line_source(n=n, ntheta=nt, nphi=npf, tol=1e-4, rmax=200)
        _log(f"line source {n}^2 {nt}x{npf}: {p['steps']} steps")
        st = _state(p, max_steps=p["steps"])
        st.step(p["steps"])
        errs.append(_azimuthal_l1(st.tt_energy()[0].cpu().numpy(), p))
        _log(f"  ranks {st.tt_get_rank_history()[-1]}, azimuthal L1 {errs[-1]:.4f}")
    assert errs[0] < 0.5
    assert errs[1] < 0.8 * errs[0]
    assert errs[2] < 0.8 * errs[1]
