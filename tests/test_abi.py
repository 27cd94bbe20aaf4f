"""Host-side checks of the C ABI (no GPU needed, no device work issued).

The library must load, export every entry point declared in include/tt.h,
and reject invalid configurations on the host before touching the device.
"""
import ctypes as C
import os
import re

import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tt.h")).read()
    src += open(os.path.join(ROOT, "include", "tt_kernels.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tt_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_18056_amd import _ffi
    return _ffi.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 15
    from paper_2503_18056_amd import _ffi
    for n in names:
        assert hasattr(lib, n), n
        assert n in _ffi.SIGNATURES, n


def _cfg(**kw):
    from paper_2503_18056_amd import make_config
    p = wl.c2()
    for k, v in kw.items():
        p[k] = v
    return make_config(p)


def test_workspace_and_validation(lib):
    cfg = _cfg()
    nb = lib.tt_workspace_bytes(C.byref(cfg), 2)
    assert nb > 256 * 1024 * 1024   # materialised concatenation at 256^2 x 384
    for bad in (dict(ntheta=7), dict(nphi=30), dict(dim=4), dict(c=0.0)):
        cfg = _cfg(**bad)
        assert lib.tt_workspace_bytes(C.byref(cfg), 2) == 0
        assert lib.tt_last_error(None)
    cfg = _cfg()
    cfg.bc_hi[0] = 1  # periodic on one face only
    assert lib.tt_workspace_bytes(C.byref(cfg), 2) == 0
    assert b"periodic" in lib.tt_last_error(None)


def test_tape_validation(lib):
    """The reverse sweep needs frozen material: asking for a tape
    (ckpt_every > 0) with coupled material is rejected on the host; with a
    tape the workspace grows by the checkpoints (FP32 X checkpoints in the
    mixed form)."""
    from paper_2503_18056_amd import TT_FP32_MIXED, make_config
    p = wl.c5(n=32, steps=10)
    base = lib.tt_workspace_bytes(C.byref(make_config(p)), 0)
    taped = lib.tt_workspace_bytes(C.byref(make_config(p, ckpt_every=5)), 0)
    ns, r1c = 32 * 32, 128
    assert taped > base + 2 * ns * r1c * 8  # two checkpoints of X at least
    base_m = lib.tt_workspace_bytes(C.byref(make_config(p, precision=TT_FP32_MIXED)), 0)
    taped_m = lib.tt_workspace_bytes(C.byref(make_config(p, ckpt_every=5, precision=TT_FP32_MIXED)), 0)
    assert taped_m > base_m + 2 * ns * r1c * 4
    q = dict(p)
    q["material"] = wl.COUPLED
    assert lib.tt_workspace_bytes(C.byref(make_config(q, ckpt_every=5)), 0) == 0
    assert b"FROZEN" in lib.tt_last_error(None)


def test_create_rejects_bad_input_on_host(lib):
    from paper_2503_18056_amd import _ffi
    cfg = _cfg(ntheta=5)
    ctx = C.c_void_p()
    st = lib.tt_create(C.byref(cfg), None, None, None, None, None, 0, None, None, None, 1, 1,
                       None, 0, None, C.byref(ctx))
    assert st == _ffi.TT_ERR_INVALID_ARG
    assert not ctx.value
    # a workspace that is too small is reported before any device call
    import numpy as np
    p = wl.small_random()
    cfg = __import__("paper_2503_18056_amd").make_config(p)
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64)  # noqa: E731
    X0, Th0, Ph0 = a(p["X0"]), a(p["Th0"]), a(p["Ph0"])
    k = a(p["kappa"])
    pd = lambda x: x.ctypes.data_as(_ffi.PD)  # noqa: E731
    st = lib.tt_create(C.byref(cfg), pd(k), pd(k), pd(k), pd(k), None, 0, pd(X0), pd(Th0), pd(Ph0),
                       X0.shape[1], Ph0.shape[0], C.c_void_p(16), 8, None, C.byref(ctx))
    assert st == _ffi.TT_ERR_OOM
    assert b"workspace" in lib.tt_last_error(None)
    st = lib.tt_create(C.byref(cfg), pd(k), pd(k), pd(k), pd(k), None, 0, pd(X0), pd(Th0), pd(Ph0),
                       10**6, 1, C.c_void_p(16), 1 << 40, None, C.byref(ctx))
    assert st == _ffi.TT_ERR_INVALID_ARG


def test_lds_budget_of_the_eigensolvers(lib):
    """Every dynamic-LDS launch of the eigensolver (order up to 1024) and of
    the SVD (Golub-Kahan order up to 2048, longer side up to 1024) fits the
    160 KiB of one CU; an order the kernels were not sized for is refused on
    the host, naming the kernel, instead of being launched."""
    nb = C.c_size_t()
    for n, n2, pc in [(1024, 2048, 1024), (897, 1794, 897), (323, 646, 323), (64, 128, 64)]:
        assert lib.tt_kernel_lds_check(n, n2, pc, C.byref(nb)) == 0, lib.tt_kernel_last_error()
        assert 0 < nb.value <= 160 * 1024
    assert lib.tt_kernel_lds_check(2048, 0, 0, C.byref(nb)) != 0
    assert nb.value > 160 * 1024
    assert b"k_sytrd_grid" in lib.tt_kernel_last_error()


def _create(lib, p, **over):
    """tt_create with a fake 8-byte workspace: host-side rejections come
    first; a valid input then fails only on the workspace size (TT_ERR_OOM),
    so no device work is issued."""
    import numpy as np
    from paper_2503_18056_amd import _ffi, make_config
    cfg = make_config(p)
    a = lambda x: np.ascontiguousarray(x, dtype=np.float64)  # noqa: E731
    arrs = {k: a(over.get(k, p[k])) for k in ("kappa", "rho", "cv", "T0", "X0", "Th0", "Ph0")}
    pd = lambda x: x.ctypes.data_as(_ffi.PD)  # noqa: E731
    inflow = over.get("inflow", p["inflow"])
    arr = (_ffi.tt_inflow * max(1, len(inflow)))()
    keep = []
    for k, (face, fw, tw, pw) in enumerate(inflow):
        fw, tw, pw = a(fw), a(tw), a(pw)
        keep += [fw, tw, pw]
        arr[k].face, arr[k].face_w, arr[k].theta_w, arr[k].phi_w = face, pd(fw), pd(tw), pd(pw)
    ctx = C.c_void_p()
    st = lib.tt_create(C.byref(cfg), pd(arrs["kappa"]), pd(arrs["rho"]), pd(arrs["cv"]), pd(arrs["T0"]),
                       arr, len(inflow), pd(arrs["X0"]), pd(arrs["Th0"]), pd(arrs["Ph0"]),
                       arrs["X0"].shape[1], arrs["Ph0"].shape[0], C.c_void_p(16), 8, None, C.byref(ctx))
    return st, lib.tt_last_error(None)


def test_create_validates_host_inputs(lib):
    import numpy as np
    from paper_2503_18056_amd import _ffi
    p = wl.small_random(bc="inflow", seed=2)
    st, msg = _create(lib, p)
    assert st == _ffi.TT_ERR_OOM, msg
    for key, bad, word in [("kappa", np.nan, b"kappa"), ("kappa", -1.0, b"kappa"),
                           ("rho", 0.0, b"rho"), ("cv", np.inf, b"cv"), ("T0", -0.5, b"T0"),
                           ("X0", np.nan, b"cores"), ("Th0", np.inf, b"cores"), ("Ph0", np.nan, b"cores")]:
        v = np.array(p[key], dtype=float, copy=True)
        v.reshape(-1)[v.size // 2] = bad
        st, msg = _create(lib, p, **{key: v})
        assert st == _ffi.TT_ERR_INVALID_ARG and word in msg, (key, bad, msg)
    inflow = [list(t) for t in p["inflow"]]
    inflow[1][2] = np.array(inflow[1][2], copy=True)
    inflow[1][2][0] = np.nan
    st, msg = _create(lib, p, inflow=[tuple(t) for t in inflow])
    assert st == _ffi.TT_ERR_INVALID_ARG and b"inflow" in msg


def test_operator_options_validation(lib):
    """Rusanov changes the block count (B = 1 + 2 dim, or 1 + dim when
    S+ = 0) and doubles the rank-1 inflow terms when S+ > 0, HLL doubles
    them and adds its face weights (beta and the threshold finite and
    positive); outflow faces, the two-rounding schedule, Rusanov and HLL
    are accepted, but not with a tape (the reverse sweep covers the upwind,
    one-rounding step without outflow faces)."""
    from paper_2503_18056_amd import TT_FLUX_RUSANOV, TT_ROUND_TWICE, make_config
    p = wl.small_random(bc="inflow", seed=2)
    n_in = len(p["inflow"])
    base = lib.tt_workspace_bytes(C.byref(make_config(p)), n_in)
    assert base > 0
    q = dict(p, flux="rusanov", s_plus=0.7)
    assert lib.tt_workspace_bytes(C.byref(make_config(q)), n_in) > base
    q0 = dict(p, flux="rusanov", s_plus=0.0)
    assert 0 < lib.tt_workspace_bytes(C.byref(make_config(q0)), n_in) < base
    assert lib.tt_workspace_bytes(C.byref(make_config(p, schedule=TT_ROUND_TWICE)), n_in) > 0
    cfg = make_config(q)
    cfg.s_plus = -1.0
    assert lib.tt_workspace_bytes(C.byref(cfg), n_in) == 0 and b"s_plus" in lib.tt_last_error(None)
    cfg = make_config(p)
    cfg.flux = 7
    assert lib.tt_workspace_bytes(C.byref(cfg), n_in) == 0 and b"flux" in lib.tt_last_error(None)
    o = wl.small_random(bc="outflow", seed=2)
    assert lib.tt_workspace_bytes(C.byref(make_config(o)), 0) > 0
    h = dict(p, flux="hll", hll_beta=2.0)
    assert lib.tt_workspace_bytes(C.byref(make_config(h)), n_in) > base  # weights, 2 terms per entry
    for beta, thr in ((0.0, 1e-2), (-1.0, 1e-2), (1.0, 0.0), (float("nan"), 1e-2), (1.0, float("inf"))):
        cfg = make_config(h)
        cfg.hll_beta, cfg.hll_tau_threshold = beta, thr
        assert lib.tt_workspace_bytes(C.byref(cfg), n_in) == 0 and b"hll" in lib.tt_last_error(None)
    for cfg in (make_config(o, ckpt_every=2), make_config(q, ckpt_every=2),
                make_config(h, ckpt_every=2),
                make_config(p, ckpt_every=2, schedule=TT_ROUND_TWICE)):
        assert lib.tt_workspace_bytes(C.byref(cfg), n_in) == 0
        assert b"adjoint" in lib.tt_last_error(None)
