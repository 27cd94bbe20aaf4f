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
