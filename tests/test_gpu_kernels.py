"""Kernel-level parity of the HIP library (include/tt_kernels.h) with plain
NumPy references on random inputs: the generic GEMM, the tall MFMA GEMM,
the tall MFMA Gram and the symmetric eigensolver."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2503_18056_amd import _ffi
    lib = _ffi.load()
    return lib, torch


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _ws(torch, nbytes):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (5, 7, 3), (70, 65, 17), (130, 33, 200), (4, 9, 0)])
def test_gemm(env, ta, tb, m, n, k):
    lib, torch = env
    rng = np.random.default_rng(m * 100 + n + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    ref = (A.T if ta else A) @ (B.T if tb else B)
    dA, dB = _dev(torch, A if A.size else np.zeros((1, 1))), _dev(torch, B if B.size else np.zeros((1, 1)))
    dC = torch.full((m, n), np.nan, dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_gemm_tall_workspace())
    st = lib.tt_kernel_gemm(_p(dA), max(1, A.shape[1]), ta, _p(dB), max(1, B.shape[1]), tb, _p(dC), n,
                            m, n, k, _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    got = dC.cpu().numpy()
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * max(1.0, np.abs(ref).max(initial=0)))


@pytest.mark.parametrize("K,k,n", [(16, 4, 16), (1, 1, 1), (37, 5, 3), (1000, 33, 64), (4097, 130, 70)])
def test_gemm_tall(env, K, k, n):
    lib, torch = env
    rng = np.random.default_rng(K + k + n)
    A = rng.standard_normal((K, k))
    B = rng.standard_normal((k, n))
    dA, dB = _dev(torch, A), _dev(torch, B)
    dC = torch.full((K, n), np.nan, dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_gemm_tall_workspace())
    st = lib.tt_kernel_gemm_tall(_p(dA), K, k, k, _p(dB), n, n, _p(dC), n, _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    got = dC.cpu().numpy()
    err = np.abs(got - A @ B).max()
    _log(f"gemm_tall K={K} k={k} n={n} err={err:.2e}")
    if err > 1e-12:
        _log("first rows got\n", got[:4, :4], "\nref\n", (A @ B)[:4, :4])
    assert err < 1e-12 * max(1.0, k)


@pytest.mark.parametrize("K,n", [(4, 16), (1, 1), (3, 5), (1000, 64), (1000, 65), (4097, 130), (65536, 322)])
def test_gram(env, K, n):
    lib, torch = env
    rng = np.random.default_rng(K + n)
    lda = n + 3
    A = rng.standard_normal((K, lda))
    dA = _dev(torch, A)
    dG = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_gram_workspace(K, n, lda))
    st = lib.tt_kernel_gram(_p(dA), K, n, lda, _p(dG), n, _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    G = dG.cpu().numpy()
    ref = A[:, :n].T @ A[:, :n]
    err = np.abs(G - ref).max() / np.abs(ref).max()
    _log(f"gram K={K} n={n} err={err:.2e}")
    if err > 1e-12:
        _log("got\n", G[:4, :4], "\nref\n", ref[:4, :4])
    assert err < 1e-13


def _eig_case(kind, n, rng):
    if kind == "random":
        Q = rng.standard_normal((n, n))
        return Q + Q.T
    if kind == "gram":   # PSD Gram with a graded spectrum
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        lam = 10.0 ** (-12 * np.arange(n) / max(1, n - 1))
        return (Q * lam) @ Q.T
    if kind == "cluster":   # exactly repeated eigenvalues in pairs
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        lam = np.repeat(np.linspace(1, 2, (n + 1) // 2), 2)[:n]
        return (Q * lam) @ Q.T
    if kind == "lowrank":
        B = rng.standard_normal((n, max(1, n // 3)))
        return B @ B.T
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["random", "gram", "cluster", "lowrank"])
@pytest.mark.parametrize("n", [1, 2, 5, 31, 64, 100, 322])
def test_eigh(env, kind, n):
    lib, torch = env
    rng = np.random.default_rng(n + len(kind))
    A = _eig_case(kind, n, rng)
    A = 0.5 * (A + A.T)
    dA = _dev(torch, A)
    dl = torch.zeros(n, dtype=torch.float64, device="cuda")
    dV = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_eigh_workspace(n))
    kept = C.c_int32()
    clip = 0.0 if kind == "random" else 1.0
    st = lib.tt_kernel_eigh(_p(dA), n, n, clip, _p(dl), _p(dV), n, C.byref(kept), _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    lam = dl.cpu().numpy()
    V = dV.cpu().numpy()[:, :kept.value]
    ref = np.linalg.eigvalsh(A)[::-1]
    nrm = np.abs(ref).max()
    lerr = np.abs(lam - ref).max() / nrm
    k = kept.value
    res = np.abs(A @ V - V * lam[:k]).max() / nrm if k else 0.0
    orth = np.abs(V.T @ V - np.eye(k)).max() if k else 0.0
    _log(f"eigh {kind} n={n} kept={k} lam_err={lerr:.2e} resid={res:.2e} orth={orth:.2e}")
    assert lerr < 1e-13 * max(1, n) ** 0.5
    assert res < 1e-12
    assert orth < 1e-11
