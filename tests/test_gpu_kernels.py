"""Kernel-level parity of the HIP library (include/tt_kernels.h) with plain
NumPy references on random inputs: the generic GEMM, the tall MFMA GEMM,
the tall MFMA Gram (FP64, and the sliced FP32 form), the symmetric
eigensolver and the small SVD (one-sided Jacobi for a short side up to 64
and p q <= 12288, the Golub-Kahan route above; both are covered)."""
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
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (5, 7, 3), (70, 65, 17), (130, 33, 200), (4, 9, 0),
                                   (512, 17, 3), (600, 70, 130), (5000, 130, 641), (1030, 260, 9)])
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


@pytest.mark.parametrize("K,k,n", [(16, 4, 16), (1, 1, 1), (37, 5, 3), (1000, 33, 64), (65536, 137, 27),
                                   (5003, 323, 64), (130, 200, 1), (4097, 130, 70),
                                   (20000, 897, 128), (5000, 641, 128), (3001, 400, 200), (129, 17, 65)])
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


@pytest.mark.parametrize("K,n", [(4, 16), (1, 1), (3, 5), (1000, 64), (1000, 65), (4097, 130), (65536, 322),
                                 (1000, 385), (4097, 400), (2000, 401), (20000, 641), (3001, 770),
                                 (30000, 897), (9000, 1024)])
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
@pytest.mark.parametrize("n", [1, 2, 3, 5, 31, 62, 63, 64, 65, 100, 142, 160, 161, 175, 181, 322, 400, 600,
                               641, 897, 1024])
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


def _svd_case(kind, a, b, rng):
    q = min(a, b)
    Ua = np.linalg.qr(rng.standard_normal((a, q)))[0]
    Vb = np.linalg.qr(rng.standard_normal((b, q)))[0]
    if kind == "random":
        return rng.standard_normal((a, b))
    if kind == "graded":     # the spectrum of M near a truncation cut
        s = 10.0 ** (-12 * np.arange(q) / max(1, q - 1))
    elif kind == "cluster":  # exactly repeated singular values in pairs
        s = np.repeat(np.linspace(2, 1, (q + 1) // 2), 2)[:q]
    elif kind == "lowrank":  # exact zeros beyond rank q/3
        s = np.where(np.arange(q) < max(1, q // 3), 1.0 / (1 + np.arange(q)), 0.0)
    else:
        raise ValueError(kind)
    return (Ua * s) @ Vb.T


@pytest.mark.parametrize("kind", ["random", "graded", "cluster", "lowrank"])
@pytest.mark.parametrize("a,b", [(1, 1), (1, 6), (6, 1), (7, 7), (40, 33), (33, 40), (142, 36),
                                 (36, 142), (62, 12), (1024, 12), (192, 64), (64, 192), (193, 64),
                                 (65, 64), (130, 200), (322, 150), (143, 322), (383, 383),
                                 (420, 390), (1024, 16), (16, 1024), (897, 641), (641, 897),
                                 (1000, 1024)])
def test_svd(env, kind, a, b):
    lib, torch = env
    rng = np.random.default_rng(a * 1000 + b + len(kind))
    M = _svd_case(kind, a, b, rng)
    q = min(a, b)
    dM = _dev(torch, M)
    ds = torch.zeros(q, dtype=torch.float64, device="cuda")
    dV = torch.zeros((a if a <= b else b, q), dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_svd_workspace(a, b))
    kept = C.c_int32()
    st = lib.tt_kernel_svd(_p(dM), a, b, b, _p(ds), _p(dV), q, C.byref(kept), _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    sig = ds.cpu().numpy()
    k = kept.value
    V = dV.cpu().numpy()[:, :k]
    U_, S, Vt_ = np.linalg.svd(M, full_matrices=False)
    s1 = S[0]
    serr = np.abs(sig - S).max() / s1
    # singular values: absolute error ~ q u sigma_1 (no squaring)
    assert serr < 20 * q * 2.0 ** -53, serr
    assert k >= int(np.count_nonzero(S > 1e-12 * s1))
    ref = U_ if a <= b else Vt_.T
    # vectors: direction error ~ u sigma_1 / gap for separated sigma
    worst = 0.0
    for c in range(k):
        others = np.delete(S, c)
        gap = np.min(np.abs(others - S[c])) if others.size else s1
        bound = 50 * np.sqrt(q) * 2.0 ** -53 * s1 / max(gap, 1e-300)
        if bound > 1e-4:
            continue
        r = ref[:, c] * np.sign(ref[np.argmax(np.abs(ref[:, c])), c])
        e = np.abs(V[:, c] - r).max()
        worst = max(worst, e / bound)
        assert e < bound + 1e-14, (c, e, bound)
    good = [c for c in range(k) if S[c] > 1e-6 * s1]
    orth = np.abs(V[:, good].T @ V[:, good] - np.eye(len(good))).max() if good else 0.0
    # the complementary vectors W = M^T U (or M V) have norms sigma
    W = (M.T @ V) if a <= b else (M @ V)
    nerr = np.abs(np.linalg.norm(W, axis=0) - sig[:k]).max() / s1 if k else 0.0
    _log(f"svd {kind} {a}x{b} kept={k} sig_err={serr:.2e} vec/bound={worst:.2e} "
         f"orth={orth:.2e} norm_err={nerr:.2e}")
    assert orth < 1e-10
    assert nerr < 1e-13 * np.sqrt(q)


@pytest.mark.parametrize("K,n", [(1, 1), (7, 5), (257, 64), (4099, 130), (65536, 142), (20000, 322),
                                 (1500, 450), (2000, 641), (600, 1024)])
def test_gram_f32(env, K, n):
    """Sliced FP32-MFMA Gram of an FP32 matrix against the FP64 Gram of the
    same values: error within 2^-44 (times a small count) of the column
    scales, on columns spanning 12 orders of magnitude; a plain FP32 Gram
    is ~1e-7 off by comparison."""
    lib, torch = env
    rng = np.random.default_rng(K + n)
    A = (rng.standard_normal((K, n)) * 10.0 ** rng.uniform(-12, 0, n)[None, :]).astype(np.float32)
    dA = torch.as_tensor(A, device="cuda")
    dG = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ws = _ws(torch, lib.tt_kernel_gram_f32_workspace(K, n, n))
    st = lib.tt_kernel_gram_f32(_p(dA), K, n, n, _p(dG), n, _p(ws), ws.numel(), None)
    assert st == 0, lib.tt_kernel_last_error()
    G = dG.cpu().numpy()
    A64 = A.astype(np.float64)
    AL = A.astype(np.longdouble)
    ref = (AL.T @ AL).astype(np.float64)  # 64-bit-mantissa reference
    cmax = np.abs(A64).max(axis=0)
    scale = K * np.outer(cmax, cmax) + 1e-300
    err = np.abs(G - ref) / scale
    plain = np.abs((A.T @ A).astype(np.float64) - ref) / scale
    _log(f"gram_f32 K={K} n={n} max err/(K cmax_a cmax_b)={err.max():.2e} (plain fp32 {plain.max():.2e})")
    assert np.array_equal(G, G.T)
    assert err.max() < 8 * 2.0 ** -44
