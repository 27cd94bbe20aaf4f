"""tt_kernel_gram_noalloc (scratch in the library's static device array)
against tt_kernel_gram (scratch in a caller workspace), through the C ABI.

Both run the same Gram kernels with the same plan and fixed-order
reductions, so the results must agree to the last bit.  Two calls in a row,
the second with a smaller input, check that the shared scratch left by the
first call does not leak into the second; a size whose partial tiles exceed
the scratch is refused on the host.
"""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gram_ws(lib, torch, A, K, n, lda):
    nb = lib.tt_kernel_gram_workspace(K, n, lda)
    ws = torch.empty(int(nb), dtype=torch.uint8, device="cuda:0")
    G = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda:0")
    st = lib.tt_kernel_gram(C.c_void_p(A.data_ptr()), K, n, lda, C.c_void_p(G.data_ptr()), n,
                            C.c_void_p(ws.data_ptr()), int(nb), None)
    assert st == 0, lib.tt_kernel_last_error()
    return G


def _gram_noalloc(lib, torch, A, K, n, lda):
    G = torch.full((n, n), np.nan, dtype=torch.float64, device="cuda:0")
    st = lib.tt_kernel_gram_noalloc(C.c_void_p(A.data_ptr()), K, n, lda, C.c_void_p(G.data_ptr()), n, None)
    assert st == 0, lib.tt_kernel_last_error()
    return G


def test_gram_noalloc_matches_workspace_gram():
    import torch
    from paper_2503_18056_amd import _ffi
    lib = _ffi.load()
    g = torch.Generator(device="cpu").manual_seed(7)
    for (K, n, lda) in [(65536, 135, 136), (3001, 41, 48)]:
        print(f"noalloc gram K={K} n={n} lda={lda}", file=sys.stderr, flush=True)
        A = torch.randn((K, lda), generator=g, dtype=torch.float64).to("cuda:0")
        ref = _gram_ws(lib, torch, A, K, n, lda)
        got = _gram_noalloc(lib, torch, A, K, n, lda)
        torch.cuda.synchronize()
        r, q = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(q))
        assert np.array_equal(r, q), np.max(np.abs(r - q))
        Ah = A.cpu().numpy()[:, :n]
        exact = Ah.T @ Ah
        assert np.max(np.abs(q - exact)) < 1e-12 * np.max(np.abs(exact))
    # a size whose partial tiles do not fit the scratch: refused on the host
    Abig = torch.zeros((4096 * 64, 384), dtype=torch.float64, device="cuda:0")
    G = torch.empty((384, 384), dtype=torch.float64, device="cuda:0")
    st = lib.tt_kernel_gram_noalloc(C.c_void_p(Abig.data_ptr()), 4096 * 64, 384, 384,
                                    C.c_void_p(G.data_ptr()), 384, None)
    assert st == _ffi.TT_ERR_INVALID_ARG
    assert b"scratch" in lib.tt_kernel_last_error()
