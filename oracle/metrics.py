"""Compression factor, reconstruction and TT differences.

Compression (Sec. 5.1):  C = N_s N_theta N_phi / (r1 N_s + r1 r2 N_theta + r2 N_phi).
Differences of two TTs are measured on the reconstructed tensor when it is
small, otherwise through the difference TT (concatenation, Sec. 4.1) left-
orthogonalised by Householder QR, whose last core carries the Frobenius
norm with an absolute error of order u ||A||.
"""
import numpy as np


def compression(ns, nt, npf, r1, r2):
    return ns * nt * npf / (r1 * ns + r1 * r2 * nt + r2 * npf)


def reconstruct(X, Th, Ph):
    r1, nt, r2 = Th.shape
    return (X @ (Th.reshape(r1, nt * r2))).reshape(-1, nt, r2) @ Ph


def tt_norm(X, Th, Ph):
    Q, R = np.linalg.qr(X)
    r1, nt, r2 = Th.shape
    C = (R @ Th.reshape(r1, nt * r2)).reshape(-1, r2)
    Q2, R2 = np.linalg.qr(C)
    return float(np.linalg.norm(R2 @ Ph))


def tt_diff_norm(A, B):
    """||A - B||_F for TTs A, B given as (X, Th, Ph) tuples."""
    Xa, Ta, Pa = A
    Xb, Tb, Pb = B
    X = np.concatenate([Xa, Xb], axis=1)
    r1a, nt, r2a = Ta.shape
    r1b, _, r2b = Tb.shape
    Th = np.zeros((r1a + r1b, nt, r2a + r2b))
    Th[:r1a, :, :r2a] = Ta
    Th[r1a:, :, r2a:] = Tb
    Ph = np.concatenate([Pa, -Pb], axis=0)
    return tt_norm(X, Th, Ph)


def rel_diff(A, B, dense_limit=2e7):
    """||A - B||_F / ||B||_F for TTs (dense when small enough)."""
    Xa, Ta, Pa = A
    size = Xa.shape[0] * Ta.shape[1] * Pa.shape[1]
    if size <= dense_limit:
        Fa, Fb = reconstruct(*A), reconstruct(*B)
        nb = np.linalg.norm(Fb)
        return float(np.linalg.norm(Fa - Fb) / (nb if nb > 0 else 1.0))
    nb = tt_norm(*B)
    return tt_diff_norm(A, B) / (nb if nb > 0 else 1.0)
