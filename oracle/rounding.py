"""TT rounding: Gram-SVD (App. A.2), TT-SVD (App. A.1), dense SVD.

Three-core TT  I_{ilp} = X_i Theta_l Phi_p  (Sec. 4.1, eq. tensor_decomp),
X: (N_s, r1), Theta: (r1, N_theta, r2), Phi: (r2, N_phi).

Rules where the paper is silent (applied identically by every form here):

* tolerance (App. A, note on rank truncation: error balanced across the
  d - 1 = 2 bonds so the overall relative error is guaranteed): per-bond
  delta^2 = eps^2 ||T||^2 / 2, with ||T||^2 := sum of the squared singular
  values found at bond 1;
* rank rule: r' = min{k >= 1 : sum_{j>k} sigma_j^2 <= delta^2}, then the
  cluster rule, then the cap (``select_rank``).  Two neighbouring singular
  values form a cluster when they differ by no more than what the Gram
  route can resolve: max(eta sigma_1, R u sigma_1^2 / sigma_r) (App. A.4:
  Gram singular values carry only sqrt(u) relative precision; an error
  ||dG|| ~ R u sigma_1^2 moves sigma_r by ~R u sigma_1^2 / sigma_r);
* clip rule for singular Gram matrices: eigenpairs with lambda <= tau
  lambda_max (tau = R u, R the Gram dimension, u = 2^-53) or lambda <= 0
  are dropped before Sigma^-1 is formed; then the kept count of each side
  is cut to the rank that side can have, its number of rows (a Gram of R
  columns built from m < R rows has rank <= m, and eigenpairs past m are
  rounding noise of size ~u lambda_max, App. A.4);
* eigen/singular vectors in descending order, each column signed so that
  its largest-magnitude entry is positive (first such entry on ties);
* a zero tensor rounds to rank 1 with zero cores.
"""
import numpy as np

U = 2.0 ** -53
ETA_FP64 = 1e-12


def gauge(V):
    """Sign-fix the columns of V; returns (V_fixed, signs)."""
    if V.size == 0:
        return V, np.ones(V.shape[1])
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return V * sgn[None, :], sgn


def select_rank(sig, delta2, rmax, eta=ETA_FP64, noise=0.0):
    """Rank rule with the cluster rule and the cap.

    tail(k) = sum_{j>k} sigma_j^2; r = min{k >= 1: tail(k) <= delta^2}.
    Cluster rule: while sigma_r - sigma_{r+1} <= thr(r), r += 1, with
    thr(r) = max(eta sigma_1, noise sigma_1^2 / sigma_r), so a cut never
    splits a set of singular values that are equal to the resolution of the
    computation (``noise`` = R u for a Gram of dimension R, 0 for a direct
    SVD).  The extension stops before a singular value that the computation
    does not resolve (sigma_{r+1} <= sqrt(noise) sigma_1, where thr exceeds
    sigma itself): below that level every gap is within the noise, and
    following the ties would keep rounding noise.  Cap: if r > rmax > 0,
    r = rmax and, if that cut splits a cluster, r moves down to just before
    the cluster (kept at rmax if the cluster starts at 1).
    """
    sig = np.asarray(sig, float)
    n = sig.size
    if n == 0 or sig[0] <= 0.0:
        return 1
    sq = sig * sig
    tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])  # tail[k] = sum_{j>=k}
    r = next(k for k in range(1, n + 1) if tail[k] <= delta2)

    def tied(j):  # sigma_j and sigma_{j+1} (1-based j) in one cluster
        thr = max(eta * sig[0], noise * sig[0] ** 2 / sig[j - 1] if sig[j - 1] > 0 else np.inf)
        return sig[j - 1] - sig[j] <= thr

    floor = np.sqrt(noise) * sig[0]

    def resolved(j):  # sigma_{j+1} (1-based) above the resolution of the computation
        return noise == 0.0 or sig[j] > floor
    while r < n and tied(r) and resolved(r):
        r += 1
    if rmax > 0 and r > rmax:
        r = rmax
        if r < n and tied(r):
            k = r
            while k > 1 and tied(k - 1):
                k -= 1
            r = k - 1 if k > 1 else rmax
    return r


def rank_margin(sig, delta2, rmax, eta=ETA_FP64, noise=0.0):
    """Smallest relative distance to its threshold among the comparisons that
    ``select_rank`` makes for these singular values: tail(k) against delta^2
    at the first k that passes and the one before it, every tie test
    sigma_j - sigma_{j+1} against its threshold, and every resolution test
    sigma_{j+1} against sqrt(noise) sigma_1.  A small margin means a
    rounding-sized change of sigma can flip the decision (diagnostic only;
    the rank rule itself is ``select_rank``)."""
    sig = np.asarray(sig, float)
    n = sig.size
    if n == 0 or sig[0] <= 0.0 or delta2 <= 0.0:
        return np.inf
    sq = sig * sig
    tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])
    r = next(k for k in range(1, n + 1) if tail[k] <= delta2)
    margins = [abs(tail[r] / delta2 - 1.0)]
    if r > 1:
        margins.append(abs(tail[r - 1] / delta2 - 1.0))

    def thr(j):
        return max(eta * sig[0], noise * sig[0] ** 2 / sig[j - 1] if sig[j - 1] > 0 else np.inf)

    def test(j):
        t = thr(j)
        margins.append(abs((sig[j - 1] - sig[j]) / t - 1.0) if np.isfinite(t) and t > 0 else np.inf)
        return sig[j - 1] - sig[j] <= t

    floor = np.sqrt(noise) * sig[0]

    def resolved(j):
        if noise == 0.0:
            return True
        margins.append(abs(sig[j] / floor - 1.0))
        return sig[j] > floor
    while r < n and test(r) and resolved(r):
        r += 1
    if rmax > 0 and r > rmax:
        r = rmax
        if r < n and test(r):
            k = r
            while k > 1 and test(k - 1):
                k -= 1
    return float(min(margins))


def eig_desc_clipped(G, rows=None):
    """Symmetric eigendecomposition, descending, gauge-fixed, clip rule.

    ``rows``: the number of rows of the factor whose Gram G is; the kept
    count is cut to it (rank bound of G)."""
    R = G.shape[0]
    lam, V = np.linalg.eigh(G)
    lam, V = lam[::-1], V[:, ::-1]
    V, _ = gauge(V)
    if R == 0:
        return lam, V
    tau = R * U
    keep = (lam > tau * lam[0]) & (lam > 0.0)
    k = int(np.count_nonzero(keep))
    if rows is not None:
        k = min(k, int(rows))
    return lam[:k].copy(), V[:, :k].copy()


def gram_truncate(A, GB, *, tol, rmax, delta2=None, eta=ETA_FP64, rank=None, perturb=None,
                  b_rows=None):
    """Gram-SVD truncate of A B^T given A and the Gram of B (App. A.2).

    G_A = A^T A = V_A Sigma_A^2 V_A^T, G_B = V_B Sigma_B^2 V_B^T,
    M = Sigma_A V_A^T V_B Sigma_B = U~ Sigma~ V~^T (truncated to r'),
    A' = A V_A Sigma_A^-1 U~,  M_upd = (V_B Sigma_B^-1 V~ Sigma~)^T.
    Returns (A', M_upd, P, info) with A' = A P.
    ``perturb`` (tests only): applied to G_A and G_B before their
    eigendecompositions, to measure the method's own sensitivity to a
    rounding-sized change of its Gram matrices.  ``b_rows``: the number of
    columns of B^T (the rank bound of G_B); A's bound is its row count.
    """
    R = A.shape[1]
    GA = A.T @ A
    if perturb is not None:
        GA, GB = perturb(GA), perturb(GB)
    lamA, VA = eig_desc_clipped(GA, rows=A.shape[0])
    lamB, VB = eig_desc_clipped(GB, rows=b_rows)
    info = dict(R=R, kA=lamA.size, kB=lamB.size)
    if lamA.size == 0 or lamB.size == 0:
        sig = np.zeros(0)
    else:
        SA, SB = np.sqrt(lamA), np.sqrt(lamB)
        M = (SA[:, None] * (VA.T @ VB)) * SB[None, :]
        Ut, sig, Vt = np.linalg.svd(M, full_matrices=False)
        Ut, sg = gauge(Ut)
        Vt = Vt * sg[:, None]
    norm2 = float(np.sum(sig * sig))
    if delta2 is None:
        delta2 = tol * tol * norm2 / 2.0
    info.update(norm2=norm2, delta2=delta2, sigma=sig.copy())
    if sig.size == 0 or sig[0] <= 0.0:
        info.update(rank=1, zero=True)
        return np.zeros((A.shape[0], 1)), np.zeros((1, R)), np.zeros((R, 1)), info
    r = (select_rank(sig, delta2, rmax, eta, noise=R * U) if rank is None
         else min(int(rank), sig.size))
    P = VA @ (Ut[:, :r] / SA[:, None])
    Mupd = (sig[:r, None] * Vt[:r]) @ (VB / SB[None, :]).T
    sq = sig * sig
    tail = lambda k: float(np.sum(sq[k:]))  # noqa: E731
    if rank is None:
        info.update(margin=rank_margin(sig, delta2, rmax, eta, noise=R * U))
    info.update(rank=r, zero=False,
                tail_over_delta2=tail(r) / delta2 if delta2 > 0 else np.inf,
                tail_prev_over_delta2=tail(r - 1) / delta2 if delta2 > 0 else np.inf,
                gap=float(sig[r - 1] - (sig[r] if r < sig.size else 0.0)))
    return A @ P, Mupd, P, info


def round_gram(X, Th, Ph, tol, rmax, ranks=None, eta=ETA_FP64, perturb=None):
    """Gram-SVD TT rounding of a 3-core TT (App. A, Algorithm 1, d = 3).

    Backward sweep: B_2^T = Phi, B_1^T = reshape(Theta x Phi, (r1, -1)); the
    Gram matrices of B_1 and B_2 are formed here (App. A.2 footnote).
    Forward sweep, k = 1, 2: A_k = reshape(G_k, (r'_{k-1} N_k, r_k));
    [A_k', M_upd] = truncate(A_k, B_k); G_k <- A_k'; G_{k+1} <- M_upd G_{k+1}.
    ``ranks`` = (r1', r2') replays given ranks instead of the rank rule;
    ``perturb``: see ``gram_truncate``.
    """
    r1, nt, r2 = Th.shape
    npf = Ph.shape[1]
    B2T = Ph
    B1T = (Th.reshape(r1 * nt, r2) @ B2T).reshape(r1, nt * npf)
    GB2 = B2T @ B2T.T
    GB1 = B1T @ B1T.T
    rk = (None, None) if ranks is None else ranks
    Xn, M1, _, info1 = gram_truncate(X, GB1, tol=tol, rmax=rmax, eta=eta, rank=rk[0],
                                     perturb=perturb, b_rows=nt * npf)
    r1n = Xn.shape[1]
    G2 = (M1 @ Th.reshape(r1, nt * r2)).reshape(r1n, nt, r2)
    A2 = G2.reshape(r1n * nt, r2)
    A2n, M2, _, info2 = gram_truncate(A2, GB2, tol=tol, rmax=rmax, eta=eta,
                                      delta2=info1["delta2"], rank=rk[1], perturb=perturb,
                                      b_rows=npf)
    r2n = A2n.shape[1]
    return (Xn, A2n.reshape(r1n, nt, r2n), M2 @ Ph), (info1, info2)


def round_dense(T, tol, rmax, eta=ETA_FP64):
    """Rounding by SVDs of the unfoldings of the full tensor (tiny tensors).

    Same tolerance split and rank rule; in exact arithmetic this equals the
    Gram-SVD result because both truncate the SVD of the same unfoldings
    (App. A, and orthonormality of the left factor, end of A.3).
    """
    ns, nt, npf = T.shape
    Uu, S, Vt = np.linalg.svd(T.reshape(ns, nt * npf), full_matrices=False)
    norm2 = float(np.sum(S * S))
    delta2 = tol * tol * norm2 / 2.0
    if S[0] <= 0:
        return np.zeros((ns, 1)), np.zeros((1, nt, 1)), np.zeros((1, npf))
    r1 = select_rank(S, delta2, rmax, eta)
    Uu, sg = gauge(Uu[:, :r1])
    W = (S[:r1, None] * Vt[:r1]) * sg[:, None]
    U2, S2, V2 = np.linalg.svd(W.reshape(r1 * nt, npf), full_matrices=False)
    r2 = select_rank(S2, delta2, rmax, eta)
    U2, sg2 = gauge(U2[:, :r2])
    Ph = (S2[:r2, None] * V2[:r2]) * sg2[:, None]
    return Uu, U2.reshape(r1, nt, r2), Ph


def round_ttsvd(X, Th, Ph, tol, rmax, eta=ETA_FP64):
    """TT-SVD rounding (App. A.1): right-to-left QR orthogonalisation, then
    left-to-right truncated SVDs of the (now orthogonal-factor) unfoldings."""
    r1, nt, r2 = Th.shape
    npf = Ph.shape[1]
    # right-orthogonalise Phi: Phi^T = Q R  ->  Phi = R^T Q^T
    Q3, R3 = np.linalg.qr(Ph.T)
    Ph_o = Q3.T
    Th2 = Th.reshape(r1 * nt, r2) @ R3.T
    k2 = Ph_o.shape[0]
    Q2, R2 = np.linalg.qr(Th2.reshape(r1, nt * k2).T)
    Th_o = Q2.T.reshape(-1, nt, k2)
    X1 = X @ R2.T
    # left-to-right truncation
    Uu, S, Vt = np.linalg.svd(X1, full_matrices=False)
    norm2 = float(np.sum(S * S))
    delta2 = tol * tol * norm2 / 2.0
    if S[0] <= 0:
        return np.zeros((X.shape[0], 1)), np.zeros((1, nt, 1)), np.zeros((1, npf))
    a = select_rank(S, delta2, rmax, eta)
    Uu, sg = gauge(Uu[:, :a])
    C = (S[:a, None] * Vt[:a]) * sg[:, None]
    Th_n = (C @ Th_o.reshape(Th_o.shape[0], nt * k2)).reshape(a * nt, k2)
    U2, S2, V2 = np.linalg.svd(Th_n, full_matrices=False)
    b = select_rank(S2, delta2, rmax, eta)
    U2, sg2 = gauge(U2[:, :b])
    C2 = (S2[:b, None] * V2[:b]) * sg2[:, None]
    return Uu, U2.reshape(a, nt, b), C2 @ Ph_o


def round_randomized(X, Th, Ph, omegas):
    """Randomized TT rounding to fixed target ranks (App. A.3, eqs.
    randfinal and randprojection), over the two bonds from left to right.

    Bond k holds the TT as A_k B_k^T: A_1 = X, B_1^T = (Theta x Phi) unfolded
    to r1 x (N_theta N_phi); A_2 = the updated middle core unfolded to
    (r1' N_theta) x r2, B_2^T = Phi.  ``omegas`` = (Omega_1, Omega_2) are the
    Gaussian test matrices, (N_theta N_phi) x r1' and N_phi x r2', drawn by
    the caller; their column counts are the target ranks.  W = B_k^T Omega_k
    (r_k x r'_k) is the sketch formed from the small factor, and Q, with
    Q R = A_k W, an orthonormal basis of the sketched range A_k B_k^T Omega_k
    (reading: the text names the QR "of W", which for Q to have A_k's rows
    can only mean of A_k W).  Then A_k' = Q and M_upd = Q^T A_k, carried
    into the next core (B_k'^T = M_upd B_k^T).  The left factors come out
    with orthonormal columns.
    """
    O1, O2 = omegas
    r1, nt, r2 = Th.shape
    npf = Ph.shape[1]
    B1T = (Th.reshape(r1 * nt, r2) @ Ph).reshape(r1, nt * npf)
    Q1, _ = np.linalg.qr(X @ (B1T @ O1))
    M1 = Q1.T @ X
    A2 = (M1 @ Th.reshape(r1, nt * r2)).reshape(-1, r2)
    Q2, _ = np.linalg.qr(A2 @ (Ph @ O2))
    M2 = Q2.T @ A2
    return Q1, Q2.reshape(Q1.shape[1], nt, Q2.shape[1]), M2 @ Ph
