"""Randomized Tucker compression: RandTucker (Alg. 2) and RandTucker2i (Alg. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Section IV-A):
  * the randomized range finder the paper takes from Halko et al.
    (draw Gaussian Omega, Z = Y_(n) Omega, orthonormal basis of Z by QR);
  * Alg. 3 sketch: X = Y x_{p != n} U_p^T, Z_n = X_(n) Omega~_n with Omega~_n of
    size (prod_{k != n} R~_k) x R~_n, U_n = orth(Z_n); the loop body runs twice
    in the paper (``sweeps``); the core is G = Y x_1 U_1^T ... x_N U_N^T;
  * Alg. 2 (sequential, dense Omega, Y shrunk mode by mode) as
    ``rand_tucker_sequential``.

Readings of the paper (each one listed in the design doc):
  * Alg. 3 prints X = Y x_{p != n} U^(p) without the transpose; the sizes
    only work with U^(p)T.
  * Jacobi order: by default every mode of a sweep uses the bases of the
    previous sweep (the first sweep uses the Gaussian Omega_p, i.e. the
    paper's random initialization of U^(p)).  ``order="gauss_seidel"`` is the
    paper-literal loop where later modes see bases already replaced.
  * QR is Householder (LAPACK geqrf/orgqr via numpy.linalg.qr); columns are
    sign-flipped so that diag(R) >= 0 (the paper is silent on signs).
  * R~_n -> R_n: the algorithms return R~-sized factors; when output ranks
    R_n < R~_n are requested the core is truncated through its own mode-n
    Gram matrices (top-R_n eigenvectors W_n of G~_(n) G~_(n)^T, in
    descending eigenvalue order, ties by ascending index, each column
    sign-fixed so its largest-magnitude entry is positive with the lowest
    index winning ties); U_n = Q_n W_n and G = G~ x_n W_n^T.

Pins: tests/test_oracle_randtucker.py (exact recovery of noise-free tensors of
known multilinear rank, orthonormality, the Tucker/Pythagoras identity, the
R~_n = I_n special case equal to the truncated HOSVD from numpy's SVD).
"""

import numpy as np

from .tensor import unfold, multi_ttm_t, ttm_t


def orth_qr(Z):
    """Orthonormal basis of range(Z) by Householder QR with diag(R) >= 0."""
    Z = np.asarray(Z, dtype=np.float64)
    Q, R = np.linalg.qr(Z, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def orth_gram_evd(Z):
    """Alternative basis of eq. (23): eig of Z^T Z = W S W^T, U = Z W S^{-1/2}.
    Only valid for full-column-rank Z; kept for the distributed design."""
    Z = np.asarray(Z, dtype=np.float64)
    s, W = np.linalg.eigh(Z.T @ Z)
    order = np.argsort(-s, kind="stable")
    s, W = s[order], W[:, order]
    return (Z @ W) / np.sqrt(s)


def sketch(Y, bases, omega_t, n):
    """One Alg. 3 sketch: X = Y x_{p != n} B_p^T; Z_n = X_(n) Omega~_n."""
    X = multi_ttm_t(Y, bases, skip=n)
    return unfold(X, n) @ np.asarray(omega_t, dtype=np.float64)


def sorted_sign_fixed_eigvecs(S, k):
    """Top-k eigenvectors of symmetric S, descending eigenvalues (ties by
    ascending index), each column's largest-|.| entry made positive (lowest
    index wins ties)."""
    w, V = np.linalg.eigh(np.asarray(S, dtype=np.float64))
    order = sorted(range(len(w)), key=lambda i: (-w[i], i))[:k]
    V = V[:, order].copy()
    for c in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, c])))
        if V[j, c] < 0:
            V[:, c] = -V[:, c]
    return w[order], V


def truncate_core(Q, Gt, ranks):
    """R~_n -> R_n through the core's mode-n Gram eigenvectors."""
    W = []
    for n, r in enumerate(ranks):
        Gn = unfold(Gt, n)
        _, Wn = sorted_sign_fixed_eigvecs(Gn @ Gn.T, r)
        W.append(Wn)
    U = [Qn @ Wn for Qn, Wn in zip(Q, W)]
    G = multi_ttm_t(Gt, W)
    return U, G, W


def rand_tucker(Y, omegas, omega_tildes, sweeps=1, ranks=None,
                order="jacobi"):
    """RandTucker2i (Alg. 3) with ``sweeps`` passes of the sketch loop.

    Y            : N-way array (promoted to FP64).
    omegas       : list of N Gaussian matrices Omega_p, I_p x R~_p (the
                   random initial U^(p) that Alg. 3 starts from).
    omega_tildes : list (length >= sweeps) of lists of N matrices
                   Omega~_n, (prod_{p != n} R~_p) x R~_n, rows in the
                   row-major order of (j_p)_{p != n}.
    ranks        : output ranks R_n (<= R~_n) or None for no truncation.
    Returns a dict with U, G, the untruncated Q and G~, and every sweep's Z.
    """
    Y = np.asarray(Y, dtype=np.float64)
    N = Y.ndim
    bases = [np.asarray(o, dtype=np.float64) for o in omegas]
    Zs, Qs = [], []
    for s in range(sweeps):
        if order == "jacobi":
            Z = [sketch(Y, bases, omega_tildes[s][n], n) for n in range(N)]
            bases = [orth_qr(z) for z in Z]
        elif order == "gauss_seidel":
            Z = []
            for n in range(N):
                z = sketch(Y, bases, omega_tildes[s][n], n)
                Z.append(z)
                bases[n] = orth_qr(z)
        else:
            raise ValueError(order)
        Zs.append(Z)
        Qs.append(list(bases))
    Q = bases
    Gt = multi_ttm_t(Y, Q)                       # Alg. 3, core line
    out = {"Q": Q, "Gt": Gt, "Z": Zs, "Q_sweeps": Qs}
    if ranks is None:
        out["U"], out["G"], out["W"] = Q, Gt, None
    else:
        out["U"], out["G"], out["W"] = truncate_core(Q, Gt, ranks)
    return out


def rand_tucker_sequential(Y, dense_omegas):
    """RandTucker (Alg. 2): for n = 1..N, Z = Y_(n) Omega_n with a dense
    Gaussian Omega_n whose row count is the product of the *current* other
    dimensions (earlier modes already shrunk to R~_k); U_n = orth(Z);
    Y <- Y x_n U_n^T.  Returns (U, G)."""
    Y = np.asarray(Y, dtype=np.float64)
    U = []
    for n, Om in enumerate(dense_omegas):
        Z = unfold(Y, n) @ np.asarray(Om, dtype=np.float64)
        Un = orth_qr(Z)
        U.append(Un)
        Y = ttm_t(Y, Un, n)
    return U, Y


def hosvd(Y, ranks):
    """Truncated HOSVD (Section II): U_n = leading left singular vectors of
    Y_(n) (numpy SVD), G = Y x_n U_n^T.  A baseline, not part of the method."""
    Y = np.asarray(Y, dtype=np.float64)
    U = []
    for n, r in enumerate(ranks):
        u, _, _ = np.linalg.svd(unfold(Y, n), full_matrices=False)
        U.append(u[:, :r])
    return U, multi_ttm_t(Y, U)


def tucker_fit(Y, U, G):
    """1 - ||Y - [[G;U]]|| / ||Y|| from the dense residual."""
    from .tensor import tucker_full
    Y = np.asarray(Y, dtype=np.float64)
    return 1.0 - np.linalg.norm(Y - tucker_full(G, U)) / np.linalg.norm(Y)
