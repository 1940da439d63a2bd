"""Tensor algebra used by the paper (Section II, Table I notation).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pinned by tests/test_oracle_tensor.py against brute-force index loops on tiny
tensors and against closed forms (a CP tensor's unfolding factors exactly as
eq. (3)-(4) state; the Gram identity eq. (9)).
"""

import numpy as np


def unfold(Y, n):
    """Mode-n matricization Y_(n) (Table I): I_n rows; columns are the
    remaining indices in increasing mode order, last one fastest."""
    Y = np.asarray(Y)
    return np.moveaxis(Y, n, 0).reshape(Y.shape[n], -1)


def fold(M, n, shape):
    """Inverse of ``unfold`` for a tensor of the given shape."""
    shape = list(shape)
    rest = shape[:n] + shape[n + 1:]
    return np.moveaxis(np.asarray(M).reshape([shape[n]] + rest), 0, n)


def ttm_t(Y, M, n):
    """Y x_n M^T for M of shape I_n x K (the paper's Y x_n U^T, eq. (1) and
    Alg. 2-3): out[.., k, ..] = sum_{i_n} Y[.., i_n, ..] M[i_n, k]."""
    out = np.tensordot(Y, M, axes=([n], [0]))      # contracted mode moves last
    return np.moveaxis(out, -1, n)


def ttm(Y, M, n):
    """Y x_n M for M of shape K x I_n (Kolda-Bader mode-n product)."""
    return ttm_t(Y, np.asarray(M).T, n)


def multi_ttm_t(Y, mats, skip=None):
    """Y x_{p != skip} M_p^T, applied in increasing p."""
    out = Y
    for p, M in enumerate(mats):
        if p == skip or M is None:
            continue
        out = ttm_t(out, M, p)
    return out


def khatri_rao(mats):
    """Column-wise Kronecker product (Table I) of matrices listed in
    increasing mode order; row index is the row-major flattening of the
    factors' row indices (first matrix slowest), matching ``unfold``."""
    mats = [np.asarray(m) for m in mats]
    R = mats[0].shape[1]
    for m in mats:
        if m.shape[1] != R:
            raise ValueError("Khatri-Rao factors need equal column counts")
    out = np.empty((int(np.prod([m.shape[0] for m in mats])), R),
                   dtype=np.result_type(*mats))
    for r in range(R):
        col = np.ones(1, dtype=out.dtype)
        for m in mats:
            col = np.kron(col, m[:, r])
        out[:, r] = col
    return out


def kruskal_full(A, lam=None):
    """Dense tensor of the CP model eq. (2): sum_r lam_r a_r^(1) o ... o a_r^(N)."""
    A = [np.asarray(a, dtype=np.float64) for a in A]
    R = A[0].shape[1]
    w = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    shape = [a.shape[0] for a in A]
    # Y_(1) = A_1 diag(w) (KR of the rest)^T, eq. (3)-(4)
    Y1 = (A[0] * w) @ khatri_rao(A[1:]).T
    return fold(Y1, 0, shape)


def tucker_full(G, U):
    """Dense tensor of the Tucker model eq. (1): G x_1 U_1 ... x_N U_N."""
    out = np.asarray(G, dtype=np.float64)
    for p, Up in enumerate(U):
        out = ttm(out, Up, p)
    return out


def hadamard_grams(A, skip):
    """eq. (9): B^T B = hadamard product over p != skip of A_p^T A_p."""
    R = A[0].shape[1]
    T = np.ones((R, R))
    for p, a in enumerate(A):
        if p != skip:
            T = T * (a.T @ a)
    return T
