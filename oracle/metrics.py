"""Comparison metrics for results that are unique only up to rotation,
sign, permutation or scale.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * subspaces: projector distance ||P_U - P_W||_2 for orthonormal bases of
    equal dimension, evaluated as ||(I - U U^T) W||_2 (equal to
    sqrt(1 - s_min(U^T W)^2) but accurate for tiny angles);
  * cores: e_G = ||G_a x_n (Uo_n^T Ua_n) - G_o|| / ||G_o|| (core of one side
    rotated into the other side's bases);
  * CP factors: column-normalized, matched by an optimal permutation
    (Hungarian, scipy.optimize.linear_sum_assignment) on |congruence|;
  * SIR (footnote of Section V-A; the printed formula has a garbled sign and
    a mislabeled estimate): SIR = 20 log10(||a|| / ||a - a_hat||) after both
    are made zero-mean and unit-variance, sign-aligned and matched.
"""

import numpy as np
from scipy.optimize import linear_sum_assignment

from .tensor import multi_ttm_t


def orthonormalize(U):
    q, _ = np.linalg.qr(np.asarray(U, dtype=np.float64), mode="reduced")
    return q


def projector_distance(U, W):
    U = orthonormalize(U)
    W = orthonormalize(W)
    if U.shape[1] != W.shape[1]:
        raise ValueError("bases of different dimension")
    resid = W - U @ (U.T @ W)
    return float(np.linalg.norm(resid, 2))


def aligned_core_error(G_a, U_a, G_o, U_o):
    rot = [np.asarray(uo, dtype=np.float64).T @ np.asarray(ua, dtype=np.float64)
           for uo, ua in zip(U_o, U_a)]
    G_rot = multi_ttm_t(np.asarray(G_a, dtype=np.float64),
                        [r.T for r in rot])
    return float(np.linalg.norm(G_rot - G_o) / np.linalg.norm(G_o))


def match_columns(A, B):
    """Optimal permutation of B's columns onto A's by |cosine|.
    Returns (perm, congruences) with B[:, perm[r]] matched to A[:, r]."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    An = A / np.maximum(np.linalg.norm(A, axis=0), 1e-300)
    Bn = B / np.maximum(np.linalg.norm(B, axis=0), 1e-300)
    C = np.abs(An.T @ Bn)
    rows, cols = linear_sum_assignment(-C)
    perm = np.empty(A.shape[1], dtype=int)
    perm[rows] = cols
    return perm, C[rows, cols]


def factor_congruence(A_list, B_list):
    """Joint permutation over all modes (product of |cosines|), then the
    minimum per-mode congruence."""
    R = A_list[0].shape[1]
    score = np.ones((R, R))
    for A, B in zip(A_list, B_list):
        An = A / np.maximum(np.linalg.norm(A, axis=0), 1e-300)
        Bn = B / np.maximum(np.linalg.norm(B, axis=0), 1e-300)
        score = score * np.abs(An.T @ Bn)
    rows, cols = linear_sum_assignment(-score)
    perm = np.empty(R, dtype=int)
    perm[rows] = cols
    per_mode = []
    for A, B in zip(A_list, B_list):
        An = A / np.maximum(np.linalg.norm(A, axis=0), 1e-300)
        Bn = B / np.maximum(np.linalg.norm(B, axis=0), 1e-300)
        per_mode.append(np.abs(np.sum(An * Bn[:, perm], axis=0)))
    return perm, float(np.min(per_mode))


def sir_db(a, a_hat):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(a_hat, dtype=np.float64)
    a = (a - a.mean()) / a.std()
    b = (b - b.mean()) / b.std()
    if np.dot(a, b) < 0:
        b = -b
    err = np.linalg.norm(a - b)
    if err == 0.0:
        return np.inf
    return float(20.0 * np.log10(np.linalg.norm(a) / err))


def sir_factors(A_true, A_est):
    """Per-component SIR after optimal matching; returns the array."""
    perm, _ = match_columns(A_true, A_est)
    return np.array([sir_db(A_true[:, r], A_est[:, perm[r]])
                     for r in range(A_true.shape[1])])
