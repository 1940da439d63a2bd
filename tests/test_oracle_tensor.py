"""Pins for oracle/tensor.py: brute-force index loops and closed forms."""

import itertools

import numpy as np
import pytest

from oracle import tensor as T


def _rng(s=0):
    return np.random.default_rng(1000 + s)


def brute_ttm_t(Y, M, n):
    shape = list(Y.shape)
    K = M.shape[1]
    out_shape = shape[:n] + [K] + shape[n + 1:]
    out = np.zeros(out_shape)
    for idx in itertools.product(*[range(s) for s in out_shape]):
        k = idx[n]
        acc = 0.0
        for i in range(shape[n]):
            src = list(idx)
            src[n] = i
            acc += Y[tuple(src)] * M[i, k]
        out[idx] = acc
    return out


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 2, 3)])
def test_ttm_matches_index_loops(shape):
    g = _rng(len(shape))
    Y = g.standard_normal(shape)
    for n in range(len(shape)):
        M = g.standard_normal((shape[n], 2))
        np.testing.assert_allclose(T.ttm_t(Y, M, n), brute_ttm_t(Y, M, n),
                                   rtol=1e-13, atol=1e-13)
        # ttm (K x I_n) is the transpose form
        np.testing.assert_allclose(T.ttm(Y, M.T, n), brute_ttm_t(Y, M, n),
                                   rtol=1e-13, atol=1e-13)


def test_ttm_commutes_across_modes():
    g = _rng(2)
    Y = g.standard_normal((4, 5, 6))
    A = g.standard_normal((4, 3))
    B = g.standard_normal((6, 2))
    a = T.ttm_t(T.ttm_t(Y, A, 0), B, 2)
    b = T.ttm_t(T.ttm_t(Y, B, 2), A, 0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 2, 3)])
def test_unfold_entrywise_and_fold_inverse(shape):
    g = _rng(3)
    Y = g.standard_normal(shape)
    N = len(shape)
    for n in range(N):
        U = T.unfold(Y, n)
        others = [p for p in range(N) if p != n]
        for idx in itertools.product(*[range(s) for s in shape]):
            col = 0
            for p in others:                      # last mode fastest
                col = col * shape[p] + idx[p]
            assert U[idx[n], col] == Y[idx]
        np.testing.assert_array_equal(T.fold(U, n, shape), Y)


def test_khatri_rao_entrywise():
    g = _rng(4)
    A, B, C = (g.standard_normal((s, 3)) for s in (2, 3, 4))
    K = T.khatri_rao([A, B, C])
    for i, j, k in itertools.product(range(2), range(3), range(4)):
        row = (i * 3 + j) * 4 + k
        np.testing.assert_allclose(K[row], A[i] * B[j] * C[k], rtol=1e-15)


def brute_kruskal(A):
    shape = [a.shape[0] for a in A]
    out = np.zeros(shape)
    for idx in itertools.product(*[range(s) for s in shape]):
        out[idx] = sum(np.prod([A[p][idx[p], r] for p in range(len(A))])
                       for r in range(A[0].shape[1]))
    return out


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 2, 3)])
def test_cp_unfolding_closed_form(shape):
    """eq. (3)-(4): Y_(n) = A_n (KR_{p != n} A_p)^T for every n, on a CP
    tensor built by explicit sums of outer products."""
    g = _rng(5)
    A = [g.standard_normal((s, 3)) for s in shape]
    Y = brute_kruskal(A)
    np.testing.assert_allclose(T.kruskal_full(A), Y, rtol=1e-12, atol=1e-12)
    for n in range(len(shape)):
        B = T.khatri_rao([A[p] for p in range(len(shape)) if p != n])
        np.testing.assert_allclose(T.unfold(Y, n), A[n] @ B.T,
                                   rtol=1e-12, atol=1e-12)


def test_gram_identity_eq9():
    g = _rng(6)
    A = [g.standard_normal((s, 4)) for s in (5, 6, 7, 3)]
    for n in range(4):
        B = T.khatri_rao([A[p] for p in range(4) if p != n])
        np.testing.assert_allclose(T.hadamard_grams(A, n), B.T @ B,
                                   rtol=1e-12, atol=1e-12)


def test_tucker_full_matches_loops():
    g = _rng(7)
    G = g.standard_normal((2, 3, 2))
    U = [g.standard_normal((s, r)) for s, r in zip((3, 4, 5), G.shape)]
    out = np.zeros((3, 4, 5))
    for i, j, k in itertools.product(range(3), range(4), range(5)):
        acc = 0.0
        for a, b, c in itertools.product(range(2), range(3), range(2)):
            acc += G[a, b, c] * U[0][i, a] * U[1][j, b] * U[2][k, c]
        out[i, j, k] = acc
    np.testing.assert_allclose(T.tucker_full(G, U), out, rtol=1e-12,
                               atol=1e-12)
