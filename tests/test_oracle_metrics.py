"""Pins for oracle/metrics.py against closed forms."""

import numpy as np

from oracle import metrics as Mt


def test_projector_distance_known_angle():
    for th in (1e-9, 1e-4, 0.3, 1.2):
        U = np.array([[1.0], [0.0], [0.0]])
        W = np.array([[np.cos(th)], [np.sin(th)], [0.0]])
        assert abs(Mt.projector_distance(U, W) - np.sin(th)) <= 1e-15 + 1e-12 * th


def test_projector_distance_rotation_invariant():
    g = np.random.default_rng(41)
    U = np.linalg.qr(g.standard_normal((10, 3)))[0]
    Rot = np.linalg.qr(g.standard_normal((3, 3)))[0]
    assert Mt.projector_distance(U, U @ Rot) <= 1e-14


def test_match_columns_recovers_permutation_and_scale():
    g = np.random.default_rng(42)
    A = g.standard_normal((20, 5))
    perm = np.array([3, 0, 4, 1, 2])
    B = A[:, perm] * np.array([2.0, -1.0, 0.5, 3.0, -4.0])
    p, cong = Mt.match_columns(A, B)
    np.testing.assert_array_equal(perm[p], np.arange(5))
    np.testing.assert_allclose(cong, 1.0, atol=1e-14)


def test_sir_closed_form():
    a = np.sin(np.linspace(0, 7, 200))
    assert Mt.sir_db(a, a) == np.inf
    e = np.random.default_rng(43).standard_normal(200)
    e = e - e.mean()
    b = a + 1e-3 * e
    an = (a - a.mean()) / a.std()
    bn = (b - b.mean()) / b.std()
    ref = 20 * np.log10(np.linalg.norm(an) / np.linalg.norm(an - bn))
    assert abs(Mt.sir_db(a, -3.0 * b + 5.0) - ref) <= 1e-9


def test_aligned_core_error_invariant_to_basis_rotation():
    g = np.random.default_rng(44)
    G = g.standard_normal((3, 4, 2))
    U = [np.linalg.qr(g.standard_normal((8, r)))[0] for r in G.shape]
    Rs = [np.linalg.qr(g.standard_normal((r, r)))[0] for r in G.shape]
    from oracle.tensor import multi_ttm_t
    Ua = [u @ r for u, r in zip(U, Rs)]
    Ga = multi_ttm_t(G, Rs)          # same tensor, rotated bases
    assert Mt.aligned_core_error(Ga, Ua, G, U) <= 1e-13
