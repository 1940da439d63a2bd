"""Pins for oracle/randtucker.py (RandTucker / RandTucker2i, Section IV-A).

Exact recovery of noise-free tensors of known multilinear rank,
orthonormality, the core/Pythagoras identity and the R~_n = I_n special case
that reduces to the truncated HOSVD computed from numpy's SVD.
"""

import numpy as np
import pytest

import synth
from oracle import randtucker as RT
from oracle import tensor as T
from oracle.metrics import projector_distance


def _randoms(case, dims, rt, sweeps=2):
    g = synth.rngs(case)
    om = synth.omegas(g["omega"], dims, rt)
    omt = [synth.omega_tildes(g["omega_t1"], rt),
           synth.omega_tildes(g["omega_t2"], rt)][:sweeps]
    return om, omt


@pytest.mark.parametrize("order", ["jacobi", "gauss_seidel"])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_exact_recovery_mixed_multilinear_rank(order, sweeps):
    dims, ranks = (20, 25, 30), (3, 5, 7)
    rt = (8, 9, 10)
    g = synth.rngs(101)
    G = g["factors"].standard_normal(ranks)
    U = synth.orthonormal_factors(g["factors"], dims, ranks)
    Y = synth.tucker_tensor(G, U)
    om, omt = _randoms(101, dims, rt, sweeps)
    out = RT.rand_tucker(Y, om, omt, sweeps=sweeps, ranks=ranks, order=order)
    for n in range(3):
        assert projector_distance(out["U"][n], U[n]) <= 1e-10
        Q = out["Q"][n]
        assert np.linalg.norm(Q.T @ Q - np.eye(rt[n])) <= 1e-13
        Un = out["U"][n]
        assert np.linalg.norm(Un.T @ Un - np.eye(ranks[n])) <= 1e-13
    rec = T.tucker_full(out["G"], out["U"])
    assert np.linalg.norm(rec - Y) / np.linalg.norm(Y) <= 1e-12


def test_exact_recovery_cp_rank_below_sketch():
    dims, R, rt = (15, 16, 17, 6), 4, (6, 6, 6, 5)
    g = synth.rngs(102)
    A = synth.gaussian_factors(g["factors"], dims, R)
    Y = synth.cp_tensor(A)
    om, omt = _randoms(102, dims, rt, 1)
    out = RT.rand_tucker(Y, om, omt, sweeps=1, ranks=(R, R, R, R))
    for n in range(4):
        assert projector_distance(out["U"][n], A[n]) <= 1e-10
    rec = T.tucker_full(out["G"], out["U"])
    assert np.linalg.norm(rec - Y) / np.linalg.norm(Y) <= 1e-12


def test_rank_deficient_sketch_still_orthonormal():
    """True multilinear rank 2 < R~ = 6: Z_n has rank 2, Householder QR
    still returns an orthonormal Q containing the true subspace."""
    dims, ranks, rt = (12, 13, 14), (2, 2, 2), (6, 6, 6)
    g = synth.rngs(103)
    G = g["factors"].standard_normal(ranks)
    U = synth.orthonormal_factors(g["factors"], dims, ranks)
    Y = synth.tucker_tensor(G, U)
    om, omt = _randoms(103, dims, rt, 1)
    out = RT.rand_tucker(Y, om, omt, sweeps=1, ranks=None)
    for n in range(3):
        Q = out["Q"][n]
        assert np.linalg.norm(Q.T @ Q - np.eye(6)) <= 1e-12
        # the true basis lies inside range(Q)
        resid = U[n] - Q @ (Q.T @ U[n])
        assert np.linalg.norm(resid) <= 1e-10


def test_core_and_pythagoras_identity_noisy():
    dims, rt, ranks = (30, 32, 34), (12, 12, 12), (8, 8, 8)
    d = synth.case_tucker(104, dims, ranks, 10.0, rt, sweeps=2)
    Y = d["Y"]
    out = RT.rand_tucker(Y, d["omegas"], d["omega_tildes"], sweeps=2,
                         ranks=ranks)
    # G = Y x_n U_n^T exactly (truncation is a rotation of the sketch core)
    np.testing.assert_allclose(out["G"], T.multi_ttm_t(Y, out["U"]),
                               rtol=1e-11, atol=1e-11)
    res = Y - T.tucker_full(out["G"], out["U"])
    lhs = np.sum(Y * Y)
    rhs = np.sum(out["G"] ** 2) + np.sum(res * res)
    assert abs(lhs - rhs) / lhs <= 1e-12


def test_full_width_sketch_equals_truncated_hosvd():
    """R~_n = I_n: range(Q_n) is all of R^{I_n}, so truncation through the
    core's Gram eigenvectors is exactly the truncated HOSVD (numpy SVD)."""
    dims, ranks = (9, 10, 11), (3, 4, 5)
    g = synth.rngs(105)
    Y = g["factors"].standard_normal(dims)
    om, omt = _randoms(105, dims, dims, 1)
    out = RT.rand_tucker(Y, om, omt, sweeps=1, ranks=ranks)
    Uh, Gh = RT.hosvd(Y, ranks)
    for n in range(3):
        assert projector_distance(out["U"][n], Uh[n]) <= 1e-10
    # cores agree up to the sign of each basis vector
    s = [np.sign(np.sum(a * b, axis=0)) for a, b in zip(out["U"], Uh)]
    Ga = T.multi_ttm_t(out["G"], [np.diag(x) for x in s])
    np.testing.assert_allclose(Ga, Gh, rtol=1e-9, atol=1e-9)


def test_sequential_alg2_exact_recovery():
    dims, ranks, rt = (10, 11, 12), (2, 3, 4), (5, 5, 5)
    g = synth.rngs(106)
    G = g["factors"].standard_normal(ranks)
    U = synth.orthonormal_factors(g["factors"], dims, ranks)
    Y = synth.tucker_tensor(G, U)
    # dense Omega_n rows = product of current other dims (earlier ones shrunk)
    cur = list(dims)
    oms = []
    for n in range(3):
        rows = int(np.prod([cur[p] for p in range(3) if p != n]))
        oms.append(g["omega"].standard_normal((rows, rt[n])))
        cur[n] = rt[n]
    Us, Gs = RT.rand_tucker_sequential(Y, oms)
    for n in range(3):
        assert projector_distance(
            Us[n] @ np.linalg.svd(T.unfold(Gs, n))[0][:, :ranks[n]],
            U[n]) <= 1e-10
    rec = T.tucker_full(Gs, Us)
    assert np.linalg.norm(rec - Y) / np.linalg.norm(Y) <= 1e-12


def test_sketch_matches_structured_random_matrix():
    """Z_n = X_(n) Omega~_n equals Y_(n) ((kron_{p != n} Omega_p) Omega~_n):
    the Jacobi sketch is the range finder applied with a Kronecker-
    structured Gaussian test matrix (Section IV-A step 1-2)."""
    dims, rt = (5, 6, 7), (3, 4, 2)
    g = synth.rngs(107)
    Y = g["factors"].standard_normal(dims)
    om, omt = _randoms(107, dims, rt, 1)
    for n in range(3):
        K = np.ones((1, 1))
        for p in range(3):
            if p != n:
                K = np.kron(K, om[p])
        Zd = T.unfold(Y, n) @ (K @ omt[0][n])
        np.testing.assert_allclose(RT.sketch(Y, om, omt[0][n], n), Zd,
                                   rtol=1e-12, atol=1e-12)


@pytest.mark.slow
def test_randtucker2i_close_to_hosvd_statistically():
    """Section IV-A claim (Fig. 4; values are figure-only, so parity
    unpinned): at the paper's 200^3, R_n = 10, p = 10 setting with heavy
    noise, RandTucker2i (two sweeps) is almost as good as the HOSVD, and
    clearly better than one sweep; at low noise both are near the HOSVD."""
    for dims, snr, tol in (((200, 200, 200), 10.0, 0.01),
                           ((100, 100, 100), 30.0, 0.005)):
        ranks, rt = (10, 10, 10), (20, 20, 20)
        d = synth.case_tucker((108, int(snr)), dims, ranks, snr, rt, sweeps=2)
        fit = {}
        for sw in (1, 2):
            out = RT.rand_tucker(d["Y"], d["omegas"], d["omega_tildes"],
                                 sweeps=sw, ranks=ranks)
            fit[sw] = RT.tucker_fit(d["Y"], out["U"], out["G"])
        Uh, Gh = RT.hosvd(d["Y"], ranks)
        fh = RT.tucker_fit(d["Y"], Uh, Gh)
        assert fit[2] >= fh - tol
        assert fit[2] > fit[1]


def test_gram_evd_basis_eq23_spans_the_qr_basis():
    """eq. (23): U = Z W S^{-1/2} from the eigendecomposition Z^T Z = W S W^T
    is orthonormal and spans range(Z), the same subspace as Householder QR,
    for a full-column-rank Z."""
    g = np.random.default_rng(131)
    for shape in ((50, 8), (300, 30), (9, 9)):
        Z = g.standard_normal(shape) @ np.diag(np.linspace(1.0, 5.0, shape[1]))
        U = RT.orth_gram_evd(Z)
        assert np.linalg.norm(U.T @ U - np.eye(shape[1])) <= 1e-12
        assert projector_distance(U, RT.orth_qr(Z)) <= 1e-12


def test_gram_evd_basis_on_orthogonal_columns_closed_form():
    """Z = Q0 D with orthonormal Q0 and distinct positive D: Z^T Z = D^2 is
    diagonal, so the eq. (23) basis is Q0's columns ordered by descending D,
    up to sign."""
    g = np.random.default_rng(132)
    Q0 = np.linalg.qr(g.standard_normal((20, 4)))[0]
    D = np.array([3.0, 5.0, 1.0, 4.0])
    U = RT.orth_gram_evd(Q0 * D)
    order = [1, 3, 0, 2]
    np.testing.assert_allclose(np.abs(U.T @ Q0[:, order]), np.eye(4), atol=1e-13)


def test_eigvec_order_and_sign_rule():
    """Top-k eigenvectors of S = V diag(w) V^T come out in descending
    eigenvalue order, each column's largest-magnitude entry positive."""
    g = np.random.default_rng(133)
    V = np.linalg.qr(g.standard_normal((6, 6)))[0]
    w = np.array([0.5, 4.0, -1.0, 2.5, 7.0, 1.0])
    S = V @ np.diag(w) @ V.T
    ws, Vs = RT.sorted_sign_fixed_eigvecs(S, 4)
    order = [4, 1, 3, 5]
    np.testing.assert_allclose(ws, w[order], atol=1e-12)
    for c, i in enumerate(order):
        v = V[:, i]
        v = v if v[np.argmax(np.abs(v))] > 0 else -v
        np.testing.assert_allclose(Vs[:, c], v, atol=1e-12)
        assert Vs[np.argmax(np.abs(Vs[:, c])), c] > 0
