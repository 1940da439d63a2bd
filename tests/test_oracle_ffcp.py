"""Pins for oracle/ffcp.py (FFCP, Alg. 1, Section III-B).

The FFCP oracle never forms the dense tensor.  Here it is compared with
textbook dense CP algorithms written independently in this file (explicit
Khatri-Rao matrix B, np.linalg.solve), run on the dense Tucker tensor
Yt = [[G; U]] from the same initial factors: eq. (12) is exact for Yt, so
the iterates must agree to rounding.
"""

import itertools

import numpy as np
import pytest

import synth
from oracle import ffcp as F
from oracle import tensor as T
from oracle.metrics import factor_congruence, sir_factors


# ------------------------------------------------ independent dense references

def _kr(mats):
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        c = np.array([1.0])
        for m in mats:
            c = np.outer(c, m[:, r]).reshape(-1)
        cols.append(c)
    return np.stack(cols, axis=1)


def _unf(Y, n):
    return np.moveaxis(Y, n, 0).reshape(Y.shape[n], -1)


def _shrink(x, c):
    """The l1 proximal step written as x minus its clip to [-c, c]."""
    return x - np.clip(x, -c, c)


def dense_cp(Y, A0, rule, iters, eps=1e-16, l1=0.0):
    """Textbook CP on a dense tensor: B = KR of the other factors,
    Q = Y_(n) B, T = B^T B; ALS: A = solve; HALS: column sweep; MU.
    With l1 > 0 the sparsity step of eq. (16) follows each update.
    Columns of modes n < N normalized after each update."""
    A = [a.copy() for a in A0]
    N = Y.ndim
    hist = []
    for _ in range(iters):
        for n in range(N):
            B = _kr([A[p] for p in range(N) if p != n])
            Q = _unf(Y, n) @ B
            Tm = B.T @ B
            if rule == "als":
                A[n] = np.linalg.solve(Tm, Q.T).T
            elif rule == "hals":
                for r in range(A[n].shape[1]):
                    A[n][:, r] = np.maximum(
                        eps, A[n][:, r] + (Q[:, r] - A[n] @ Tm[:, r]) / Tm[r, r])
            elif rule == "mu":
                A[n] = A[n] * np.maximum(Q, 0) / (A[n] @ Tm + eps)
            if l1 > 0.0:
                A[n] = _shrink(A[n], l1)
                if rule == "hals":
                    A[n] = np.where(A[n] < eps, eps, A[n])
            if n < N - 1:
                nr = np.linalg.norm(A[n], axis=0)
                A[n] = A[n] / np.where(nr > 0, nr, 1.0)
        hist.append([a.copy() for a in A])
    return hist


def dense_fit(Y, A):
    Yh = np.zeros_like(Y)
    R = A[0].shape[1]
    for r in range(R):
        t = np.array([1.0])
        for a in A:
            t = np.multiply.outer(t, a[:, r])
        Yh += t.reshape(Y.shape)
    return 1.0 - np.linalg.norm(Y - Yh) / np.linalg.norm(Y)


def _tucker_case(seed, dims, ranks, nonneg=False):
    g = np.random.default_rng(seed)
    if nonneg:
        G = g.uniform(0, 1, ranks)
    else:
        G = g.standard_normal(ranks)
    U = [np.linalg.qr(g.standard_normal((I, r)))[0] for I, r in zip(dims, ranks)]
    return G, U, g


# ------------------------------------------------------------------ MTTKRP

def test_mttkrp_core_three_forms_agree():
    g = np.random.default_rng(11)
    G = g.standard_normal((3, 4, 2, 3))
    V = [g.standard_normal((s, 5)) for s in G.shape]
    for n in range(4):
        H = F.mttkrp_core(G, V, n)
        Hc = F.mttkrp_core_columns(G, V, n)
        # brute force H(j_n, r) = sum_j G(j) prod_{p != n} V_p(j_p, r)
        Hb = np.zeros_like(H)
        for j in itertools.product(*[range(s) for s in G.shape]):
            prod = np.ones(5)
            for p in range(4):
                if p != n:
                    prod = prod * V[p][j[p]]
            Hb[j[n]] += G[j] * prod
        np.testing.assert_allclose(H, Hb, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Hc, Hb, rtol=1e-12, atol=1e-12)


def test_compressed_mttkrp_exact_for_tucker_tensor():
    """eq. (12): Yt_(n) B = U_n G_(n) KR V_p for Yt = [[G;U]], V = U^T A
    (exact when U_p^T U_p = I)."""
    G, U, g = _tucker_case(12, (7, 8, 9), (3, 4, 2))
    Yt = T.tucker_full(G, U)
    A = [g.standard_normal((I, 4)) for I in (7, 8, 9)]
    V = [u.T @ a for u, a in zip(U, A)]
    for n in range(3):
        B = _kr([A[p] for p in range(3) if p != n])
        np.testing.assert_allclose(U[n] @ F.mttkrp_core(G, V, n),
                                   _unf(Yt, n) @ B, rtol=1e-11, atol=1e-11)


# --------------------------------------------------------- iterate equality

@pytest.mark.parametrize("rule", ["als", "hals", "mu"])
def test_ffcp_iterates_equal_dense_cp_on_tucker_tensor(rule):
    nonneg = rule != "als"
    dims, ranks, R = (9, 10, 11), (4, 5, 4), 3
    G, U, g = _tucker_case(13, dims, ranks, nonneg)
    Yt = T.tucker_full(G, U)
    A0 = [g.uniform(0, 1, (I, R)) if nonneg else g.standard_normal((I, R))
          for I in dims]
    iters = 30
    out = F.ffcp(U, G, A0, update=rule, max_it=iters, tol=0.0,
                 keep_iterates=iters)
    ref = dense_cp(Yt, A0, rule, iters)
    for t in range(iters):
        for n in range(3):
            a, b = out["iterates"][t][n], ref[t][n]
            assert np.linalg.norm(a - b) <= 1e-10 * max(1.0, np.linalg.norm(b))
        # closed-form fit equals the dense residual fit
        assert abs(out["fits"][t] - dense_fit(Yt, ref[t])) <= 1e-10


@pytest.mark.parametrize("rule", ["als", "hals", "mu"])
def test_ffcp_l1_iterates_equal_dense_cp_with_shrinkage(rule):
    """eq. (16): the l1-regularized variant applies S_c after every update;
    FFCP with l1 > 0 follows the dense reference that shrinks the same way
    (written as x - clip(x, -c, c)), iterate by iterate; under HALS both
    floor the result at eps.  c is large enough that entries are shrunk to
    zero (to eps under HALS) but small enough that no column vanishes."""
    nonneg = rule != "als"
    dims, ranks, R = (9, 10, 11), (4, 5, 4), 3
    G, U, g = _tucker_case(23, dims, ranks, nonneg)
    Yt = T.tucker_full(G, U)
    A0 = [g.uniform(0, 1, (I, R)) if nonneg else g.standard_normal((I, R))
          for I in dims]
    iters, c = 20, {"als": 0.02, "hals": 0.01, "mu": 0.005}[rule]
    out = F.ffcp(U, G, A0, update=rule, max_it=iters, tol=0.0, l1=c,
                 keep_iterates=iters)
    ref = dense_cp(Yt, A0, rule, iters, l1=c)
    zeros = 0
    for t in range(iters):
        for n in range(3):
            a, b = out["iterates"][t][n], ref[t][n]
            assert np.linalg.norm(a - b) <= 1e-10 * max(1.0, np.linalg.norm(b))
        zeros += sum(int(np.sum(np.abs(a) <= 1e-16)) for a in out["iterates"][t])
        # the closed-form fit still equals the dense residual fit
        assert abs(out["fits"][t] - dense_fit(Yt, ref[t])) <= 1e-10
    assert zeros > 0
    assert not out["ridged"]
    assert all(np.all(np.isfinite(a)) for a in out["A"])


def test_soft_threshold_branches_eq16():
    """The three branches of the sparsity operator S_c (eq. 16) at points on
    both sides of, and at, the thresholds +-c."""
    c = 0.25
    x = np.array([1.5, 0.75, 0.25, 0.125, 0.0, -0.125, -0.25, -0.5, -2.0])
    want = np.array([1.25, 0.5, 0.0, 0.0, 0.0, 0.0, 0.0, -0.25, -1.75])
    assert np.array_equal(F.soft_threshold(x, c), want)
    assert np.array_equal(F.soft_threshold(x, 0.0), x)


def test_soft_threshold_is_the_l1_proximal_point():
    """S_c(x) minimizes (z - x)^2 / 2 + c |z| over z (the property that makes
    it the update of l1-regularized CP, eq. 16); brute force over a grid of
    spacing 1e-5."""
    grid = np.linspace(-3.0, 3.0, 600001)
    for c in (0.0, 0.2, 0.7):
        for x in (-2.5, -0.65, -0.2, -0.05, 0.0, 0.1, 0.45, 1.9):
            z = grid[np.argmin(0.5 * (grid - x) ** 2 + c * np.abs(grid))]
            assert abs(F.soft_threshold(np.array([x]), c)[0] - z) <= 1e-5


def test_ffcp_equals_cp_of_core_eq17():
    """eq. (17) / eq. (10): with orthonormal U, FFCP-ALS from A0 follows
    CP-ALS of the core from V0 = U^T A0, with A = U V, when A0 lies in
    range(U) (so V = U^T A loses nothing)."""
    dims, ranks, R = (12, 13, 14), (4, 4, 4), 3
    G, U, g = _tucker_case(14, dims, ranks)
    V0 = [g.standard_normal((r, R)) for r in ranks]
    A0 = [u @ v for u, v in zip(U, V0)]
    out = F.ffcp(U, G, A0, update="als", max_it=25, tol=0.0, keep_iterates=25)
    core = F.core_cp_als(G, V0, max_it=25, tol=0.0)
    for n in range(3):
        np.testing.assert_allclose(out["A"][n], U[n] @ core["A"][n],
                                   rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(out["lam"], core["lam"], rtol=1e-9)
    np.testing.assert_allclose(out["fits"], core["fits"], rtol=1e-10,
                               atol=1e-12)


@pytest.mark.parametrize("rule", ["als", "hals"])
def test_fit_monotone(rule):
    nonneg = rule == "hals"
    dims, R = (20, 21, 22), 4
    g = np.random.default_rng(15)
    if nonneg:
        A = [g.uniform(0, 1, (I, R)) for I in dims]
    else:
        A = [g.standard_normal((I, R)) for I in dims]
    Y = synth.cp_tensor(A) + 0.05 * g.standard_normal(dims)
    # exact Tucker format of Y (full ranks) so FFCP sees Y itself
    U = [np.eye(I) for I in dims]
    A0 = [g.uniform(0, 1, (I, R)) for I in dims]
    out = F.ffcp(U, Y, A0, update=rule, max_it=60, tol=0.0)
    d = np.diff(out["fits"])
    assert np.all(d >= -1e-12)


def test_hals_kkt_at_convergence():
    dims, R = (15, 16, 17), 3
    g = np.random.default_rng(16)
    A = [g.uniform(0, 1, (I, R)) for I in dims]
    Y = synth.cp_tensor(A) + 0.01 * np.abs(g.standard_normal(dims))
    U = [np.eye(I) for I in dims]
    A0 = [g.uniform(0, 1, (I, R)) for I in dims]
    out = F.ffcp(U, Y, A0, update="hals", max_it=3000, tol=1e-15)
    Af = [a.copy() for a in out["A"]]
    Af[-1] = Af[-1] * out["lam"]
    for n in range(3):
        B = _kr([Af[p] for p in range(3) if p != n])
        grad = Af[n] @ (B.T @ B) - _unf(Y, n) @ B      # eq. (5)
        assert np.all(Af[n] >= 0)
        kkt = np.abs(np.minimum(Af[n], grad))
        scale = np.abs(_unf(Y, n) @ B).max()    # size of the gradient's terms
        assert kkt.max() <= 1e-6 * scale


def test_closed_form_fit_vs_dense_for_general_U():
    """||Yt||^2 = <G, G x_n U_n^T U_n> holds for non-orthonormal U too."""
    g = np.random.default_rng(17)
    G = g.standard_normal((3, 2, 4))
    U = [g.standard_normal((I, r)) for I, r in zip((6, 5, 7), G.shape)]
    Yt = T.tucker_full(G, U)
    assert abs(F.tucker_norm2(U, G) - np.sum(Yt * Yt)) <= 1e-10 * np.sum(Yt * Yt)
    A0 = [g.standard_normal((I, 2)) for I in (6, 5, 7)]
    out = F.ffcp(U, G, A0, update="als", max_it=8, tol=0.0, keep_iterates=8)
    for t in range(8):
        assert abs(out["fits"][t] - dense_fit(Yt, out["iterates"][t])) <= 1e-10


def test_ridge_fallback_on_singular_gram():
    """A zero column in the initial factors makes T singular: the ALS solve
    takes the ridge path and reports it."""
    G, U, g = _tucker_case(18, (8, 9, 10), (3, 3, 3))
    A0 = [g.standard_normal((I, 3)) for I in (8, 9, 10)]
    A0[1][:, 2] = 0.0
    A0[2][:, 2] = 0.0
    out = F.ffcp(U, G, A0, update="als", max_it=3, tol=0.0)
    assert out["ridged"]
    assert np.all(np.isfinite(out["A"][0]))


# ------------------------------------------------- brute force, tiny tensors

@pytest.mark.parametrize("shape,R", [((3, 3, 3), 2), ((4, 4, 4), 3)])
def test_bruteforce_tiny_cp_noise_free(shape, R):
    """Best of 20 seeded ALS starts recovers an exact CP tensor.  The fit is
    measured from the dense residual: the closed-form fit of the stopping
    rule cancels to about sqrt(eps) when the fit is near 1."""
    g = np.random.default_rng(19 + R)
    A = [g.standard_normal((I, R)) for I in shape]
    Y = synth.cp_tensor(A)
    U = [np.eye(I) for I in shape]
    best, best_fit = None, -np.inf
    for s in range(20):
        gs = np.random.default_rng(500 + s)
        A0 = [gs.standard_normal((I, R)) for I in shape]
        out = F.ffcp(U, Y, A0, update="als", max_it=1500, tol=0.0)
        f = F.cp_fit_dense(Y, out["A"], out["lam"])
        if f > best_fit:
            best, best_fit = out, f
    assert best_fit >= 1.0 - 1e-12
    Ab = [a.copy() for a in best["A"]]
    _, cong = factor_congruence(A, Ab)
    assert cong >= 1.0 - 1e-10


def test_bruteforce_tiny_cp_noisy_single_start_near_best():
    shape, R = (4, 4, 4), 2
    g = np.random.default_rng(23)
    A = [g.standard_normal((I, R)) for I in shape]
    Y = synth.cp_tensor(A) + 0.05 * g.standard_normal(shape)
    U = [np.eye(I) for I in shape]
    fits = []
    for s in range(30):
        gs = np.random.default_rng(700 + s)
        A0 = [gs.standard_normal((I, R)) for I in shape]
        fits.append(F.ffcp(U, Y, A0, update="als", max_it=3000,
                           tol=1e-14)["fits"][-1])
    gs = np.random.default_rng(9999)
    A0 = [gs.standard_normal((I, R)) for I in shape]
    one = F.ffcp(U, Y, A0, update="als", max_it=3000, tol=1e-14)["fits"][-1]
    assert max(fits) - one <= 1e-8


def test_fit_definitions_agree():
    g = np.random.default_rng(24)
    A = [g.standard_normal((I, 3)) for I in (5, 6, 7)]
    Y = synth.cp_tensor(A) + 0.1 * g.standard_normal((5, 6, 7))
    lam = np.array([1.0, 2.0, 0.5])
    assert abs(F.cp_fit_dense(Y, A, lam) - F.cp_fit_mttkrp(Y, A, lam)) <= 1e-12


def test_hosvd_init_eigenvectors():
    G, U, g = _tucker_case(25, (10, 11, 12), (4, 5, 3))
    pad = [g.standard_normal((r, 2)) if r < 5 else None for r in (4, 5, 3)]
    pad[2] = g.standard_normal((3, 2))
    A = F.hosvd_init(U, G, 5, pad=[pad[0], None, pad[2]])
    for n, r in enumerate((4, 5, 3)):
        V = U[n].T @ A[n]
        Gn = _unf(G, n)
        k = min(r, 5)
        Vk = V[:, :k]
        S = Gn @ Gn.T
        # eigen-equation and orthonormality of the eigen part
        lam = np.diag(Vk.T @ S @ Vk)
        np.testing.assert_allclose(S @ Vk, Vk * lam, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(Vk.T @ Vk, np.eye(k), atol=1e-12)
        assert np.all(np.diff(lam) <= 1e-12)


# ------------------------------------------- the paper's noise-free example

def test_nonneg_tucker_format_is_the_cp_model():
    """The seeded Tucker format of the 10^4-per-mode HALS workload (here at
    small sizes): [[G; U]] equals the dense nonnegative CP tensor, U_n is
    orthonormal, each factor has exactly 20 % zeros."""
    dims, R = (12, 13, 14, 15), 3
    d = synth.nonneg_tucker_format(28, dims, R, "exp", 10.0, 0.2)
    Y = np.einsum("ir,jr,kr,lr->ijkl", *d["A"])
    Yt = T.multi_ttm_t(d["G"], [u.T for u in d["U"]])
    assert np.linalg.norm(Yt - Y) <= 1e-13 * np.linalg.norm(Y)
    for I, u, a in zip(dims, d["U"], d["A"]):
        assert np.linalg.norm(u.T @ u - np.eye(R)) <= 1e-13
        assert int(np.sum(a == 0.0)) == round(0.2 * I * R)
        assert a.min() >= 0.0


@pytest.mark.slow
def test_paper_noise_free_nonneg_recovery_sir():
    """Section V-A (the 10^4 x 10^4 x 10^4 x 10^4 example, scaled to
    I = 2000): exponential(mean 10) factors with 20% zeros, R = 10, exact
    Tucker format U_n = orth(A_n), G = I_R x_n R_n.  FFCP-HALS recovers the
    components with SIR > 200 dB."""
    dims, R = (2000, 2000, 2000, 2000), 10
    g = synth.rngs(26)
    A = synth.nonneg_factors(g["factors"], dims, R, "exp", 10.0, 0.2)
    U, Rs = [], []
    for a in A:
        q, r = np.linalg.qr(a)
        U.append(q)
        Rs.append(r)
    G = np.zeros((R,) * 4)
    for r in range(R):
        G[(r,) * 4] = 1.0
    G = T.multi_ttm_t(G, [r_.T for r_ in Rs])
    A0 = synth.init_factors(g["init"], dims, R, nonneg=True)
    out = F.ffcp(U, G, A0, update="hals", max_it=3000, tol=1e-16)
    sirs = np.concatenate([sir_factors(A[n], out["A"][n]) for n in range(4)])
    assert sirs.min() > 200.0
