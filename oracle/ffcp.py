"""FFCP: CP / nonnegative CP fitted through a Tucker format (Section III-B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1, per iteration, for n = 1..N in ascending order:
  H_n  = G_(n) [KR_{p != n} V_p]                       (eq. 12-13)
  Q_n  = U_n H_n        (approximates Y_(n) B_n, exact for the Tucker tensor)
  T_n  = hadamard_{p != n} A_p^T A_p                   (eq. 9)
  update A_n with ALS (eq. 14), HALS (eq. 8) or MU (eq. 15); optional
  soft threshold S_c (eq. 16)
  V_n  = U_n^T A_n                                     (eq. 13)

Readings of the paper (each listed in the design doc):
  * eq. (8) as printed puts the projection inside the increment, so a column
    could never shrink; the update used is the standard HALS one,
    a_r <- max(eps, a_r + (q_r - A t_r) / t_rr), columns r = 1..R in order,
    in place, eps = 1e-16 so t_rr stays positive.
  * ALS solves A_n T_n = Q_n by Cholesky; if T_n is not positive definite a
    ridge delta = 1e-12 tr(T_n) / R is added and a flag is set.
  * MU (eq. 15) adds eps = 1e-16 to the denominator.
  * The sparsity step S_c of eq. (16) follows the update.  Under HALS the
    result is put back onto HALS's feasible set a >= eps: the shrinkage can
    zero a whole column, and t_rr of the next update would then vanish.
    max(eps, S_c(a)) is the proximal point of c*a plus the constraint
    a >= eps, i.e. the same l1 term under the same constraint.
  * Scale: lambda is absorbed into A_N (eq. 2); after each update of a mode
    n < N its columns are normalized to unit 2-norm (zero columns stay zero);
    at the end lambda_r = ||a_r^(N)|| and A_N is normalized.
  * Fit (Section III-B): Fit = 1 - ||Yt - Yhat|| / ||Yt|| (not squared), with
    Yt = [[G; U]] the tensor FFCP actually fits.  It is evaluated in closed
    form after mode N: ||Yt||^2 = <G, G x_n U_n^T U_n>, <Yt, Yhat> =
    sum(H_N * V_N), ||Yhat||^2 = 1^T (hadamard_p A_p^T A_p) 1.
  * Stop (Section V-A): at iteration t >= 2 when |Fit_t - Fit_{t-1}| < tol,
    or at max_it.

Pins: tests/test_oracle_ffcp.py (iterate-by-iterate equality with textbook
dense CP-ALS / HALS on the dense Tucker tensor; equality with CP-ALS of the
core when U is orthonormal, eq. (17); closed-form fit vs dense residual;
monotone fit; KKT of HALS at convergence; brute-force CP on tiny tensors;
the noise-free nonnegative recovery of Section V-A with SIR > 200 dB).
"""

import numpy as np

from .tensor import unfold, khatri_rao, multi_ttm_t, hadamard_grams, ttm_t
from .randtucker import sorted_sign_fixed_eigvecs

HALS_EPS = 1e-16
MU_EPS = 1e-16


def mttkrp_core(G, V, n):
    """H = G_(n) [KR_{p != n} V_p] (eq. 12), the compressed MTTKRP."""
    others = [V[p] for p in range(G.ndim) if p != n]
    return unfold(G, n) @ khatri_rao(others)


def mttkrp_core_columns(G, V, n):
    """Column form of H: h_r = G x_{p != n} v_r^(p)T (Section III-B)."""
    R = V[0].shape[1]
    cols = []
    for r in range(R):
        vecs = [None if p == n else V[p][:, r:r + 1] for p in range(G.ndim)]
        cols.append(multi_ttm_t(G, vecs).reshape(-1))
    return np.stack(cols, axis=1)


def soft_threshold(A, c):
    """S_c of eq. (16), element-wise."""
    return np.sign(A) * np.maximum(np.abs(A) - c, 0.0)


def tucker_norm2(U, G):
    """||[[G; U]]||^2 = <G, G x_n (U_n^T U_n)> (exact for any U)."""
    G = np.asarray(G, dtype=np.float64)
    return float(np.sum(G * multi_ttm_t(G, [u.T @ u for u in U])))


def als_update(Q, T):
    """A = Q T^{-1} by Cholesky (eq. 14); ridge fallback. Returns (A, ridged)."""
    R = T.shape[0]
    try:
        L = np.linalg.cholesky(T)
        ridged = False
    except np.linalg.LinAlgError:
        L = np.linalg.cholesky(T + (1e-12 * np.trace(T) / R) * np.eye(R))
        ridged = True
    # solve A L L^T = Q
    Y = np.linalg.solve(L, Q.T)          # L Y = Q^T
    X = np.linalg.solve(L.T, Y)          # L^T X = Y
    return X.T, ridged


def hals_update(A, Q, T, eps=HALS_EPS):
    """Column-wise HALS (eq. 8, standard form), in order r = 1..R."""
    A = A.copy()
    for r in range(A.shape[1]):
        A[:, r] = np.maximum(eps, A[:, r] + (Q[:, r] - A @ T[:, r]) / T[r, r])
    return A


def mu_update(A, Q, T, eps=MU_EPS):
    """Multiplicative update through the Tucker format (eq. 15)."""
    return A * np.maximum(Q, 0.0) / (A @ T + eps)


def normalize_columns(A):
    nrm = np.linalg.norm(A, axis=0)
    safe = np.where(nrm > 0, nrm, 1.0)
    return A / safe, nrm


def ffcp(U, G, A_init, update="als", max_it=1000, tol=1e-6, l1=0.0,
         normY2=None, keep_iterates=0):
    """Alg. 1 on the Tucker format [[G; U]].

    U       : list of N factor matrices I_n x R_n.
    G       : core R_1 x ... x R_N.
    A_init  : list of N matrices I_n x R (used as given).
    update  : "als" | "hals" | "mu".
    Returns dict(A=normalized factors, lam, fits, iterations, converged,
    ridged, iterates=[A after each of the first keep_iterates iterations]).
    """
    G = np.asarray(G, dtype=np.float64)
    U = [np.asarray(u, dtype=np.float64) for u in U]
    A = [np.asarray(a, dtype=np.float64).copy() for a in A_init]
    N = G.ndim
    V = [U[n].T @ A[n] for n in range(N)]
    grams = [a.T @ a for a in A]
    nrm2 = tucker_norm2(U, G) if normY2 is None else float(normY2)
    fits, iterates = [], []
    ridged = False
    converged = False
    it = 0
    for it in range(1, max_it + 1):
        for n in range(N):
            H = mttkrp_core(G, V, n)
            Q = U[n] @ H
            T = hadamard_grams(A, n) if N > 1 else np.ones((1, 1))
            if update == "als":
                A[n], r_ = als_update(Q, T)
                ridged |= r_
            elif update == "hals":
                A[n] = hals_update(A[n], Q, T)
            elif update == "mu":
                A[n] = mu_update(A[n], Q, T)
            else:
                raise ValueError(update)
            if l1 > 0.0:
                A[n] = soft_threshold(A[n], l1)
                if update == "hals":
                    # back onto HALS's feasible set a >= eps (t_rr > 0)
                    A[n] = np.maximum(HALS_EPS, A[n])
            if n < N - 1:
                A[n], _ = normalize_columns(A[n])
            V[n] = U[n].T @ A[n]
            grams[n] = A[n].T @ A[n]
            if n == N - 1:
                inner = float(np.sum(H * V[n]))
        Ghad = np.ones_like(grams[0])
        for g in grams:
            Ghad = Ghad * g
        res2 = nrm2 - 2.0 * inner + float(np.sum(Ghad))
        fit = 1.0 - np.sqrt(max(res2, 0.0)) / np.sqrt(nrm2)
        fits.append(fit)
        if len(iterates) < keep_iterates:
            iterates.append([a.copy() for a in A])
        if it >= 2 and abs(fits[-1] - fits[-2]) < tol:
            converged = True
            break
    AN, lam = normalize_columns(A[N - 1])
    A_out = [a.copy() for a in A[:N - 1]] + [AN]
    return {"A": A_out, "lam": lam, "fits": fits, "iterations": it,
            "converged": converged, "ridged": ridged, "iterates": iterates}


def hosvd_init(U, G, R, pad=None):
    """HOSVD initialization (Alg. 1's initialization step): V_n = top-R eigenvectors of
    G_(n) G_(n)^T; when R > R_n the missing columns come from ``pad[n]``
    (R_n x (R - R_n), given Gaussian numbers).  Returns A_n = U_n V_n."""
    A = []
    for n in range(G.ndim):
        Gn = unfold(G, n)
        k = min(R, Gn.shape[0])
        _, Vn = sorted_sign_fixed_eigvecs(Gn @ Gn.T, k)
        if k < R:
            Vn = np.concatenate([Vn, np.asarray(pad[n], dtype=np.float64)],
                                axis=1)
        A.append(np.asarray(U[n], dtype=np.float64) @ Vn)
    return A


def cp_fit_dense(Y, A, lam=None):
    """Fit(Y, Yhat) = 1 - ||Y - Yhat|| / ||Y|| from the dense residual."""
    from .tensor import kruskal_full
    Y = np.asarray(Y, dtype=np.float64)
    return 1.0 - np.linalg.norm(Y - kruskal_full(A, lam)) / np.linalg.norm(Y)


def cp_fit_mttkrp(Y, A, lam=None):
    """Same fit through one MTTKRP over Y: <Y, Yhat> = sum(A_N * Y_(N) B_N)."""
    Y = np.asarray(Y, dtype=np.float64)
    A = [np.asarray(a, dtype=np.float64) for a in A]
    N = Y.ndim
    R = A[0].shape[1]
    w = np.ones(R) if lam is None else np.asarray(lam, dtype=np.float64)
    AN = A[N - 1] * w
    inner = float(np.sum(AN * (unfold(Y, N - 1) @ khatri_rao(A[:N - 1]))))
    Ghad = np.outer(w, w)
    for a in A:
        Ghad = Ghad * (a.T @ a)
    y2 = float(np.sum(Y * Y))
    res2 = y2 - 2.0 * inner + float(np.sum(Ghad))
    return 1.0 - np.sqrt(max(res2, 0.0)) / np.sqrt(y2)


def core_cp_als(G, V_init, max_it=1000, tol=1e-6):
    """Tucker+CP (eq. 10): CP-ALS of the core itself with the same stopping
    and scaling rules; used to pin eq. (17)."""
    N = G.ndim
    I = [np.eye(s) for s in G.shape]
    return ffcp(I, G, V_init, update="als", max_it=max_it, tol=tol)
