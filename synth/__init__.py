"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds none of the method's arithmetic: it only draws random
numbers and assembles test tensors from CP / Tucker models with NumPy (or
torch, for tensors too large for host FP64) library contractions.  Every
random matrix the method consumes (Omega_n, Omega~_n, initial factors) is
drawn here and passed to both the HIP library and the oracle.

Seeds: numpy SeedSequence(entropy=14121885, spawn_key=(case,)), children in
the fixed order [factors, noise, omega, omega_tilde_1, omega_tilde_2, init].

Workload recipes follow the paper's synthetic experiments (Section V-A):
Gaussian CP factors, exponential / uniform nonnegative factors with a fixed
fraction of zeros, Tucker models with orthonormal factors, and additive
Gaussian noise at an exact SNR (SNR_dB = 10 log10(||Y*||^2 / ||E||^2)).
"""

import numpy as np

ENTROPY = 14121885
CHILDREN = ("factors", "noise", "omega", "omega_t1", "omega_t2", "init")


def rngs(case):
    """Named numpy Generators for a case id (int or tuple)."""
    key = case if isinstance(case, tuple) else (case,)
    ss = np.random.SeedSequence(entropy=ENTROPY, spawn_key=key)
    return {name: np.random.default_rng(child)
            for name, child in zip(CHILDREN, ss.spawn(len(CHILDREN)))}


# ----------------------------------------------------------------- factors

def gaussian_factors(rng, dims, R):
    return [rng.standard_normal((I, R)) for I in dims]


def congruent_factors(rng, dims, R, c_lo, c_hi):
    """Unit-norm columns with all pairwise cosines equal to c_n ~ U[c_lo, c_hi]
    per mode: A_n = Q_n L^T, Q_n orthonormal (I x R), L L^T = (1-c) I + c 11^T."""
    out = []
    for I in dims:
        c = rng.uniform(c_lo, c_hi)
        q, _ = np.linalg.qr(rng.standard_normal((I, R)))
        C = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
        L = np.linalg.cholesky(C)
        out.append(q @ L.T)
    return out


def nonneg_factors(rng, dims, R, dist="exp", scale=10.0, zero_frac=0.1):
    """Nonnegative factors: exponential (mean ``scale``) or U[0,1], with
    exactly round(zero_frac * I * R) entries per factor set to zero."""
    out = []
    for I in dims:
        if dist == "exp":
            A = rng.exponential(scale, size=(I, R))
        elif dist == "uniform":
            A = rng.uniform(0.0, 1.0, size=(I, R))
        else:
            raise ValueError(dist)
        nz = int(round(zero_frac * I * R))
        idx = rng.choice(I * R, size=nz, replace=False)
        A.reshape(-1)[idx] = 0.0
        out.append(A)
    return out


def orthonormal_factors(rng, dims, ranks):
    return [np.linalg.qr(rng.standard_normal((I, r)))[0]
            for I, r in zip(dims, ranks)]


# ----------------------------------------------------------------- tensors

_LETTERS = "abcdefghij"


def cp_tensor(A, lam=None):
    """Dense sum_r lam_r a_r^(1) o ... o a_r^(N) by numpy einsum."""
    N = len(A)
    R = A[0].shape[1]
    w = np.ones(R) if lam is None else np.asarray(lam)
    spec = ",".join(_LETTERS[n] + "z" for n in range(N)) + ",z->" + \
        _LETTERS[:N]
    return np.einsum(spec, *A, w, optimize=True)


def tucker_tensor(G, U):
    """Dense G x_1 U_1 ... x_N U_N by numpy einsum."""
    N = G.ndim
    core = _LETTERS[:N]
    outs = "klmnopqrst"[:N]
    spec = core + "," + ",".join(outs[n] + core[n] for n in range(N)) + \
        "->" + outs
    return np.einsum(spec, G, *U, optimize=True)


def add_gaussian_noise(Y, rng, snr_db):
    """Y* + E with E Gaussian scaled so 10 log10(||Y*||^2/||E||^2) = snr_db."""
    E = rng.standard_normal(Y.shape)
    s = np.sqrt(np.sum(Y * Y) / (np.sum(E * E) * 10.0 ** (snr_db / 10.0)))
    return Y + s * E


# -------------------------------------------------------- method's randoms

def omegas(rng, dims, ranks_tilde):
    """Gaussian Omega_n, I_n x R~_n."""
    return [rng.standard_normal((I, r)) for I, r in zip(dims, ranks_tilde)]


def omega_tildes(rng, ranks_tilde):
    """Gaussian Omega~_n, (prod_{p != n} R~_p) x R~_n."""
    N = len(ranks_tilde)
    out = []
    for n in range(N):
        rows = int(np.prod([ranks_tilde[p] for p in range(N) if p != n]))
        out.append(rng.standard_normal((rows, ranks_tilde[n])))
    return out


def f32(x):
    """Round FP64 arrays to the FP32 values both sides consume."""
    if isinstance(x, list):
        return [np.ascontiguousarray(a, dtype=np.float32) for a in x]
    return np.ascontiguousarray(x, dtype=np.float32)


# ----------------------------------------------------------------- cases

def case_cp_gaussian(case, dims, R, snr_db, ranks_tilde, sweeps=1):
    """CP tensor with N(0,1) factors + Gaussian noise (Section V-A recipe)."""
    g = rngs(case)
    A = gaussian_factors(g["factors"], dims, R)
    Ystar = cp_tensor(A)
    Y = add_gaussian_noise(Ystar, g["noise"], snr_db)
    return _with_randoms(g, Y, Ystar, A, dims, ranks_tilde, sweeps)


def case_cp_congruent(case, dims, R, c_lo, c_hi, snr_db, ranks_tilde,
                      sweeps=1):
    g = rngs(case)
    A = congruent_factors(g["factors"], dims, R, c_lo, c_hi)
    Ystar = cp_tensor(A)
    Y = add_gaussian_noise(Ystar, g["noise"], snr_db)
    return _with_randoms(g, Y, Ystar, A, dims, ranks_tilde, sweeps)


def case_tucker(case, dims, ranks, snr_db, ranks_tilde, sweeps=1):
    """Tucker model: N(0,1) core, orthonormal random factors, noise."""
    g = rngs(case)
    G = g["factors"].standard_normal(tuple(ranks))
    U = orthonormal_factors(g["factors"], dims, ranks)
    Ystar = tucker_tensor(G, U)
    Y = add_gaussian_noise(Ystar, g["noise"], snr_db) if snr_db is not None \
        else Ystar
    d = _with_randoms(g, Y, Ystar, None, dims, ranks_tilde, sweeps)
    d["G_true"], d["U_true"] = G, U
    return d


def case_nonneg(case, dims, R, ranks_tilde, dist="uniform", scale=1.0,
                zero_frac=0.2, abs_noise_sigma=0.01, sweeps=2):
    """Nonnegative CP + |N(0, sigma)| noise."""
    g = rngs(case)
    A = nonneg_factors(g["factors"], dims, R, dist, scale, zero_frac)
    Ystar = cp_tensor(A)
    Y = Ystar + np.abs(g["noise"].normal(0.0, abs_noise_sigma, Ystar.shape))
    return _with_randoms(g, Y, Ystar, A, dims, ranks_tilde, sweeps)


def _with_randoms(g, Y, Ystar, A, dims, ranks_tilde, sweeps):
    om = omegas(g["omega"], dims, ranks_tilde)
    omt = [omega_tildes(g["omega_t1"], ranks_tilde)]
    if sweeps >= 2:
        omt.append(omega_tildes(g["omega_t2"], ranks_tilde))
    return {"Y": Y, "Ystar": Ystar, "A_true": A, "omegas": om,
            "omega_tildes": omt, "init_rng": g["init"]}


def init_factors(rng, dims, R, nonneg=False):
    """Random FFCP initial factors: U[0,1] for nonnegative fits, N(0,1)
    otherwise."""
    if nonneg:
        return [rng.uniform(0.0, 1.0, size=(I, R)) for I in dims]
    return [rng.standard_normal((I, R)) for I in dims]


def nonneg_tucker_format(case, dims, R, dist="exp", scale=10.0, zero_frac=0.2):
    """An exact Tucker format of a noise-free nonnegative CP model, for FFCP
    on tensors too large to form (Section V-A's 10^4 x 10^4 x 10^4 x 10^4
    example): true factors A_n (``nonneg_factors``), U_n R_n = A_n their
    reduced QR, core G = sum_r R_1[:, r] o ... o R_N[:, r] (R^N entries), and
    U[0,1] initial factors from the case's init stream."""
    g = rngs(case)
    A = nonneg_factors(g["factors"], dims, R, dist, scale, zero_frac)
    U, Rs = [], []
    for a in A:
        q, r = np.linalg.qr(a)
        U.append(q)
        Rs.append(r)
    letters = "abcdefghijklmnopq"[:len(dims)]
    G = np.einsum(",".join(c + "z" for c in letters) + "->" + letters, *Rs)
    A0 = init_factors(g["init"], dims, R, nonneg=True)
    return {"A": A, "U": U, "G": G, "A0": A0}


# ------------------------------------------------ device-resident workloads

def cp_congruent_device(case, dims, R, c_lo, c_hi, snr_db, ranks_tilde,
                        sweeps=1, device="cuda"):
    """Large CP workload built directly in device memory.

    Factors, Omega_n and Omega~_n come from the same seeded numpy streams as
    ``case_cp_congruent``; Y* = [[A_1, ..., A_N]] is formed in FP64 by torch
    (mode-1 unfolding times the transposed Khatri-Rao product of the other
    factors), Gaussian noise from torch's generator seeded with the case's
    noise stream is scaled to the exact SNR, and the sum is rounded once to
    FP32.  Returns Y (device float32), the factors and the method's randoms
    (host FP64)."""
    import torch
    g = rngs(case)
    A = congruent_factors(g["factors"], dims, R, c_lo, c_hi)
    om = omegas(g["omega"], dims, ranks_tilde)
    omt = [omega_tildes(g["omega_t1"], ranks_tilde)]
    if sweeps >= 2:
        omt.append(omega_tildes(g["omega_t2"], ranks_tilde))
    noise_seed = int(g["noise"].integers(0, 2**62))
    At = [torch.from_numpy(a).to(device) for a in A]
    kr = At[-1]
    for a in reversed(At[1:-1]):   # rows: (i_2, ..., i_N) row-major
        kr = (a[:, None, :] * kr[None, :, :]).reshape(-1, R)
    Ystar = At[0] @ kr.T           # I_1 x prod_{n>1} I_n, FP64
    del kr
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    E = torch.randn(Ystar.shape, dtype=torch.float64, device=device,
                    generator=gen)
    s = torch.sqrt(torch.sum(Ystar * Ystar) /
                   (torch.sum(E * E) * 10.0 ** (snr_db / 10.0)))
    E.mul_(s).add_(Ystar)
    del Ystar
    Y = E.to(torch.float32).reshape(tuple(dims))
    del E
    return {"Y": Y, "A_true": A, "omegas": om, "omega_tildes": omt,
            "init_rng": g["init"]}


def nonneg_cp_device(case, dims, R, ranks_tilde, zero_frac=0.2, noise_sigma=0.01,
                     sweeps=2, device="cuda"):
    """The nonnegative CP workload of ``case_nonneg`` (U[0,1] factors with
    exactly ``zero_frac`` zeros, |N(0, sigma)| noise) built in device memory:
    factors and the method's randoms from the same seeded numpy streams;
    Y* = [[A_1, ..., A_N]] formed in FP64 by torch (mode-1 unfolding times the
    transposed Khatri-Rao product of the other factors); the noise from
    torch's generator seeded with the case's noise stream; the sum rounded
    once to FP32."""
    import torch
    g = rngs(case)
    A = nonneg_factors(g["factors"], dims, R, "uniform", 1.0, zero_frac)
    om = omegas(g["omega"], dims, ranks_tilde)
    omt = [omega_tildes(g["omega_t1"], ranks_tilde)]
    if sweeps >= 2:
        omt.append(omega_tildes(g["omega_t2"], ranks_tilde))
    noise_seed = int(g["noise"].integers(0, 2**62))
    At = [torch.from_numpy(a).to(device) for a in A]
    kr = At[-1]
    for a in reversed(At[1:-1]):   # rows: (i_2, ..., i_N) row-major
        kr = (a[:, None, :] * kr[None, :, :]).reshape(-1, R)
    Y = At[0] @ kr.T               # I_1 x prod_{n>1} I_n, FP64
    del kr
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    for r0 in range(0, Y.shape[0], 16):   # |N(0, sigma)| added in row blocks
        blk = Y[r0:r0 + 16]
        blk.add_(torch.randn(blk.shape, dtype=torch.float64, device=device,
                             generator=gen).abs_().mul_(noise_sigma))
    Y32 = Y.to(torch.float32).reshape(tuple(dims))
    del Y
    return {"Y": Y32, "A_true": A, "omegas": om, "omega_tildes": omt,
            "init_rng": g["init"]}


def tucker_device(case, dims, ranks, snr_db, ranks_tilde, sweeps=2, device="cuda"):
    """The Tucker-model workload of ``case_tucker`` (N(0,1) core, orthonormal
    random factors, Gaussian noise at an exact SNR) built in device memory:
    core, factors and the method's randoms from the same seeded numpy
    streams; Y* = G x_1 U_1 ... x_N U_N formed in FP64 by torch, one mode
    product at a time (mode-n unfolding times U_n^T); the noise from torch's
    generator seeded with the case's noise stream and scaled to the exact
    SNR; the sum rounded once to FP32."""
    import torch
    g = rngs(case)
    G = g["factors"].standard_normal(tuple(ranks))
    U = orthonormal_factors(g["factors"], dims, ranks)
    om = omegas(g["omega"], dims, ranks_tilde)
    omt = [omega_tildes(g["omega_t1"], ranks_tilde)]
    if sweeps >= 2:
        omt.append(omega_tildes(g["omega_t2"], ranks_tilde))
    noise_seed = int(g["noise"].integers(0, 2**62))
    X = torch.from_numpy(G).to(device)
    for n, u in enumerate(U):
        Ut = torch.from_numpy(u).to(device)                   # I_n x R_n
        X = torch.movedim(torch.tensordot(X, Ut, dims=([n], [1])), -1, n).contiguous()
    gen = torch.Generator(device=device)
    gen.manual_seed(noise_seed)
    Xf = X.reshape(X.shape[0], -1)
    e2 = 0.0
    for r0 in range(0, Xf.shape[0], 8):        # the noise's norm, then its scale
        e2 += float(torch.randn(Xf[r0:r0 + 8].shape, dtype=torch.float64, device=device,
                                generator=gen).pow_(2).sum())
    s = (float((Xf * Xf).sum()) / (e2 * 10.0 ** (snr_db / 10.0))) ** 0.5
    gen.manual_seed(noise_seed)
    for r0 in range(0, Xf.shape[0], 8):        # the same noise again, added
        blk = Xf[r0:r0 + 8]
        blk.add_(torch.randn(blk.shape, dtype=torch.float64, device=device,
                             generator=gen).mul_(s))
    Y32 = X.to(torch.float32)
    del X, Xf
    return {"Y": Y32, "G_true": G, "U_true": U, "omegas": om, "omega_tildes": omt,
            "init_rng": g["init"]}


def mlp_weights(case, dims):
    """He-initialized weights of the learned initializer: W_l ~ N(0, 2/fan_in)
    (d_l x d_{l+1}), zero biases; FP32 values (returned as float32 arrays)."""
    rng = rngs(case)["init"]
    W, b = [], []
    for l in range(len(dims) - 1):
        W.append((rng.standard_normal((dims[l], dims[l + 1])) *
                  np.sqrt(2.0 / dims[l])).astype(np.float32))
        b.append(np.zeros(dims[l + 1], dtype=np.float32))
    return W, b
