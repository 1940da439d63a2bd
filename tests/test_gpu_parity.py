"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs (FP32 values promoted exactly to FP64 for the oracle).

Tolerances: FP64 path at the level of FP64 rounding; FP32 path at the level
of FP32 accumulation over the contraction lengths used here (a few hundred
to a few thousand terms): relative 1e-5 on sketches, 1e-4 on subspaces and
aligned cores (the truncation divides by eigen-gaps of O(1) relative size).
FFCP runs in FP64 on the device from the same FP32 U, G and initial A, so its
iterates match the oracle's to 1e-9.
"""

import zlib

import numpy as np
import pytest

import synth
from oracle import ffcp as F
from oracle import randtucker as RT
from oracle import tensor as T
from oracle.metrics import aligned_core_error, projector_distance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    """Element-wise error over scale: max |a - b| / max |b|.  Unlike the
    Frobenius ratio it cannot hide one wrong entry among many right ones."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def seed_of(*key):
    """A fixed 32-bit seed for a test case (string hashes are salted per
    process, so hash() would draw new data on every run)."""
    return zlib.crc32(repr(key).encode())


# ------------------------------------------------------------------ TTM

@pytest.mark.parametrize("shape", [(37, 41, 43), (9, 10, 11, 12), (300, 2, 5)])
@pytest.mark.parametrize("K", [5, 30])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ttm_parity(P, shape, K, dtype):
    g = np.random.default_rng(seed_of("ttm", shape, K))
    Y = g.standard_normal(shape)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    tol = 2e-6 if dtype == "f32" else 1e-13
    Yf = Y.astype(np.float32).astype(np.float64) if dtype == "f32" else Y
    for n in range(len(shape)):
        M = g.standard_normal((shape[n], K))
        Mf = M.astype(np.float32).astype(np.float64) if dtype == "f32" else M
        out = P.ttm(dev(Yf, tdt), dev(Mf, tdt), n)
        ref = T.ttm_t(Yf, Mf, n)
        assert rel(host(out), ref) <= tol
        assert maxrel(host(out), ref) <= tol


# ------------------------------------------------------------ tucker_rand

def run_tucker(P, d, ranks, sweeps, precision="f32", truncate=True, order="jacobi"):
    tdt = torch.float64 if precision == "f64" else torch.float32
    cast = (lambda a: a) if precision == "f64" else synth.f32
    Y = cast(d["Y"])
    om = [cast(o) for o in d["omegas"]]
    omt = [[cast(o) for o in lst] for lst in d["omega_tildes"][:sweeps]]
    out = P.tucker_rand(dev(Y, tdt), [dev(o, tdt) for o in om],
                        [[dev(o, tdt) for o in lst] for lst in omt],
                        ranks=ranks, sweeps=sweeps, precision=precision,
                        truncate=truncate, trace=True, order=order)
    ref = RT.rand_tucker(np.asarray(Y, np.float64), [np.asarray(o, np.float64) for o in om],
                         [[np.asarray(o, np.float64) for o in lst] for lst in omt],
                         sweeps=sweeps, ranks=ranks if truncate else None, order=order)
    return out, ref, np.asarray(Y, np.float64)


def check_tucker(out, ref, Y, N, sweeps, tol_z, tol_u, tol_g):
    for s in range(sweeps):
        for n in range(N):
            z = host(out["trace"]["Z"][s * N + n])
            zr = ref["Z"][s][n]
            assert rel(z, zr) <= tol_z, ("Z", s, n)
            assert maxrel(z, zr) <= tol_z, ("Z element-wise", s, n)
            q = host(out["trace"]["Q"][s * N + n])
            # range(Z) moves by at most ||dZ||_2 / (s_min(Z) - ||dZ||_2) (Wedin);
            # the trailing sketch directions are noise with small s_min, so the
            # full-width basis is compared against that bound, not a constant.
            dz = np.linalg.norm(z - zr, 2)
            smin = np.linalg.svd(zr, compute_uv=False).min()
            bound = 2.0 * dz / max(smin - dz, 1e-300) + 1e-6
            assert projector_distance(q, ref["Q_sweeps"][s][n]) <= bound, ("Q", s, n)
            assert np.linalg.norm(q.T @ q - np.eye(q.shape[1])) <= 10 * tol_z
    for n in range(N):
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= tol_u, ("U", n)
    eG = aligned_core_error(host(out["G"]), [host(u) for u in out["U"]],
                            ref["G"], ref["U"])
    assert eG <= tol_g
    info = out["info"]
    assert abs(info["normY2"] - np.sum(Y * Y)) <= 1e-6 * np.sum(Y * Y)
    assert info["nonfinite"] == 0


def test_tucker_c1_fp64(P):
    """100^3 CP rank 10 + noise at 40 dB, Omega_n 100 x 15, ranks (10,10,10):
    the plain method in FP64 end to end."""
    d = synth.case_cp_gaussian(1, (100, 100, 100), 10, 40.0, (15, 15, 15))
    out, ref, Y = run_tucker(P, d, (10, 10, 10), 1, "f64")
    check_tucker(out, ref, Y, 3, 1, 1e-12, 1e-10, 1e-10)


@pytest.mark.parametrize("sweeps", [1, 2])
def test_tucker_fp32_3way_ragged(P, sweeps):
    d = synth.case_tucker(301, (64, 72, 81), (6, 7, 8), 20.0, (12, 13, 14), sweeps=2)
    out, ref, Y = run_tucker(P, d, (6, 7, 8), sweeps, "f32")
    check_tucker(out, ref, Y, 3, sweeps, 1e-5, 1e-4, 1e-4)


@pytest.mark.parametrize("dims", [(9, 70, 260), (5, 50, 1000), (12, 61, 200),
                                  (20, 33, 100), (7, 3, 36)])
def test_tucker_fp32_mfma_streaming_shapes(P, dims):
    """Shapes that exercise the MFMA streaming pass: last dimension a
    multiple of 4 but not of 32 (ragged column tile), I_{N-1} not a multiple
    of 32 (ragged row chunk), and 1, 2, 4 or 8 wavefronts sharing a slab."""
    rt = tuple(min(12, d) for d in dims)
    ranks = tuple(min(3, r) for r in rt)   # truncate to the signal's ranks
    d = synth.case_tucker(305 + dims[2], dims, ranks, 30.0, rt, sweeps=2)
    out, ref, Y = run_tucker(P, d, ranks, 2, "f32")
    check_tucker(out, ref, Y, 3, 2, 1e-5, 2e-4, 2e-4)


@pytest.mark.parametrize("dims,rt", [((40, 45, 52), (20, 24, 17)),    # one workgroup, K > 16
                                     ((4100, 6, 8), (10, 6, 8)),      # I_n > 4096: row chunks
                                     ((50, 60, 64), (40, 12, 12))])   # K > 32: row chunks
def test_tucker_fp32_qr_forms(P, dims, rt):
    """The sketch bases come from the one-workgroup CholeskyQR2 for sketches
    of at most 4096 rows and 32 columns and from the row-chunked form
    otherwise; both match the oracle's Householder bases."""
    ranks = tuple(min(4, r) for r in rt)
    d = synth.case_tucker(307 + dims[0], dims, ranks, 30.0, rt, sweeps=2)
    out, ref, Y = run_tucker(P, d, ranks, 2, "f32")
    check_tucker(out, ref, Y, 3, 2, 1e-5, 2e-4, 2e-4)


def test_tucker_fp32_4way(P):
    d = synth.case_tucker(302, (18, 20, 22, 24), (4, 5, 6, 7), 30.0, (6, 7, 8, 9),
                          sweeps=2)
    out, ref, Y = run_tucker(P, d, (4, 5, 6, 7), 2, "f32")
    check_tucker(out, ref, Y, 4, 2, 1e-5, 1e-4, 1e-4)


def test_tucker_no_truncate(P):
    d = synth.case_tucker(303, (30, 31, 32), (4, 4, 4), 30.0, (7, 8, 9))
    out, ref, Y = run_tucker(P, d, None, 1, "f32", truncate=False)
    for n in range(3):
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= 1e-4
    assert aligned_core_error(host(out["G"]), [host(u) for u in out["U"]],
                              ref["G"], ref["U"]) <= 1e-4


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_tucker_rank_deficient_sketch(P, precision):
    """Noise-free Tucker tensor of multilinear rank 3 sketched with 8 columns:
    the sketch Gram matrices are singular, CholeskyQR2 rejects them and the
    Householder fallback forms the bases.  The signal subspace, the truncated
    factors and the core still match the oracle; every basis is orthonormal."""
    d = synth.case_tucker(306, (40, 44, 48), (3, 3, 3), None, (8, 8, 8))
    out, ref, Y = run_tucker(P, d, (3, 3, 3), 1, precision)
    tol = 1e-4 if precision == "f32" else 1e-10
    for n in range(3):
        q = host(out["trace"]["Q"][n])
        assert np.linalg.norm(q.T @ q - np.eye(8)) <= 10 * tol
        # the signal part of range(Q) is the oracle's
        us = T.unfold(d["Y"], n)
        u_sig = np.linalg.svd(us, full_matrices=False)[0][:, :3]
        assert np.linalg.norm(u_sig - q @ (q.T @ u_sig)) <= tol
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= tol
    assert aligned_core_error(host(out["G"]), [host(u) for u in out["U"]],
                              ref["G"], ref["U"]) <= tol


# ------------------------------------------------- Gauss-Seidel sweep order

def test_tucker_gauss_seidel_c1_fp64(P):
    """The loop of Algorithm 3 as printed (mode n's sketch uses the bases
    modes < n received in the same sweep) on the 100^3 FP64 workload, two
    sweeps, against the oracle's order="gauss_seidel"."""
    d = synth.case_cp_gaussian(1, (100, 100, 100), 10, 40.0, (15, 15, 15), sweeps=2)
    out, ref, Y = run_tucker(P, d, (10, 10, 10), 2, "f64", order="gauss_seidel")
    check_tucker(out, ref, Y, 3, 2, 1e-12, 1e-10, 1e-10)


@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("dims,ranks,rt", [((64, 72, 81), (6, 7, 8), (12, 13, 14)),
                                           ((18, 20, 22, 24), (4, 5, 6, 7), (6, 7, 8, 9)),
                                           ((9, 70, 260), (3, 3, 3), (9, 12, 12))])
def test_tucker_gauss_seidel_fp32(P, sweeps, dims, ranks, rt):
    """Every sketch but the first reads bases the device computed earlier in
    the sweep, so its input differs from the oracle's by FP32 rounding
    amplified through the trailing (noise) directions of those bases: each
    sketch is checked, element-wise at 1e-5, against the oracle's sketch
    step applied to the bases the device returned for the same point of the
    loop (the Gauss-Seidel dependence written out here); the first sketch of
    the first sweep, and the final bases and core, against the oracle run."""
    d = synth.case_tucker(seed_of("gs", dims), dims, ranks, 25.0, rt, sweeps=2)
    out, ref, Y = run_tucker(P, d, ranks, sweeps, "f32", order="gauss_seidel")
    N = len(dims)
    om = [synth.f32(o).astype(np.float64) for o in d["omegas"]]
    omt = [[synth.f32(o).astype(np.float64) for o in lst] for lst in d["omega_tildes"]]
    Qs = [[host(out["trace"]["Q"][s * N + n]) for n in range(N)] for s in range(sweeps)]
    assert maxrel(host(out["trace"]["Z"][0]), ref["Z"][0][0]) <= 1e-5
    for s in range(sweeps):
        prev = om if s == 0 else Qs[s - 1]
        for n in range(N):
            bases = [Qs[s][p] if p < n else prev[p] for p in range(N)]
            want = RT.sketch(Y, bases, omt[s][n], n)
            e = maxrel(host(out["trace"]["Z"][s * N + n]), want)
            assert e <= 1e-5, ("Z", s, n, e)
            q = Qs[s][n]
            assert np.linalg.norm(q.T @ q - np.eye(q.shape[1])) <= 1e-4
    for n in range(N):
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= 2e-4, ("U", n)
    eG = aligned_core_error(host(out["G"]), [host(u) for u in out["U"]], ref["G"], ref["U"])
    assert eG <= 2e-4


def test_gauss_seidel_differs_from_jacobi_after_the_first_mode(P):
    """In the first sweep both orders sketch mode 1 from the same Gaussian
    bases (identical sketches); every later mode sees the updated bases in
    the Gauss-Seidel order only."""
    d = synth.case_tucker(309, (30, 34, 36), (4, 4, 4), 30.0, (8, 8, 8), sweeps=1)
    a, _, _ = run_tucker(P, d, (4, 4, 4), 1, "f32", order="jacobi")
    b, _, _ = run_tucker(P, d, (4, 4, 4), 1, "f32", order="gauss_seidel")
    assert torch.equal(a["trace"]["Z"][0], b["trace"]["Z"][0])
    for n in (1, 2):
        assert rel(host(b["trace"]["Z"][n]), host(a["trace"]["Z"][n])) > 1e-2


@pytest.mark.parametrize("sweeps", [1, 2])
def test_tucker_gauss_seidel_bf16_vs_fp64_oracle(P, sweeps):
    """The precision form in the Gauss-Seidel order against the FP64 oracle
    in that order on the unrounded tensor: each subspace within
    4 2^-9 ||Y|| / gap_n (the BF16 rounding of Y, Wedin)."""
    dims, R, rt = (40, 120, 96), (5, 5, 5), (12, 12, 12)
    d = synth.case_tucker(413, dims, R, 30.0, rt, sweeps=2)
    out, ref, Y = run_tucker(P, d, R, sweeps, "bf16", order="gauss_seidel")
    nY = np.linalg.norm(Y)
    for n in range(3):
        sv = np.linalg.svd(T.unfold(Y, n), compute_uv=False)
        bound = 4 * 2.0 ** -9 * nY / (sv[R[n] - 1] - sv[R[n]])
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= bound, n
    eG = aligned_core_error(host(out["G"]), [host(u) for u in out["U"]], ref["G"], ref["U"])
    assert eG <= 4 * 2.0 ** -9 * nY / np.linalg.norm(ref["G"]) + 1e-4


@pytest.mark.parametrize("dims", [(20, 21, 24), (6, 40, 520)])
@pytest.mark.parametrize("precision", ["f32", "bf16"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_tucker_nonfinite_flag(P, precision, bad, dims):
    """A NaN or Inf anywhere in Y sets the info flag (both streaming forms,
    narrow and wide slabs) and the Python wrapper raises."""
    d = synth.case_tucker(304, dims, (3, 3, 3), 30.0, (5, 5, 5))
    Y = synth.f32(d["Y"]).copy()
    Y[min(3, dims[0] - 1), 4, 5] = bad
    args = (dev(Y), [dev(synth.f32(o)) for o in d["omegas"]],
            [[dev(synth.f32(o)) for o in d["omega_tildes"][0]]])
    out = P.tucker_rand(*args, ranks=(3, 3, 3), sweeps=1, precision=precision,
                        check_finite=False)
    assert out["info"]["nonfinite"] == 1
    with pytest.raises(P.NonFiniteInput):
        P.tucker_rand(*args, ranks=(3, 3, 3), sweeps=1, precision=precision)


@pytest.mark.parametrize("dims", [(6, 20, 24), (6, 20, 520)])
@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_tucker_largest_finite_values_are_finite(P, precision, dims):
    """Values of magnitude FLT_MAX are finite: no flag, and ||Y||^2 is the
    FP64 sum of squares (FLT_MAX^2 ~ 1.2e77 is an ordinary FP64 number).
    In the precision form that slab is scaled by 2^-127 before rounding."""
    d = synth.case_tucker(308, dims, (3, 3, 3), 30.0, (5, 5, 5))
    Y = synth.f32(d["Y"]).copy()
    fmax = np.finfo(np.float32).max
    Y[2, 4, 5] = fmax
    Y[2, 7, 9] = -fmax
    out = P.tucker_rand(dev(Y), [dev(synth.f32(o)) for o in d["omegas"]],
                        [[dev(synth.f32(o)) for o in d["omega_tildes"][0]]],
                        ranks=(3, 3, 3), sweeps=1, precision=precision)
    assert out["info"]["nonfinite"] == 0
    Y64 = Y.astype(np.float64)
    n2 = float(np.sum(Y64 * Y64))
    assert np.isfinite(out["info"]["normY2"])
    assert abs(out["info"]["normY2"] - n2) <= 1e-6 * n2


# ------------------------------------------------------------------ FFCP

def _tucker_format(seed, dims, ranks, nonneg=False, with_factors=False):
    """Random Tucker format.  nonneg=True builds the exact Tucker format of a
    nonnegative CP tensor (U_n = orth(A_n), G = I x_n R_n, the construction
    of Section V-A), so nonnegative updates face a well-posed problem."""
    g = np.random.default_rng(seed)
    A = None
    if nonneg:
        Rt = ranks[0]
        A = [g.uniform(0, 1, (I, Rt)) for I in dims]
        U, Rs = [], []
        for a in A:
            q, r = np.linalg.qr(a)
            U.append(q)
            Rs.append(r)
        G = np.zeros((Rt,) * len(dims))
        for r in range(Rt):
            G[(r,) * len(dims)] = 1.0
        G = T.multi_ttm_t(G, [r_.T for r_ in Rs])
    else:
        G = g.standard_normal(ranks)
        U = [np.linalg.qr(g.standard_normal((I, r)))[0] for I, r in zip(dims, ranks)]
    out = (synth.f32(G).astype(np.float64), [synth.f32(u).astype(np.float64) for u in U], g)
    return out + (A,) if with_factors else out


# Cases for the iterate parity.  Small R runs the per-group cross products of
# the general kernel; R = R_n = 15 its per-thread branch (R_n R + R^2 >= 256);
# R = 20 and 40 the 32- and 64-column instantiations.  ALS on three-way cores
# with R and R_n <= 20 runs the three-way kernel, zero-padded to 8, 16 or 20
# (ranks that differ from each other and from R pad differently); ALS in four
# modes and at R = 24, 32 and 48 runs the general kernel (the 48^3 core read
# from global memory).  Every case was checked on the CPU
# to be well posed for 12 iterations: a 1e-13 relative change of the start
# moves the oracle's fits by < 1e-13 and its factors by < 1e-11.  For HALS at
# R = 40 that needs a start near the solution (the true factors times
# U[0.5, 1.5] entries): from a U[0, 1] start the first update zeroes whole
# columns, and renormalizing their rounding residue makes the run chaotic.
ITERATE_CASES = [
    ("als", (50, 60, 70), (6, 7, 8), 5, "random"),
    ("als", (30, 31, 32, 33), (4, 5, 4, 5), 3, "random"),
    ("als", (40, 44, 48), (12, 14, 16), 13, "random"),
    ("als", (40, 44, 48), (20, 18, 19), 17, "random"),
    ("als", (40, 44, 48), (24, 24, 24), 24, "random"),
    ("als", (40, 44, 48), (32, 32, 32), 32, "random"),
    ("als", (56, 60, 64), (48, 48, 48), 48, "random"),
    ("hals", (50, 60, 70), (6, 6, 6), 5, "random"),
    ("hals", (30, 31, 32, 33), (4, 4, 4, 4), 3, "random"),
    ("hals", (40, 44, 48), (15, 15, 15), 15, "near"),
    ("hals", (40, 44, 48), (20, 20, 20), 20, "near"),
    ("hals", (64, 70, 72), (40, 40, 40), 40, "near"),
    ("mu", (50, 60, 70), (6, 6, 6), 5, "random"),
    ("mu", (30, 31, 32, 33), (4, 4, 4, 4), 3, "random"),
    ("mu", (40, 44, 48), (15, 15, 15), 15, "near"),
    ("mu", (40, 44, 48), (20, 20, 20), 20, "near"),
    ("mu", (64, 70, 72), (40, 40, 40), 40, "near"),
]


def _iterate_case(rule, dims, ranks, R, start):
    nonneg = rule != "als"
    G, U, g, A = _tucker_format(seed_of(rule, dims, R), dims, ranks, nonneg,
                                with_factors=True)
    if start == "near":
        A0 = [a * g.uniform(0.5, 1.5, a.shape) for a in A]
    else:
        A0 = [g.uniform(0, 1, (I, R)) if nonneg else g.standard_normal((I, R))
              for I in dims]
    return G, U, [synth.f32(a).astype(np.float64) for a in A0]


def _check_iterates(P, rule, G, U, A0, R, iters=12, l1=0.0):
    out = P.ffcp([dev(u) for u in U], dev(G), R, update=rule,
                 A_init=[dev(a) for a in A0], max_it=iters, tol=0.0, l1=l1,
                 fit_trace=True)
    ref = F.ffcp(U, G, A0, update=rule, max_it=iters, tol=0.0, l1=l1)
    assert int(out["info"]["iterations"]) == iters
    np.testing.assert_allclose(out["fits"], ref["fits"], rtol=0, atol=1e-9)
    for n in range(len(U)):
        a = host(out["A"][n])
        assert rel(a, ref["A"][n]) <= 1e-6          # FP32 output
        assert maxrel(a, ref["A"][n]) <= 1e-6
    assert maxrel(host(out["lam"]), ref["lam"]) <= 1e-6
    assert int(out["info"]["ridged"]) == int(ref["ridged"])
    return out, ref


@pytest.mark.parametrize("rule,dims,ranks,R,start", ITERATE_CASES,
                         ids=[f"{c[0]}-R{c[3]}-{len(c[1])}way" for c in ITERATE_CASES])
def test_ffcp_iterates(P, rule, dims, ranks, R, start):
    G, U, A0 = _iterate_case(rule, dims, ranks, R, start)
    _check_iterates(P, rule, G, U, A0, R)


# l1 cases: the Tucker format of a CP tensor with a start near its factors
# (a run from a random start on a random core zeroes whole columns and ends
# in the ridge), at levels where entries are shrunk to zero (to the floor
# under HALS) in every iteration but no column vanishes; checked on the CPU
# with the oracle, which also confirms that a 1e-13 change of the start moves
# the fits by < 1e-12
L1_CASES = [("als", (50, 60, 70), 5, 0.02),
            ("als", (40, 44, 48), 20, 0.01),
            ("hals", (50, 60, 70), 5, 0.01),
            ("hals", (40, 44, 48), 20, 0.005),
            ("mu", (50, 60, 70), 5, 0.005)]


@pytest.mark.parametrize("rule,dims,R,c", L1_CASES,
                         ids=[f"{c[0]}-R{c[2]}-c{c[3]}" for c in L1_CASES])
def test_ffcp_l1_iterates(P, rule, dims, R, c):
    """The sparsity step S_c of eq. (16) after each update (with the HALS
    floor re-applied under HALS): fits 1e-9, factors 1e-6 element-wise."""
    G, U, g, A = _tucker_format(seed_of("l1", rule, dims, R), dims, (R,) * len(dims),
                                True, with_factors=True)
    A0 = [synth.f32(a * g.uniform(0.5, 1.5, a.shape)).astype(np.float64) for a in A]
    out, ref = _check_iterates(P, rule, G, U, A0, R, iters=12, l1=c)
    assert not ref["ridged"]
    small = sum(int(np.sum(np.abs(a) <= 1e-16)) for a in ref["A"])
    assert small > 0            # the threshold did act


def test_ffcp_convergence_matches_oracle(P):
    d = synth.case_cp_gaussian(2, (60, 61, 62), 4, 30.0, (8, 8, 8))
    tk = RT.rand_tucker(synth.f32(d["Y"]).astype(np.float64), d["omegas"],
                        d["omega_tildes"], sweeps=1, ranks=(6, 6, 6))
    U = [synth.f32(u).astype(np.float64) for u in tk["U"]]
    G = synth.f32(tk["G"]).astype(np.float64)
    A0 = [synth.f32(a).astype(np.float64)
          for a in synth.init_factors(d["init_rng"], (60, 61, 62), 4)]
    out = P.ffcp([dev(u) for u in U], dev(G), 4, update="als",
                 A_init=[dev(a) for a in A0], max_it=500, tol=1e-9, fit_trace=True)
    ref = F.ffcp(U, G, A0, update="als", max_it=500, tol=1e-9)
    assert abs(int(out["info"]["iterations"]) - ref["iterations"]) <= 2
    assert abs(out["info"]["fit"] - ref["fits"][-1]) <= 1e-8
    assert out["info"]["converged"] == int(ref["converged"])


def test_ffcp_hosvd_init_with_padding(P):
    G, U, g = _tucker_format(77, (40, 41, 42), (5, 6, 4))
    R = 6
    pad = [synth.f32(g.standard_normal((r, R - r))).astype(np.float64) if R > r else None
           for r in (5, 6, 4)]
    out = P.ffcp([dev(u) for u in U], dev(G), R, update="als", init="hosvd",
                 pad=[dev(p) if p is not None else None for p in pad],
                 max_it=3, tol=0.0, fit_trace=True)
    A0 = F.hosvd_init(U, G, R, pad=pad)
    ref = F.ffcp(U, G, A0, update="als", max_it=3, tol=0.0)
    np.testing.assert_allclose(out["fits"], ref["fits"], rtol=0, atol=1e-9)
    for n in range(3):
        assert rel(host(out["A"][n]), ref["A"][n]) <= 1e-6


def test_ffcp_coefficient_start(P):
    """init="coeff": A_n = U_n V_n from caller coefficients, iterates equal to
    the oracle started from A_n = U_n V_n."""
    G, U, g = _tucker_format(81, (40, 41, 42), (5, 6, 4))
    R = 4
    V = [synth.f32(g.standard_normal((r, R))).astype(np.float64) for r in (5, 6, 4)]
    out = P.ffcp([dev(u) for u in U], dev(G), R, update="als", init="coeff",
                 A_init=[dev(v) for v in V], max_it=8, tol=0.0, fit_trace=True)
    ref = F.ffcp(U, G, [u @ v for u, v in zip(U, V)], update="als", max_it=8, tol=0.0)
    np.testing.assert_allclose(out["fits"], ref["fits"], rtol=0, atol=1e-9)
    for n in range(3):
        assert rel(host(out["A"][n]), ref["A"][n]) <= 1e-6


@pytest.mark.parametrize("good", [True, False])
def test_ffcp_guarded_start(P, good):
    """init="coeff_guarded" keeps the caller's start only when its initial fit
    is at least the HOSVD start's: a near-exact start is kept, a poor one is
    replaced, and the run then equals the oracle from the chosen start."""
    dims, R = (30, 31, 32), 4
    rng = np.random.default_rng(82)
    A = [rng.standard_normal((I, R)) for I in dims]
    Y = T.kruskal_full(A)
    ref_t = RT.rand_tucker(Y, [rng.standard_normal((I, 6)) for I in dims],
                           [[rng.standard_normal((36, 6)) for _ in dims]], ranks=(4, 4, 4))
    U = [synth.f32(u).astype(np.float64) for u in ref_t["U"]]
    G = synth.f32(ref_t["G"]).astype(np.float64)
    if good:   # the compressed true factors, slightly perturbed
        V = [u.T @ a + 1e-3 * rng.standard_normal((4, R)) for u, a in zip(U, A)]
    else:      # an unrelated start
        V = [rng.standard_normal((4, R)) for _ in dims]
    V = [synth.f32(v).astype(np.float64) for v in V]
    out = P.ffcp([dev(u) for u in U], dev(G), R, update="als", init="coeff_guarded",
                 A_init=[dev(v) for v in V], max_it=5, tol=0.0, fit_trace=True)
    A_user = [u @ v for u, v in zip(U, V)]
    A_hosvd = F.hosvd_init(U, G, R)
    assert out["info"]["init_used"] == (1 if good else 0)
    start = A_user if good else A_hosvd
    ref = F.ffcp(U, G, start, update="als", max_it=5, tol=0.0)
    # near an exact fit the closed form 1 - sqrt(||Yt||^2 - 2<Yt,Yhat> +
    # ||Yhat||^2)/||Yt|| cancels: an FP64 rounding of the bracket moves the
    # fit by about sqrt(eps) ~ 1e-8, so the good start is compared at 1e-7
    np.testing.assert_allclose(out["fits"], ref["fits"], rtol=0,
                               atol=1e-7 if good else 1e-9)


def test_ffcp_ridge_flag(P):
    G, U, g = _tucker_format(78, (20, 21, 22), (3, 3, 3))
    A0 = [g.standard_normal((I, 3)) for I in (20, 21, 22)]
    A0[1][:, 2] = 0.0
    A0[2][:, 2] = 0.0
    out = P.ffcp([dev(u) for u in U], dev(G), 3, update="als",
                 A_init=[dev(a) for a in A0], max_it=3, tol=0.0)
    ref = F.ffcp(U, G, A0, update="als", max_it=3, tol=0.0)
    assert out["info"]["ridged"] == 1 and ref["ridged"]
    for n in range(3):
        assert np.all(np.isfinite(host(out["A"][n])))


def test_cp_fit_dense(P):
    d = synth.case_cp_gaussian(3, (30, 40, 50), 5, 20.0, (6, 6, 6))
    Y = synth.f32(d["Y"]).astype(np.float64)
    A = [synth.f32(a).astype(np.float64) for a in d["A_true"]]
    lam = np.array([1.0, 0.5, 2.0, 1.5, 0.25], dtype=np.float32).astype(np.float64)
    fit, y2, inner = P.cp_fit_dense(dev(Y), [dev(a) for a in A], dev(lam))
    assert abs(fit - F.cp_fit_mttkrp(Y, A, lam)) <= 1e-6
    assert abs(y2 - np.sum(Y * Y)) <= 1e-9 * np.sum(Y * Y)


# ----------------------------------------------------- streamed pass itself

@pytest.mark.parametrize("shape", [(1, 32, 32), (3, 70, 260), (2, 50, 1000), (5, 61, 200),
                                   (4, 33, 100), (6, 3, 36), (2, 40, 96), (3, 17, 44)])
@pytest.mark.parametrize("K", [(30, 30), (12, 7), (25, 32)])
def test_stream_pass_parity(P, shape, K):
    g = np.random.default_rng(sum(shape) + K[0])
    Y = synth.f32(g.standard_normal(shape)).astype(np.float64)
    B2 = synth.f32(g.standard_normal((shape[2], K[0]))).astype(np.float64)
    B1 = synth.f32(g.standard_normal((shape[1], K[1]))).astype(np.float64)
    TA, TB, n2 = P.stream_pass(dev(Y), dev(B2), dev(B1))
    for got, want in ((TA, T.ttm_t(Y, B2, 2)), (TB, T.ttm_t(Y, B1, 1))):
        assert rel(host(got), want) <= 2e-6
        assert maxrel(host(got), want) <= 2e-6
    # squares are summed in FP64 (each square of an FP32 value is exact)
    assert abs(n2 - np.sum(Y * Y)) <= 1e-12 * np.sum(Y * Y)
    TA2, TB2, _ = P.stream_pass(dev(Y), dev(B2))
    assert TB2 is None
    assert rel(host(TA2), T.ttm_t(Y, B2, 2)) <= 2e-6


# ------------------------------------------------------------- ffcp_dense

@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_ffcp_dense_is_tucker_then_ffcp(P, precision):
    """rt_ffcp_dense (Algorithm 1 with input Y) runs the same kernels on the
    same values as rt_tucker_rand followed by rt_ffcp, so its factors,
    weights and fit trace are bit-identical to the two calls'; in FP32 its
    fit trace also follows the oracle's (RandTucker2i, then FFCP from the
    HOSVD start of the oracle's core) to FP32 rounding of the format."""
    dims, R, rk, rt = (40, 44, 48), 4, (6, 6, 6), (8, 8, 8)
    d = synth.case_cp_gaussian(seed_of("dense", precision), dims, R, 30.0, rt, sweeps=2)
    Y = synth.f32(d["Y"])
    om = [dev(synth.f32(o)) for o in d["omegas"]]
    omt = [[dev(synth.f32(o)) for o in lst] for lst in d["omega_tildes"]]
    kw = dict(update="als", init="hosvd", max_it=40, tol=0.0, fit_trace=True)
    one = P.ffcp_dense(dev(Y), om, omt, R, ranks=rk, sweeps=2, precision=precision, **kw)
    t = P.tucker_rand(dev(Y), om, omt, ranks=rk, sweeps=2, precision=precision)
    two = P.ffcp(t["U"], t["G"], R, **kw)
    for n in range(3):
        assert torch.equal(one["A"][n], two["A"][n]), n
    assert torch.equal(one["lam"], two["lam"])
    assert np.array_equal(one["fits"], two["fits"])
    assert one["tucker_info"]["normY2"] == t["info"]["normY2"]
    if precision == "f32":
        ref_t = RT.rand_tucker(Y.astype(np.float64),
                               [synth.f32(o).astype(np.float64) for o in d["omegas"]],
                               [[synth.f32(o).astype(np.float64) for o in lst]
                                for lst in d["omega_tildes"]], sweeps=2, ranks=rk)
        A0 = F.hosvd_init(ref_t["U"], ref_t["G"], R)
        ref = F.ffcp(ref_t["U"], ref_t["G"], A0, update="als", max_it=40, tol=0.0)
        np.testing.assert_allclose(one["fits"], ref["fits"], rtol=0, atol=1e-5)
