"""Sequential RandTucker (Algorithm 2) on the GPU against the FP64 oracle.

Both sides draw the dense Gaussian test matrices from the same
counter-based generator (Philox4x32-10 and Box-Muller in FP64), each
written from the generator's definition: the device in
csrc/sequential.hip, the oracle in oracle/rng.py.  Their values agree to
the last bits of FP64 (the two sides' log and cos may differ by an ulp),
i.e. bit for bit after rounding to FP32 except for an occasional ulp.

Checked: the generator itself; the whole method on noise-free tensors of
multilinear rank equal to the sketch widths (every sketch has full rank, so
the bases are determined and compared as subspaces) in FP64 and FP32; on a
noisy tensor the first sketch (identical inputs on both sides), the core's
norm (the Tucker fit) and orthonormality.
"""

import numpy as np
import pytest

import synth
from oracle import randtucker as RT
from oracle import rng as G
from oracle import tensor as T
from oracle.metrics import projector_distance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 14121885


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def test_gaussian_matrix_matches_the_oracle_generator(P):
    rows, cols = 7000, 30
    want = G.gaussian_matrix(rows, cols, 2, SEED)
    got64 = P.gaussian_matrix(rows, cols, 2, SEED, dtype=torch.float64).cpu().numpy()
    assert np.max(np.abs(got64 - want)) <= 4e-15 * np.max(np.abs(want))
    got32 = P.gaussian_matrix(rows, cols, 2, SEED).cpu().numpy()
    w32 = want.astype(np.float32)
    ulps = np.abs(got32.view(np.int32).astype(np.int64) - w32.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1 and np.mean(ulps == 0) > 0.999
    # an entry depends on (seed, mode, row, column) only
    part = P.gaussian_matrix(100, 7, 2, SEED, dtype=torch.float64).cpu().numpy()
    assert np.array_equal(part, got64[:100, :7])


def exact_rank_tensor(seed, dims, rt):
    rng = np.random.default_rng(seed)
    Gc = rng.standard_normal(rt)
    U = [np.linalg.qr(rng.standard_normal((I, r)))[0] for I, r in zip(dims, rt)]
    return T.tucker_full(Gc, U)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("dims,rt", [((30, 34, 38), (5, 6, 7)), ((12, 14, 16, 18), (3, 4, 5, 6)),
                                     ((70, 9, 130), (12, 9, 20))])
def test_sequential_exact_rank_vs_oracle(P, precision, dims, rt):
    Y = exact_rank_tensor(sum(dims), dims, rt)
    tdt = torch.float64 if precision == "f64" else torch.float32
    Yd = torch.from_numpy(Y).to(tdt).cuda()
    Yh = Yd.double().cpu().numpy()
    out = P.tucker_sequential(Yd, rt, SEED, keep_omegas=True)
    oms = G.sequential_omegas(dims, rt, SEED)
    if precision == "f32":
        oms = [o.astype(np.float32).astype(np.float64) for o in oms]
    for n in range(len(dims)):
        got = out["omegas"][n].double().cpu().numpy()
        assert got.shape == oms[n].shape
        assert np.max(np.abs(got - oms[n])) <= (1e-14 if precision == "f64" else 2.4e-7) * 6.0
    Uo, Go = RT.rand_tucker_sequential(Yh, oms)
    tol = 1e-10 if precision == "f64" else 1e-4
    U = [u.double().cpu().numpy() for u in out["U"]]
    for n in range(len(dims)):
        assert np.linalg.norm(U[n].T @ U[n] - np.eye(rt[n])) <= tol
        assert projector_distance(U[n], Uo[n]) <= tol, n
    Gd = out["G"].double().cpu().numpy()
    rec = T.tucker_full(Gd, U)
    assert np.linalg.norm(rec - Yh) <= tol * np.linalg.norm(Yh)


def test_sequential_noisy_vs_oracle(P):
    dims, ranks, rt = (60, 64, 72), (4, 5, 6), (10, 11, 12)
    d = synth.case_tucker(3101, dims, ranks, 20.0, rt)
    Y32 = synth.f32(d["Y"])
    out = P.tucker_sequential(torch.from_numpy(Y32).cuda(), rt, SEED)
    Y = Y32.astype(np.float64)
    oms = [o.astype(np.float32).astype(np.float64) for o in G.sequential_omegas(dims, rt, SEED)]
    Uo, Go = RT.rand_tucker_sequential(Y, oms)
    # the first sketch sees identical inputs on both sides
    Z1 = T.unfold(Y, 0) @ oms[0]
    Q1 = RT.orth_qr(Z1)
    U1 = out["U"][0].double().cpu().numpy()
    assert projector_distance(U1, Q1) <= 1e-4
    # the captured energy (Tucker fit) agrees; later bases depend on the
    # device's own earlier bases, whose trailing directions are noise
    Gd = out["G"].double().cpu().numpy()
    y2 = float(np.sum(Y * Y))
    assert abs(np.sum(Gd * Gd) - np.sum(Go * Go)) <= 1e-5 * y2
    for u in out["U"]:
        uu = u.double().cpu().numpy()
        assert np.linalg.norm(uu.T @ uu - np.eye(uu.shape[1])) <= 1e-5
