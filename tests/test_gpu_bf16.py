"""GPU parity of the BF16 precision form (precision="bf16", RT_BF16_MIXED).

The streamed contractions read Y rounded to BF16 (round to nearest even,
after an exact power-of-two scale per slab) and the streamed factor rounded
to BF16; products accumulate in FP32.  Two kinds of checks:

* exact-input parity: the oracle recomputes the first-sweep sketches from
  the same rounded operands (rounding written here, independently of the
  library), so the only difference left is FP32 accumulation: relative
  1e-5;
* end-to-end accuracy against the FP64 oracle on the unrounded tensor: the
  rounding perturbs Y by E with ||E||_F <= 2^-9 ||Y||_F, so each subspace
  moves by at most about ||E||_2 / (sigma_R - sigma_{R+1}) (Wedin); the
  bound used is 4 * 2^-9 ||Y||_F / gap_n, computed from the data.
"""

import numpy as np
import pytest

import synth
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


def bf16_bits(x):
    """Round-to-nearest-even FP32 -> BF16 bit patterns (uint16)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_round(x):
    return bf16_value(bf16_bits(x))


def slab_exponents(Y):
    """Scale exponent e_a per slab of the [A, I_{N-1}, I_N] view: 0 while
    floor(log2(max |slab|)) lies in [-100, 100], that exponent otherwise."""
    A = int(np.prod(Y.shape[:-2]))
    m = np.abs(Y.reshape(A, -1)).max(axis=1)
    e = np.where(m > 0, np.frexp(m)[1] - 1, 0)
    return np.where(np.abs(e) <= 100, 0, e)


def first_sweep_sketches(Y32, om32, omt32):
    """Sketches of the first sweep on the operands the BF16 path consumes:
    BF16(Y); the mode-N (resp. N-1) contraction that streams Y uses BF16
    Omega_N (resp. Omega_{N-1}); every other contraction the FP32 values."""
    N = Y32.ndim
    Yr = bf16_round(Y32)
    om = [np.asarray(o, np.float64) for o in om32]
    Z = []
    for n in range(N):
        streamed = N - 1 if n != N - 1 else N - 2
        X = T.ttm_t(Yr, bf16_round(om32[streamed]), streamed)
        for p in range(N):
            if p != n and p != streamed:
                X = T.ttm_t(X, om[p], p)
        Z.append(T.unfold(X, n) @ np.asarray(omt32[n], np.float64))
    return Z


def run(P, Y32, om32, omt32, ranks, sweeps, **kw):
    return P.tucker_rand(dev(Y32), [dev(o) for o in om32],
                         [[dev(o) for o in lst] for lst in omt32],
                         ranks=ranks, sweeps=sweeps, precision="bf16", trace=True, **kw)


SHAPES = [((12, 70, 104), (8, 9, 10)),     # ragged row block, partial column tile
          ((5, 300, 96), (5, 16, 30)),     # several row blocks per wave
          ((3, 33, 64), (3, 5, 32)),       # exactly one column tile, R~ = 32
          ((4, 5, 40, 48), (4, 5, 6, 7)),  # 4-way: slabs over two modes
          ((6, 50, 60), (6, 8, 9)),        # I_N % 8 == 4: half chunks at row ends
          ((3, 40, 300), (3, 10, 30)),     # the learned-init workload's width
          ((2, 800, 72), (2, 9, 10)),      # four row blocks per wave, the last masked
          ((2, 1000, 36), (2, 7, 12))]     # four row blocks per wave, half chunks


@pytest.mark.parametrize("dims,rt", SHAPES)
def test_bf16_first_sweep_sketches_exact_inputs(P, dims, rt):
    d = synth.case_tucker(401 + len(dims), dims, tuple(min(3, r) for r in rt), 30.0, rt)
    Y32 = synth.f32(d["Y"])
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(d["omega_tildes"][0])]
    out = run(P, Y32, om32, omt32, tuple(min(3, r) for r in rt), 1)
    Zr = first_sweep_sketches(Y32, om32, omt32[0])
    for n in range(len(dims)):
        assert rel(host(out["trace"]["Z"][n]), Zr[n]) <= 1e-5, n
    assert abs(out["info"]["normY2"] - np.sum(Y32.astype(np.float64) ** 2)) <= \
        1e-9 * np.sum(Y32.astype(np.float64) ** 2)


def test_bf16_copy_is_scaled_rne(P):
    """The BF16 copy holds bf16_rne(Y * 2^-e_a), bit for bit: e_a = 0 for
    slabs whose largest magnitude has its exponent in [-100, 100], that
    exponent for the others (slabs scaled very differently, two outside the
    window, one of them with FP32 subnormals)."""
    d = synth.case_tucker(410, (8, 40, 56), (3, 3, 3), 30.0, (6, 6, 6))
    scales = np.array([1e-36, 1e-28, 1e-3, 1.0, 7.0, 1e5, 3e20, 1e32])
    Y32 = synth.f32(d["Y"] * scales[:, None, None])
    e_want = slab_exponents(Y32)
    assert e_want[0] < -100 and e_want[-1] > 100 and not e_want[1:-1].any()
    assert np.any((Y32[0] != 0) & (np.abs(Y32[0]) < np.finfo(np.float32).tiny))
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(d["omega_tildes"][0])]
    out = run(P, Y32, om32, omt32, (3, 3, 3), 1)
    e = slab_exponents(Y32)
    scaled = np.ldexp(Y32.astype(np.float64), -e[:, None, None]).astype(np.float32)
    want = bf16_bits(scaled)
    got = out["ybf16"].cpu().numpy().view(np.uint16)
    # rows padded to a multiple of 64 values, the padding zero
    assert got.shape == (8, 40, 64)
    assert np.array_equal(got[..., :56], want)
    assert not got[..., 56:].any()


def test_bf16_input_path(P):
    """Caller-provided BF16 tensor (no scaling): sketches equal the oracle's
    on the same values."""
    dims, rt = (7, 64, 80), (7, 11, 12)
    d = synth.case_tucker(411, dims, (3, 3, 3), 30.0, rt)
    Y32 = synth.f32(d["Y"])
    bits = bf16_bits(Y32)
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(d["omega_tildes"][0])]
    Yb = torch.from_numpy(bits.view(np.int16)).cuda()
    out = P.tucker_rand(Yb, [dev(o) for o in om32], [[dev(o) for o in omt32[0]]],
                        ranks=(3, 3, 3), sweeps=1, precision="bf16", trace=True,
                        bf16_input=True, dims=dims)
    Zr = first_sweep_sketches(Y32, om32, omt32[0])
    for n in range(3):
        assert rel(host(out["trace"]["Z"][n]), Zr[n]) <= 1e-5, n
    yr = bf16_value(bits)
    assert abs(out["info"]["normY2"] - np.sum(yr ** 2)) <= 1e-9 * np.sum(yr ** 2)


@pytest.mark.parametrize("sweeps", [1, 2])
def test_bf16_end_to_end_vs_fp64_oracle(P, sweeps):
    dims, R, rt = (40, 120, 96), (5, 5, 5), (12, 12, 12)
    d = synth.case_tucker(412, dims, R, 30.0, rt, sweeps=2)
    Y32 = synth.f32(d["Y"])
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"][:sweeps]]
    out = run(P, Y32, om32, omt32, R, sweeps)
    Y = Y32.astype(np.float64)
    ref = RT.rand_tucker(Y, [o.astype(np.float64) for o in om32],
                         [[o.astype(np.float64) for o in lst] for lst in omt32],
                         sweeps=sweeps, ranks=R)
    nY = np.linalg.norm(Y)
    for n in range(3):
        s = np.linalg.svd(T.unfold(Y, n), compute_uv=False)
        bound = 4 * 2.0 ** -9 * nY / (s[R[n] - 1] - s[R[n]])
        assert projector_distance(host(out["U"][n]), ref["U"][n]) <= bound, n
    eG = aligned_core_error(host(out["G"]), [host(u) for u in out["U"]], ref["G"], ref["U"])
    assert eG <= 4 * 2.0 ** -9 * nY / np.linalg.norm(ref["G"]) + 1e-4
