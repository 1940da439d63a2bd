"""The precision form on wide slabs: I_N in (384, 1024], where one pass
reads each 32-row block of a slab as one contiguous span, and the first
pass converts the FP32 tensor to BF16 in the same read that feeds the first
sweep's products.  Later passes also contract mode N-1 inside each slab
(C = TA x_{N-1} B_{N-1}^T), from which the sketches of modes < N-1 and the
core are finished.  Shapes include more than 1024 rows per slab (no row
limit on this pass), 7..16 column tiles, a row length with a half 8-value
chunk at its end, and a 4-way tensor.

Checked in FP64 against quantities recomputed here from the operands the
path multiplies (BF16 rounding written here, independently of the library):
the first sweep's sketches, the second sweep's sketches from the first
sweep's returned bases, and the core from the final returned bases, each
element-wise at 1e-4 of the result's largest magnitude (FP32 sums of up to
a few thousand terms); ||Y||^2 to 1e-9; the BF16 copy bit for bit.  Slabs
whose scale exponent lies outside [-100, 100] are converted again and their
products recomputed after the first read: checked on tensors where every
slab takes that route.
"""

import numpy as np
import pytest

import synth

from _fullsize import bf16_round, maxrel, path_core, path_sketches

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-4


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


WIDE = [((20, 70, 600), (3, 3, 3), (10, 12, 14)),        # 10 column tiles
        ((2, 1100, 1000), (2, 3, 3), (2, 9, 11)),        # 1100 rows, 16 column tiles
        ((9, 64, 392), (3, 3, 3), (9, 6, 7)),            # 7 column tiles
        ((3, 40, 452), (3, 3, 3), (3, 10, 30)),          # half chunk at the row end
        ((4, 5, 50, 520), (2, 2, 3, 3), (4, 5, 6, 32))]  # 4-way, R~_N = 32


@pytest.mark.parametrize("dims,R,rt", WIDE)
def test_wide_slabs_two_sweeps_and_core(P, dims, R, rt):
    d = synth.case_tucker(1700 + dims[-1], dims, R, 30.0, rt, sweeps=2)
    Y32 = synth.f32(d["Y"])
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    out = P.tucker_rand(dev(Y32), [dev(o) for o in om32], [[dev(o) for o in l] for l in omt32],
                        ranks=R, sweeps=2, precision="bf16", trace=True)
    torch.cuda.synchronize()
    N = len(dims)
    Yb = bf16_round(Y32)
    # the copy, bit for bit (rows padded to a multiple of 64, zeros)
    got = out["ybf16"].cpu().numpy().view(np.uint16)
    A = int(np.prod(dims[:-2]))
    ld = got.shape[-1]
    assert ld == -(-dims[-1] // 64) * 64
    got = got.reshape(A, dims[-2], ld)
    want = bf16_bits(Y32).reshape(A, dims[-2], dims[-1])
    assert np.array_equal(got[..., :dims[-1]], want)
    assert not got[..., dims[-1]:].any()
    n2 = float(np.sum(Y32.astype(np.float64) ** 2))
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2
    # sweep 1: the first read (FP32 in, products of the rounded values)
    Z1 = path_sketches(Yb, [o.astype(np.float64) for o in om32], omt32[0], bf16=True)
    for n in range(N):
        e = maxrel(host(out["trace"]["Z"][n]), Z1[n])
        assert e <= TOL, ("sweep 1", n, e)
    # sweep 2 from the first sweep's returned bases (modes < N-1 through C)
    Q1 = [host(out["trace"]["Q"][n]) for n in range(N)]
    Z2 = path_sketches(Yb, Q1, omt32[1], bf16=True)
    for n in range(N):
        e = maxrel(host(out["trace"]["Z"][N + n]), Z2[n])
        assert e <= TOL, ("sweep 2", n, e)
    # the core from the final bases (mode N-1 inside the pass)
    Q2 = [host(out["trace"]["Q"][N + n]) for n in range(N)]
    e = maxrel(host(out["trace"]["Gt"]), path_core(Yb, Q2, bf16=True))
    assert e <= TOL, ("core", e)


@pytest.mark.parametrize("scale", [1e35, 1e-33])
def test_wide_slabs_outside_the_scale_window(P, scale):
    """Every slab's largest magnitude has its exponent outside [-100, 100]:
    the copy holds bf16_rne(Y 2^-e_a) and the first sweep's products are
    those of the scaled copy times 2^e_a (recomputed after the first read)."""
    dims, R, rt = (6, 40, 520), (3, 3, 3), (6, 8, 9)
    d = synth.case_tucker(1750, dims, R, 30.0, rt)
    Y32 = synth.f32(d["Y"] * scale)
    m = np.abs(Y32.reshape(6, -1)).max(axis=1)
    e = np.frexp(m)[1] - 1
    assert np.all(np.abs(e) > 100)
    if scale < 1:
        assert np.any((Y32 != 0) & (np.abs(Y32) < np.finfo(np.float32).tiny))
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(d["omega_tildes"][0])]
    out = P.tucker_rand(dev(Y32), [dev(o) for o in om32], [[dev(o) for o in omt32[0]]],
                        ranks=R, sweeps=1, precision="bf16", trace=True)
    torch.cuda.synchronize()
    scaled = np.ldexp(Y32.astype(np.float64), -e[:, None, None]).astype(np.float32)
    got = out["ybf16"].cpu().numpy().view(np.uint16)
    assert np.array_equal(got[..., :520], bf16_bits(scaled))
    assert not got[..., 520:].any()
    Yr = np.ldexp(bf16_round(scaled), e[:, None, None])
    Z = path_sketches(Yr, [o.astype(np.float64) for o in om32], omt32[0], bf16=True)
    for n in range(3):
        err = maxrel(host(out["trace"]["Z"][n]), Z[n])
        assert err <= TOL, (n, err)
    n2 = float(np.sum(Y32.astype(np.float64) ** 2))
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2
