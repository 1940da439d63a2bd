"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 1000 x 1000 x 1000 FP32 CP-20 tensor (column congruence
U[0.5, 0.95], SNR 30 dB, Omega_n 1000 x 30, Omega~_n 900 x 30, two sweeps,
Tucker ranks 20), in the plain FP32 form and in the precision form.

The oracle cannot run the whole method at this size, so:

* sampled outputs it computes one by one from the seeded inputs alone:
  rows of the first sweep's sketches Z_1 and Z_3 (the sketch step of Alg. 3 with
  the second test matrix), each from one 1000 x 1000 slice of Y, in FP64;
  ||Y||^2 as the plain FP64 sum of squares; the BF16 copy of sampled slabs
  from its definition, bf16_rne(Y[a] 2^-e_a) with e_a = 0 while the
  exponent of the slab's largest magnitude lies in [-100, 100];
* properties that hold at any size: orthonormal U_n and sweep-1 bases, the
  Pythagoras bound ||G|| <= ||Y|| for the projected core, and FFCP-ALS's
  non-decreasing closed-form fit, ending with a change below the tolerance.

Tolerance of the sketch rows (norm-wise relative): each entry sums 1e6
products; the GPU accumulates in FP32 in three stages (1000 terms in the
streaming pass, chunks of 480 in the sketch product, 63 chunk sums), so the
rounding error is at most about (1000 + 480 + 63) u ~ 9e-5 of the sum of
the terms' magnitudes, and with the terms' random signs typically about
sqrt of that count times u ~ 2e-6 of the result; 1e-4 is the bound.  In the
precision form the oracle consumes the same BF16-rounded operands the GPU
multiplies (the rounding written here, not the library's), so the same
bound holds.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT = 1000, 20, 30
ROWS = (0, 517, 999)


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def work():
    dev = torch.device("cuda:0")
    d = synth.cp_congruent_device(1885, (I, I, I), R, 0.5, 0.95, 30.0, (RT,) * 3,
                                  sweeps=2, device=dev)
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    torch.cuda.synchronize()
    return {"Y": d["Y"], "om32": om32, "omt32": omt32,
            "om_d": [torch.from_numpy(o).to(dev) for o in om32],
            "omt_d": [[torch.from_numpy(o).to(dev) for o in lst] for lst in omt32]}


def bf16_round(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def bf16_bits(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sketch_row(S, Oa, Ob, Ot):
    """One row of Z_n: vec(Oa^T S Ob) (row-major over the two kept test-matrix
    indices) times Omega~_n, for the 1000 x 1000 slice S of Y at that row."""
    X = Oa.T @ S @ Ob
    return X.reshape(-1) @ Ot


def run(P, w, precision, **kw):
    out = P.tucker_rand(w["Y"], w["om_d"], w["omt_d"], ranks=(R, R, R), sweeps=2,
                        precision=precision, trace=True, **kw)
    torch.cuda.synchronize()
    return out


def check_sketch_rows(out, w, bf16):
    om = [o.astype(np.float64) for o in w["om32"]]
    omt = [o.astype(np.float64) for o in w["omt32"][0]]
    rnd = bf16_round if bf16 else (lambda x: np.asarray(x, np.float64))
    Z1 = out["trace"]["Z"][0].cpu().numpy().astype(np.float64)
    Z3 = out["trace"]["Z"][2].cpu().numpy().astype(np.float64)
    for i in ROWS:
        # mode 1: the streamed contraction is mode 3's (Omega_3 in BF16)
        S = rnd(w["Y"][i].cpu().numpy())
        o3 = rnd(w["om32"][2]) if bf16 else om[2]
        assert rel(Z1[i], sketch_row(S, om[1], o3, omt[0])) <= 1e-4, ("Z_1", i)
        # mode 3: the streamed contraction is mode 2's (Omega_2 in BF16)
        S = rnd(w["Y"][:, :, i].contiguous().cpu().numpy())
        o2 = rnd(w["om32"][1]) if bf16 else om[1]
        assert rel(Z3[i], sketch_row(S, om[0], o2, omt[2])) <= 1e-4, ("Z_3", i)


def check_properties(out, w):
    N = 3
    for n in range(N):
        U = out["U"][n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(U.T @ U - np.eye(R)) <= 1e-5, n
        Q = out["trace"]["Q"][n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(Q.T @ Q - np.eye(RT)) <= 1e-5, n
    # ||Y||^2 as the plain FP64 sum, slab by slab on the host
    n2 = 0.0
    for a0 in range(0, I, 100):
        blk = w["Y"][a0:a0 + 100].cpu().numpy().astype(np.float64)
        n2 += float(np.sum(blk * blk))
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2
    G = out["G"].cpu().numpy().astype(np.float64)
    assert float(np.sum(G * G)) <= n2 * (1 + 1e-5)
    return n2


def test_fullsize_plain_fp32(P, work):
    out = run(P, work, "f32")
    check_sketch_rows(out, work, bf16=False)
    check_properties(out, work)


def test_fullsize_precision_form(P, work):
    ybf16 = torch.empty(P.bf16_copy_shape((I, I, I)), dtype=torch.int16, device="cuda")
    assert ybf16.shape == (I, I, 1024)
    out = run(P, work, "bf16", ybf16=ybf16)
    check_sketch_rows(out, work, bf16=True)
    check_properties(out, work)
    # the BF16 copy of sampled slabs, bit for bit
    got = out["ybf16"]
    for a in (0, 123, 999):
        Y32 = work["Y"][a].cpu().numpy()
        m = float(np.abs(Y32).max())
        e = int(np.frexp(m)[1] - 1) if m > 0 else 0
        e = e if abs(e) > 100 else 0   # scale only outside the window
        want = bf16_bits(np.ldexp(Y32.astype(np.float64), -e).astype(np.float32))
        row = got[a].cpu().numpy().view(np.uint16)
        assert np.array_equal(row[:, :I], want), a
        assert not row[:, I:].any(), a


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_fullsize_ffcp_fit_trace(P, work, precision):
    out = run(P, work, precision)
    f = P.ffcp(out["U"], out["G"], R, update="als", init="hosvd", max_it=1000, tol=1e-7,
               fit_trace=True)
    fits = f["fits"]
    it = int(f["info"]["iterations"])
    assert f["info"]["converged"] == 1 and it == len(fits)
    assert np.all(np.diff(fits) >= -1e-9)          # ALS never lowers the fit
    assert 0.99 < fits[-1] <= 1.0
    assert abs(fits[-1] - fits[-2]) < 1e-7
    # columns of A_n, n < N, have unit norm; lambda carries the scale
    for n in range(2):
        A = f["A"][n].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(np.linalg.norm(A, axis=0), 1.0, atol=1e-5)
