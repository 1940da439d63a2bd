"""Parity at the full size of the nonnegative 4-way workload: the
200 x 200 x 200 x 200 FP32 tensor of a nonnegative CP model of rank 15 (U[0,1]
factors with exactly 20 % zeros, |N(0, 0.01)| noise; the Section V-A
construction), compressed by the precision form (two sweeps, Omega_n
200 x 25, Omega~_n 15625 x 25, Tucker ranks 15) and factored by FFCP-HALS.

The streaming view is [A = 40000 slabs, 200, 200]: the fused conversion runs
40000 slab rows of blocks, and the contraction kernels take one 32-row block
per wavefront.

As at 1000^3 the oracle cannot run the whole method at this size, so:

* sampled rows of the first sweep's sketches Z_1 and Z_4 (the sketch step of
  Alg. 3 with the first test matrix), each from one 200^3 slice of Y, in
  FP64 on the operands the path multiplies: the BF16 copy and the BF16
  factor in the streamed contraction (mode 4 for Z_1, mode 3 for Z_4), the
  FP32 values elsewhere;
* ||Y||^2 as the plain FP64 sum of squares;
* properties that hold at any size: orthonormal U_n and sweep-1 bases, the
  Pythagoras bound ||G|| <= ||Y||, and FFCP-HALS's non-decreasing fit with
  nonnegative factors.

Tolerance of the sketch rows (norm-wise relative) 1e-4, from the same count
as at 1000^3: each entry sums 8e6 products accumulated in FP32 in stages of
200 (streamed contraction), 200 and 200 (the other two modes) and the split
sketch product.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT, RN = 200, 15, 25, 15
DIMS = (I, I, I, I)
ROWS = (0, 97, 199)


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def work():
    dev = torch.device("cuda:0")
    d = synth.nonneg_cp_device(1886, DIMS, R, (RT,) * 4, sweeps=2, device=dev)
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    A0 = [synth.f32(a) for a in synth.init_factors(d["init_rng"], DIMS, R, nonneg=True)]
    torch.cuda.synchronize()
    return {"Y": d["Y"], "om32": om32, "omt32": omt32, "A0": A0,
            "om_d": [torch.from_numpy(o).to(dev) for o in om32],
            "omt_d": [[torch.from_numpy(o).to(dev) for o in lst] for lst in omt32]}


def bf16_round(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_fullsize_4way_precision_form_and_hals(P, work):
    w = work
    out = P.tucker_rand(w["Y"], w["om_d"], w["omt_d"], ranks=(RN,) * 4, sweeps=2,
                        precision="bf16", trace=True)
    torch.cuda.synchronize()
    om = [o.astype(np.float64) for o in w["om32"]]
    omt = [o.astype(np.float64) for o in w["omt32"][0]]
    Z1 = out["trace"]["Z"][0].cpu().numpy().astype(np.float64)
    Z4 = out["trace"]["Z"][3].cpu().numpy().astype(np.float64)
    o3b, o4b = bf16_round(w["om32"][2]), bf16_round(w["om32"][3])
    for i in ROWS:
        # Z_1 row i: Y[i] (modes 2, 3, 4); mode 4 streamed in BF16
        S = bf16_round(w["Y"][i].cpu().numpy())
        X = np.tensordot(S, o4b, axes=([2], [0]))             # j2, j3, k4
        X = np.tensordot(X, om[2], axes=([1], [0]))           # j2, k4, k3
        X = np.tensordot(om[1], X, axes=([0], [0]))           # k2, k4, k3
        X = X.transpose(0, 2, 1)                              # k2, k3, k4
        assert rel(Z1[i], X.reshape(-1) @ omt[0]) <= 1e-4, ("Z_1", i)
        # Z_4 row i: Y[..., i] (modes 1, 2, 3); mode 3 streamed in BF16
        S = bf16_round(w["Y"][:, :, :, i].contiguous().cpu().numpy())
        X = np.tensordot(S, o3b, axes=([2], [0]))             # j1, j2, k3
        X = np.tensordot(X, om[1], axes=([1], [0]))           # j1, k3, k2
        X = np.tensordot(om[0], X, axes=([0], [0]))           # k1, k3, k2
        X = X.transpose(0, 2, 1)                              # k1, k2, k3
        assert rel(Z4[i], X.reshape(-1) @ omt[3]) <= 1e-4, ("Z_4", i)
    for n in range(4):
        U = out["U"][n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(U.T @ U - np.eye(RN)) <= 1e-5, n
        Q = out["trace"]["Q"][n].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(Q.T @ Q - np.eye(RT)) <= 1e-5, n
    n2 = 0.0
    for a0 in range(0, I, 10):
        blk = w["Y"][a0:a0 + 10].cpu().numpy().astype(np.float64)
        n2 += float(np.sum(blk * blk))
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2
    assert out["info"]["nonfinite"] == 0
    G = out["G"].cpu().numpy().astype(np.float64)
    assert float(np.sum(G * G)) <= n2 * (1 + 1e-5)

    # FFCP-HALS (nonnegative) on the Tucker format, from U[0,1] factors
    f = P.ffcp(out["U"], out["G"], R, update="hals",
               A_init=[torch.from_numpy(a).cuda() for a in w["A0"]],
               max_it=300, tol=1e-7, fit_trace=True, normY2=n2)
    fits = f["fits"]
    it = int(f["info"]["iterations"])
    assert it == len(fits) and it >= 2
    assert np.all(np.diff(fits) >= -1e-7)   # HALS never lowers the fit
    # the noise alone caps the fit near 0.977 (||Y - Y*|| / ||Y|| = 0.023
    # for this model at 40^4); a rank-15 nonnegative fit from a random start
    # reaches most of that
    assert 0.9 < fits[-1] < 0.99
    for n in range(4):
        assert float(f["A"][n].min()) >= 0.0, n
