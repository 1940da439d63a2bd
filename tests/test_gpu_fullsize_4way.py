"""Parity at the full size of the nonnegative 4-way workload: the
200 x 200 x 200 x 200 FP32 tensor of a nonnegative CP model of rank 15 (U[0,1]
factors with exactly 20 % zeros, |N(0, 0.01)| noise; the Section V-A
construction), compressed by the precision form (two sweeps, Omega_n
200 x 25, Omega~_n 15625 x 25, Tucker ranks 15) and factored by FFCP-HALS.

The streaming view is [A = 40000 slabs, 200, 200]: the conversion runs
40000 x 5 blocks in one dimension, the contraction kernels one slab per
workgroup.

Checked on the whole tensor, in FP64 on the host:

* the first sweep's sketches Z_n element-wise, recomputed from the operands
  the path multiplies (Y and the streamed test matrix rounded to BF16 here,
  independently of the library; every slab's exponent is 0, checked).  Each
  entry sums 8e6 products accumulated in FP32 in stages of 200 (streamed
  contraction), 200 and 200 (the other two modes) and the split sketch
  product: 1e-4 of max |Z_n| as at 1000^3;
* the second sweep's sketches and the core, recomputed from the bases the
  library returned (the same bound);
* ||Y||^2 as the plain FP64 sum of squares; orthonormal bases.

Against the FP64 oracle: both sides run the whole method (precision form on
the device, FP64 on the host, same Omega with Omega_1's first 40 rows) on the
mode-1 slab Y[0:40] (3.2e8 entries); the subspaces within twice the Wedin
estimate of the BF16 rounding (as at 1000^3).  FFCP-HALS on the full tensor's
Tucker format: non-decreasing fit, nonnegative factors.
"""

import numpy as np
import pytest

import synth
from oracle import randtucker as RT
from oracle.metrics import aligned_core_error, projector_distance

from _fullsize import bf16_round, dev64, maxrel, path_core, path_sketches

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT_, RN, N = 200, 15, 25, 15, 4
DIMS = (I, I, I, I)
TOL_Z = 1e-4
SLAB = 40


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def work():
    dev = torch.device("cuda:0")
    d = synth.nonneg_cp_device(1886, DIMS, R, (RT_,) * 4, sweeps=2, device=dev)
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    A0 = [synth.f32(a) for a in synth.init_factors(d["init_rng"], DIMS, R, nonneg=True)]
    torch.cuda.synchronize()
    return {"Y": d["Y"], "om32": om32, "omt32": omt32, "A0": A0,
            "om_d": [torch.from_numpy(o).to(dev) for o in om32],
            "omt_d": [[torch.from_numpy(o).to(dev) for o in lst] for lst in omt32]}


def host_bf16(Y, rows=10):
    out = np.empty(tuple(Y.shape), dtype=np.float64)
    n2 = 0.0
    for a in range(0, Y.shape[0], rows):
        blk = Y[a:a + rows].cpu().numpy()
        b64 = blk.astype(np.float64)
        n2 += float(np.sum(b64 * b64))
        out[a:a + rows] = bf16_round(blk)
    return out, n2


def test_fullsize_4way_precision_form_and_hals(P, work):
    w = work
    out = P.tucker_rand(w["Y"], w["om_d"], w["omt_d"], ranks=(RN,) * 4, sweeps=2,
                        precision="bf16", trace=True)
    torch.cuda.synchronize()
    mx = float(w["Y"].abs().max())
    assert 0.0 < mx and np.frexp(mx)[1] - 1 <= 100
    assert float(w["Y"].reshape(I * I, -1).abs().amax(dim=1).min()) >= 2.0 ** -100
    Yb, n2 = host_bf16(w["Y"])
    om = [o.astype(np.float64) for o in w["om32"]]
    Zx = path_sketches(Yb, om, [o.astype(np.float64) for o in w["omt32"][0]], bf16=True)
    for n in range(N):
        e = maxrel(dev64(out["trace"]["Z"][n]), Zx[n])
        assert e <= TOL_Z, ("sweep-1 Z vs exact-input FP64", n, e)
    del Zx
    Q1 = [dev64(out["trace"]["Q"][n]) for n in range(N)]
    Q2 = [dev64(out["trace"]["Q"][N + n]) for n in range(N)]
    Zp = path_sketches(Yb, Q1, [o.astype(np.float64) for o in w["omt32"][1]], bf16=True)
    for n in range(N):
        e = maxrel(dev64(out["trace"]["Z"][N + n]), Zp[n])
        assert e <= TOL_Z, ("sweep-2 Z from the returned bases", n, e)
    del Zp
    e = maxrel(dev64(out["trace"]["Gt"]), path_core(Yb, Q2, bf16=True))
    assert e <= TOL_Z, ("core from the returned bases", e)
    del Yb
    for n in range(N):
        U = dev64(out["U"][n])
        assert np.linalg.norm(U.T @ U - np.eye(RN)) <= 1e-5, n
        for q in (Q1[n], Q2[n]):
            assert np.linalg.norm(q.T @ q - np.eye(RT_)) <= 1e-5, n
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2
    assert out["info"]["nonfinite"] == 0

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
    for n in range(N):
        assert float(f["A"][n].min()) >= 0.0, n


def test_slab_precision_form_vs_fp64_oracle(P, work):
    """The whole method on Y[0:40] on both sides (a fresh device call on the
    slab): d(U_n) within twice the Wedin estimate of the BF16 rounding, e_G
    within twice their root-sum-square plus 2^-9."""
    w = work
    Ys = w["Y"][:SLAB].contiguous()
    om_d = [w["om_d"][0][:SLAB].contiguous()] + w["om_d"][1:]
    out = P.tucker_rand(Ys, om_d, w["omt_d"], ranks=(RN,) * 4, sweeps=2,
                        precision="bf16")
    Y64 = Ys.double().cpu().numpy()
    Yb = bf16_round(Ys.cpu().numpy())
    om = [o.astype(np.float64) for o in w["om32"]]
    om[0] = om[0][:SLAB]
    omt = [[o.astype(np.float64) for o in lst] for lst in w["omt32"]]
    tk = RT.rand_tucker(Y64, om, omt, sweeps=2, ranks=(RN,) * 4)
    rms = float(np.sqrt(np.mean((Yb - Y64) ** 2)))
    del Yb, Y64
    U = [dev64(u) for u in out["U"]]
    d = [projector_distance(U[n], tk["U"][n]) for n in range(N)]
    eG = aligned_core_error(dev64(out["G"]), U, tk["G"], tk["U"])
    dims = Ys.shape
    total = float(np.prod(dims))
    bound = []
    for n in range(N):
        sv = np.linalg.svd(np.moveaxis(tk["Gt"], n, 0).reshape(RT_, -1), compute_uv=False)
        gap = sv[RN - 1] - sv[RN]
        s_n = rms * (np.sqrt(dims[n]) + np.sqrt(total / dims[n]))
        bound.append(s_n / (gap - s_n) if gap > s_n else np.inf)
    print(f"slab: d(U_n) {d}, e_G {eG}, Wedin estimates {bound}", flush=True)
    for n in range(N):
        assert d[n] <= 2.0 * bound[n], (n, d[n], bound[n])
    assert eG <= 2.0 * float(np.sqrt(np.sum(np.square(bound)))) + 2.0 ** -9, (eG, bound)
