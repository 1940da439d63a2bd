"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 1000 x 1000 x 1000 FP32 CP-20 tensor (column congruence
U[0.5, 0.95], SNR 30 dB, Omega_n 1000 x 30, Omega~_n 900 x 30, two sweeps,
Tucker ranks 20), in the plain FP32 form and in the precision form.

The FP64 oracle runs the whole method on the whole tensor on the host
(RandTucker2i with the same Omega, two sweeps, truncation; FFCP-ALS from the
HOSVD start of its core; Fit_Y against Y), a few seconds with threaded BLAS.
Checked against it:

* the first sweep's sketches Z_n, element-wise.  Plain FP32: the oracle's
  own sketches.  Precision form: the same sketches recomputed in FP64 from
  the operands the path multiplies (Y and the streamed test matrix rounded
  to BF16 here, independently of the library; every slab's exponent is 0 at
  this size, checked).  Each entry sums 1e6 products that the device
  accumulates in FP32 in three stages (1000 terms in the streaming pass,
  chunks of 480 in the sketch product, 63 chunk sums): the rounding error is
  at most about (1000 + 480 + 63) u ~ 9e-5 of the terms' magnitudes and
  typically sqrt of that count times u ~ 2e-6; 1e-4 of max |Z_n| is the
  bound;
* the final bases and core against the oracle's: projector distance and the
  aligned core error, at 1e-4 (plain FP32).  The precision form against the
  unrounded FP64 oracle: the BF16 rounding of Y acts like noise about 26 dB
  below this tensor's own noise, and moves each subspace by up to its norm
  over the eigen-gap (Wedin); with column congruences up to 0.95 the gap of
  this workload is small, so the bound is computed from the data (twice the
  Wedin estimate for d(U_n), and for e_G twice the root-sum-square of the
  per-mode estimates plus 2^-9 for the rounding of the streamed basis);
* Fit_Y of FFCP against the oracle's, 1e-5 (FP32) / 1e-4 (precision form).

Properties of the returned quantities, at any size: the second sweep's
sketches are the sketches of Y with the first sweep's returned bases, and
the core is the projection of Y on the final returned bases (both recomputed
in FP64 from the returned FP32 bases, the same 1e-4 element-wise bound);
bases orthonormal; ||Y||^2 the FP64 sum of squares; the BF16 copy of sampled
slabs bit for bit; FFCP-ALS's fit non-decreasing.
"""

import numpy as np
import pytest

import synth
from oracle import ffcp as F
from oracle import randtucker as RT
from oracle.metrics import aligned_core_error, projector_distance

from _fullsize import bf16_round, dev64, host_f64, maxrel, path_core, path_sketches

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT_, N = 1000, 20, 30, 3
TOL_Z = 1e-4


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def work():
    dev = torch.device("cuda:0")
    d = synth.cp_congruent_device(1885, (I, I, I), R, 0.5, 0.95, 30.0, (RT_,) * 3,
                                  sweeps=2, device=dev)
    om32 = synth.f32(d["omegas"])
    omt32 = [synth.f32(x) for x in d["omega_tildes"]]
    torch.cuda.synchronize()
    return {"Y": d["Y"], "om32": om32, "omt32": omt32,
            "om_d": [torch.from_numpy(o).to(dev) for o in om32],
            "omt_d": [[torch.from_numpy(o).to(dev) for o in lst] for lst in omt32]}


@pytest.fixture(scope="module")
def host(work):
    Y64 = host_f64(work["Y"])
    return {"Y64": Y64, "n2": float(np.einsum("ijk,ijk->", Y64, Y64))}


@pytest.fixture(scope="module")
def oracle(work, host):
    """The FP64 oracle on the whole tensor: RandTucker2i (S = 2, ranks 20),
    FFCP-ALS from the HOSVD start of its core, Fit_Y against Y."""
    om = [o.astype(np.float64) for o in work["om32"]]
    omt = [[o.astype(np.float64) for o in lst] for lst in work["omt32"]]
    tk = RT.rand_tucker(host["Y64"], om, omt, sweeps=2, ranks=(R, R, R))
    A0 = F.hosvd_init(tk["U"], tk["G"], R)
    f = F.ffcp(tk["U"], tk["G"], A0, update="als", max_it=1000, tol=1e-7)
    fit_y = F.cp_fit_mttkrp(host["Y64"], f["A"], f["lam"])
    return {"tk": tk, "ffcp": f, "fit_y": fit_y}


def run(P, w, precision, **kw):
    out = P.tucker_rand(w["Y"], w["om_d"], w["omt_d"], ranks=(R, R, R), sweeps=2,
                        precision=precision, trace=True, **kw)
    torch.cuda.synchronize()
    return out


def check_properties(out, host, Yop, bf16):
    """Second-sweep sketches and the core recomputed from the returned bases
    (Yop: the values the path multiplies), orthonormality, ||Y||^2."""
    omt2 = [dev64(o) for o in out["_omt2"]]
    Q1 = [dev64(out["trace"]["Q"][n]) for n in range(N)]
    Q2 = [dev64(out["trace"]["Q"][N + n]) for n in range(N)]
    Zp = path_sketches(Yop, Q1, omt2, bf16=bf16)
    for n in range(N):
        e = maxrel(dev64(out["trace"]["Z"][N + n]), Zp[n])
        assert e <= TOL_Z, ("sweep-2 Z", n, e)
    Gp = path_core(Yop, Q2, bf16=bf16)
    e = maxrel(dev64(out["trace"]["Gt"]), Gp)
    assert e <= TOL_Z, ("core G~", e)
    for n in range(N):
        U = dev64(out["U"][n])
        assert np.linalg.norm(U.T @ U - np.eye(R)) <= 1e-5, n
        for q in (Q1[n], Q2[n]):
            assert np.linalg.norm(q.T @ q - np.eye(RT_)) <= 1e-5, n
    n2 = host["n2"]
    assert abs(out["info"]["normY2"] - n2) <= 1e-9 * n2


def errors_vs_oracle(out, oracle):
    tk = oracle["tk"]
    U = [dev64(u) for u in out["U"]]
    d = [projector_distance(U[n], tk["U"][n]) for n in range(N)]
    eG = aligned_core_error(dev64(out["G"]), U, tk["G"], tk["U"])
    print(f"errors vs FP64 oracle: d(U_n) {d}, e_G {eG}", flush=True)
    return d, eG


def rounding_bounds(host, Yb, oracle):
    """Subspace bound of the precision form from the data (Wedin):
    d_n <= s_n / (gap_n - s_n) with gap_n = sigma_R - sigma_{R+1} of the
    oracle's G~_(n) (the leading singular values of Y_(n) it captures) and
    s_n the spectral norm of the BF16 rounding E = bf16(Y) - Y unfolded,
    estimated as rms(E) (sqrt(I_n) + sqrt(prod_{p != n} I_p)), the norm of
    an I_n x prod I_p matrix of independent entries of that size."""
    e2 = 0.0
    for a in range(0, I, 100):
        e2 += float(np.sum((Yb[a:a + 100] - host["Y64"][a:a + 100]) ** 2))
    rms = np.sqrt(e2 / Yb.size)
    Gt = oracle["tk"]["Gt"]
    out = []
    for n in range(N):
        sv = np.linalg.svd(np.moveaxis(Gt, n, 0).reshape(RT_, -1), compute_uv=False)
        gap = sv[R - 1] - sv[R]
        s_n = rms * (np.sqrt(I) + np.sqrt(I * I))
        out.append(s_n / (gap - s_n))
    print(f"BF16 rounding: rms {rms:.3e}, Wedin estimates {out}", flush=True)
    return out


def test_fullsize_plain_fp32(P, work, host, oracle):
    out = run(P, work, "f32")
    out["_omt2"] = work["omt_d"][1]
    for n in range(N):      # sweep 1: the oracle's own sketches
        e = maxrel(dev64(out["trace"]["Z"][n]), oracle["tk"]["Z"][0][n])
        assert e <= TOL_Z, ("sweep-1 Z vs oracle", n, e)
    check_properties(out, host, host["Y64"], bf16=False)
    d, eG = errors_vs_oracle(out, oracle)
    assert max(d) <= 1e-4 and eG <= 1e-4, (d, eG)


def test_fullsize_precision_form(P, work, host, oracle):
    ybf16 = torch.empty(P.bf16_copy_shape((I, I, I)), dtype=torch.int16, device="cuda")
    assert ybf16.shape == (I, I, 1024)
    out = run(P, work, "bf16", ybf16=ybf16)
    out["_omt2"] = work["omt_d"][1]
    # every slab's largest |Y| has its binary exponent inside [-100, 100],
    # so the copy is bf16_rne(Y) with no scale
    mx = float(work["Y"].abs().amax())
    mn = float(work["Y"].abs().amax(dim=(1, 2)).min())
    assert -100 <= np.frexp(mn)[1] - 1 and np.frexp(mx)[1] - 1 <= 100
    Yb = host_f64(work["Y"], bf16=True)
    om = [o.astype(np.float64) for o in work["om32"]]
    omt1 = [o.astype(np.float64) for o in work["omt32"][0]]
    Zx = path_sketches(Yb, om, omt1, bf16=True)
    for n in range(N):
        e = maxrel(dev64(out["trace"]["Z"][n]), Zx[n])
        assert e <= TOL_Z, ("sweep-1 Z vs exact-input FP64", n, e)
    check_properties(out, host, Yb, bf16=True)
    bound = rounding_bounds(host, Yb, oracle)
    del Yb
    d, eG = errors_vs_oracle(out, oracle)
    for n in range(N):
        assert d[n] <= 2.0 * bound[n], ("d(U_n) vs FP64 oracle", n, d[n], bound[n])
    assert eG <= 2.0 * float(np.sqrt(np.sum(np.square(bound)))) + 2.0 ** -9, (eG, bound)
    # the BF16 copy of sampled slabs, bit for bit, padding zero
    got = out["ybf16"]
    for a in (0, 123, 999):
        Y32 = work["Y"][a].cpu().numpy()
        want = bf16_round(Y32).astype(np.float32).view(np.uint32) >> 16
        row = got[a].cpu().numpy().view(np.uint16)
        assert np.array_equal(row[:, :I], want.astype(np.uint16)), a
        assert not row[:, I:].any(), a


@pytest.mark.parametrize("precision", ["f32", "bf16"])
def test_fullsize_ffcp_fit_vs_oracle(P, work, oracle, precision):
    out = run(P, work, precision)
    f = P.ffcp(out["U"], out["G"], R, update="als", init="hosvd", max_it=1000, tol=1e-7,
               fit_trace=True)
    fits = f["fits"]
    it = int(f["info"]["iterations"])
    assert f["info"]["converged"] == 1 and it == len(fits)
    assert np.all(np.diff(fits) >= -1e-9)          # ALS never lowers the fit
    assert abs(fits[-1] - fits[-2]) < 1e-7
    for n in range(2):   # unit columns for n < N; lambda carries the scale
        A = dev64(f["A"][n])
        np.testing.assert_allclose(np.linalg.norm(A, axis=0), 1.0, atol=1e-5)
    fit_y = P.cp_fit_dense(work["Y"], f["A"], f["lam"])[0]
    tol = 1e-5 if precision == "f32" else 1e-4
    assert abs(fit_y - oracle["fit_y"]) <= tol, (fit_y, oracle["fit_y"])
