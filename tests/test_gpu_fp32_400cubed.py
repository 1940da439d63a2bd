"""The plain FP32 path on its own workload, the 400 x 400 x 400 FP32 tensor
(64M entries) of a CP model of rank 20 with per-mode column congruence drawn
from U[0, 0.5] and Gaussian noise at SNR 20 dB (Section V-A's recipe):
Omega_n 400 x 30, Omega~_n 900 x 30, one sweep, Tucker ranks (20, 20, 20),
then FFCP-ALS to a fit change below 1e-7.

The FP64 oracle runs the whole method on the same FP32 tensor and the same
Omega (a fraction of a second per step at this size), so everything is
compared with it directly:

* sketches Z_n element-wise, 1e-5 of max |Z_n| (each entry sums 1.6e5
  products accumulated in FP32 in stages of at most 400 and 480 terms:
  (400 + 480 + 40) u ~ 5e-5 of the terms' magnitudes at worst, about
  sqrt(920) u ~ 2e-6 typically);
* U_n by projector distance, the core after alignment: 1e-4 (the
  truncation divides the FP32 rounding of G~ by eigen-gaps of O(1)
  relative size);
* FFCP from the same FP32 start: the first 10 iterates (factors after each
  iteration, columns normalized) within 1e-4 relative, the converged
  factors' congruence with the oracle's >= 1 - 1e-4 after matching, and
  Fit_Y within 1e-5.
"""

import numpy as np
import pytest

import synth
from oracle import ffcp as F
from oracle import randtucker as RT
from oracle.metrics import aligned_core_error, factor_congruence, projector_distance

from _fullsize import dev64, maxrel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT_, N = 400, 20, 30, 3


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


@pytest.fixture(scope="module")
def case():
    d = synth.case_cp_congruent(400, (I, I, I), R, 0.0, 0.5, 20.0, (RT_,) * 3)
    Y32 = synth.f32(d["Y"])
    om32 = synth.f32(d["omegas"])
    omt32 = synth.f32(d["omega_tildes"][0])
    A0 = synth.f32(synth.init_factors(d["init_rng"], (I, I, I), R))
    Y64 = Y32.astype(np.float64)
    tk = RT.rand_tucker(Y64, [o.astype(np.float64) for o in om32],
                        [[o.astype(np.float64) for o in omt32]], sweeps=1,
                        ranks=(R, R, R))
    return {"Y32": Y32, "Y64": Y64, "om32": om32, "omt32": omt32,
            "A0": [a.astype(np.float64) for a in A0], "tk": tk}


@pytest.fixture(scope="module")
def gpu(P, case):
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    Y = up(case["Y32"])
    out = P.tucker_rand(Y, [up(o) for o in case["om32"]], [[up(o) for o in case["omt32"]]],
                        ranks=(R, R, R), sweeps=1, trace=True)
    return {"Y": Y, "out": out, "up": up}


def test_400cubed_tucker_vs_oracle(P, case, gpu):
    out, tk = gpu["out"], case["tk"]
    for n in range(N):
        e = maxrel(dev64(out["trace"]["Z"][n]), tk["Z"][0][n])
        assert e <= 1e-5, ("Z", n, e)
    U = [dev64(u) for u in out["U"]]
    for n in range(N):
        d = projector_distance(U[n], tk["U"][n])
        assert d <= 1e-4, ("U", n, d)
    eG = aligned_core_error(dev64(out["G"]), U, tk["G"], tk["U"])
    assert eG <= 1e-4, eG
    y2 = float(np.sum(case["Y64"] ** 2))
    assert abs(out["info"]["normY2"] - y2) <= 1e-12 * y2


def _gpu_ffcp(P, gpu, case, max_it, tol):
    up = gpu["up"]
    return P.ffcp(gpu["out"]["U"], gpu["out"]["G"], R, update="als",
                  A_init=[up(a) for a in case["A0"]], max_it=max_it, tol=tol,
                  fit_trace=True)


def _unit(A, lam):
    """Columns normalized in every mode (the scale moved out)."""
    return [a / np.linalg.norm(a, axis=0) for a in A]


def test_400cubed_ffcp_first_iterates(P, case, gpu):
    """Both sides start from the same FP32 factors; their Tucker formats
    differ only by FP32 rounding, so the iterates agree to ~1e-5."""
    U = [np.asarray(u, np.float64) for u in case["tk"]["U"]]
    G = case["tk"]["G"]
    for k in range(1, 11):
        f = _gpu_ffcp(P, gpu, case, k, 0.0)
        ref = F.ffcp(U, G, case["A0"], update="als", max_it=k, tol=0.0)
        got = _unit([dev64(a) for a in f["A"]], None)
        want = _unit(ref["A"], None)
        for n in range(N):
            e = float(np.linalg.norm(got[n] - want[n]) / np.linalg.norm(want[n]))
            assert e <= 1e-4, (k, n, e)
        lam_e = float(np.linalg.norm(dev64(f["lam"]) - ref["lam"]) /
                      np.linalg.norm(ref["lam"]))
        assert lam_e <= 1e-4, (k, lam_e)


@pytest.mark.parametrize("start", ["random", "hosvd"])
def test_400cubed_ffcp_converged_vs_oracle(P, case, gpu, start):
    """To the stop rule from the same FP32 random start, and from each side's
    HOSVD start of its own core."""
    U = [np.asarray(u, np.float64) for u in case["tk"]["U"]]
    G = case["tk"]["G"]
    if start == "random":
        f = _gpu_ffcp(P, gpu, case, 1000, 1e-7)
        ref = F.ffcp(U, G, case["A0"], update="als", max_it=1000, tol=1e-7)
    else:
        f = P.ffcp(gpu["out"]["U"], gpu["out"]["G"], R, update="als", init="hosvd",
                   max_it=1000, tol=1e-7, fit_trace=True)
        ref = F.ffcp(U, G, F.hosvd_init(U, G, R), update="als", max_it=1000, tol=1e-7)
    assert f["info"]["converged"] == 1 and ref["converged"]
    assert abs(int(f["info"]["iterations"]) - ref["iterations"]) <= 3
    _, cong = factor_congruence([dev64(a) for a in f["A"]], ref["A"])
    assert cong >= 1 - 1e-4, cong
    fit_gpu = P.cp_fit_dense(gpu["Y"], f["A"], f["lam"])[0]
    fit_ref = F.cp_fit_mttkrp(case["Y64"], ref["A"], ref["lam"])
    assert abs(fit_gpu - fit_ref) <= 1e-5, (fit_gpu, fit_ref)
