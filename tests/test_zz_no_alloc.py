"""rt_ffcp_noalloc (rt_ffcp with the library's static per-GPU scratch instead
of a caller workspace) against rt_ffcp on the same inputs, through the C ABI.

Both run the same kernels on the same values in the same order, so the
factors, weights, fit traces and info must be bit-identical.  Each rule is
run twice in a row, the second problem smaller than the first, so the
second call finds the first call's values in the shared scratch.
"""

import ctypes

import numpy as np
import pytest

import synth
from oracle import tensor as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def _format(seed, dims, R):
    """Exact Tucker format of a nonnegative CP tensor (Section V-A's
    construction) and a U[0, 1] start."""
    g = np.random.default_rng(seed)
    A = [g.uniform(0, 1, (I, R)) for I in dims]
    U, Rs = [], []
    for a in A:
        q, r = np.linalg.qr(a)
        U.append(q)
        Rs.append(r)
    G = np.zeros((R,) * len(dims))
    for r in range(R):
        G[(r,) * len(dims)] = 1.0
    G = T.multi_ttm_t(G, [r_.T for r_ in Rs])
    A0 = [g.uniform(0, 1, (I, R)) for I in dims]
    dev = lambda a: torch.from_numpy(synth.f32(a)).cuda()
    return [dev(u) for u in U], dev(G), [dev(a) for a in A0]


CASES = {  # two problems per rule, the second smaller
    "als": [((300, 320, 340), 12, 9001), ((50, 60, 70), 5, 9002)],
    "hals": [((400, 420, 440), 10, 9003), ((40, 44, 48), 4, 9004)],
}


@pytest.mark.parametrize("rule", ["als", "hals"])
def test_noalloc_matches_workspace_entry_point(P, rule):
    for dims, R, seed in CASES[rule]:
        print(f"noalloc {rule} dims={dims} R={R} seed={seed}", flush=True)
        U, G, A0 = _format(seed, dims, R)
        kw = dict(update=rule, A_init=A0, max_it=25, tol=0.0, fit_trace=True)
        ref = P.ffcp(U, G, R, **kw)
        got = P.ffcp_noalloc(U, G, R, **kw)
        for n in range(len(dims)):
            assert torch.equal(got["A"][n], ref["A"][n]), (rule, dims, n)
        assert torch.equal(got["lam"], ref["lam"]), (rule, dims)
        assert np.array_equal(got["fits"], ref["fits"]), (rule, dims)
        assert got["info"].tobytes() == ref["info"].tobytes(), (rule, dims)
        assert int(got["info"]["iterations"]) == 25


def test_noalloc_hosvd_start(P):
    """The HOSVD start (eigensolver scratch in the same array) also matches."""
    U, G, _ = _format(9005, (60, 64, 68), 6)
    ref = P.ffcp(U, G, 6, update="als", init="hosvd", max_it=10, tol=0.0, fit_trace=True)
    got = P.ffcp_noalloc(U, G, 6, update="als", init="hosvd", max_it=10, tol=0.0,
                         fit_trace=True)
    for n in range(3):
        assert torch.equal(got["A"][n], ref["A"][n]), n
    assert np.array_equal(got["fits"], ref["fits"])


def test_noalloc_rejects_problems_above_its_scratch(P):
    """A problem whose workspace exceeds the static scratch is refused before
    anything is enqueued: the outputs stay untouched."""
    dims, R = (40000, 40000, 40000, 40000), 20
    need = P.ffcp_workspace(P.ffcp_desc(dims, (R,) * 4, R, "hals"))
    assert need > 32 << 20
    U = [torch.zeros((I, R), dtype=torch.float32, device="cuda") for I in dims]
    G = torch.zeros((R,) * 4, dtype=torch.float32, device="cuda")
    with pytest.raises(P.RtError) as e:
        P.ffcp_noalloc(U, G, R, update="hals", A_init=U, max_it=2, tol=0.0)
    assert e.value.status == -2 and "scratch" in str(e.value)
