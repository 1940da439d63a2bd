"""FFCP on long modes (I_n >= 2048): the iteration runs over the whole chip
(one cooperative launch, each workgroup owning a chunk of every mode's rows,
cross products summed from per-workgroup partials in a fixed order).  Same
iterate parity as the single-workgroup cases: 12 iterations from the same
start against the FP64 oracle, fits to 1e-9, factors to 1e-6 element-wise
over scale (FP32 output), lambda, and the ridge flag.  Each case was checked
on the CPU to be well posed: a 1e-13 relative change of the start moves the
oracle's fits by < 2e-13 and its factors by < 2e-11.  The 10^4-per-mode
HALS workload is covered in test_gpu_hals_1e4.py."""

import numpy as np
import pytest

import synth

from test_gpu_parity import P, _check_iterates, _iterate_case, _tucker_format, seed_of  # noqa: F401

pytestmark = pytest.mark.gpu

GRID_CASES = [("hals", (3000, 2100, 2500), (6, 6, 6), 5, "random"),
              ("mu", (2500, 2048, 3000), (6, 6, 6), 5, "random"),
              ("hals", (2048, 2100, 2200), (20, 20, 20), 20, "near"),
              ("mu", (2048, 2100, 2200), (20, 20, 20), 20, "near")]


@pytest.mark.parametrize("rule,dims,ranks,R,start", GRID_CASES,
                         ids=[f"{c[0]}-R{c[3]}" for c in GRID_CASES])
def test_ffcp_grid_iterates(P, rule, dims, ranks, R, start):
    G, U, A0 = _iterate_case(rule, dims, ranks, R, start)
    _check_iterates(P, rule, G, U, A0, R)


# the soft threshold on long modes: ALS (the general kernel's Cholesky path,
# which ends in the ridge on this case, as the oracle does) and HALS
GRID_L1_CASES = [("als", (2048, 2500, 2100), 5, 0.02), ("hals", (2100, 2048, 2300), 5, 0.05)]


@pytest.mark.parametrize("rule,dims,R,c", GRID_L1_CASES,
                         ids=[f"{c[0]}-c{c[3]}" for c in GRID_L1_CASES])
def test_ffcp_grid_l1_iterates(P, rule, dims, R, c):
    G, U, g, A = _tucker_format(seed_of("l1", rule, dims, R), dims, (R,) * len(dims),
                                True, with_factors=True)
    A0 = [synth.f32(a * g.uniform(0.5, 1.5, a.shape)).astype(np.float64) for a in A]
    out, ref = _check_iterates(P, rule, G, U, A0, R, iters=12, l1=c)
    small = sum(int(np.sum(np.abs(a) <= 1e-16)) for a in ref["A"])
    assert small > 0            # the threshold did act
