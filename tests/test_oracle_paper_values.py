"""Oracle against values the paper prints (tests/golden/)."""

import json
import os

import numpy as np
import pytest

import synth
from oracle import ffcp as F
from oracle import randtucker as RT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.slow
def test_table3_ffcp_hals_in_distribution():
    """Table III, FFCP-HALS, N=3, I=200, R=10: mean Fit(Y*, Yhat) 99.1 +- 0.1 %.
    Our random numbers differ from the paper's, so the check is in
    distribution: the mean over 2 runs within 4 printed standard deviations."""
    ref = json.load(open(os.path.join(GOLDEN, "paper_table3.json")))
    fits = []
    for s in range(2):
        dims, R = (200, 200, 200), 10
        g = synth.rngs((200, s))
        A = synth.nonneg_factors(g["factors"], dims, R, "exp", 10.0, 0.1)
        Ys = synth.cp_tensor(A)
        Y = synth.add_gaussian_noise(Ys, g["noise"], 10.0)
        U, G = RT.hosvd(Y, (R, R, R))
        A0 = synth.init_factors(g["init"], dims, R, nonneg=True)
        out = F.ffcp(U, G, A0, update="hals", max_it=1000, tol=1e-6)
        fits.append(F.cp_fit_dense(Ys, out["A"], out["lam"]))
    assert abs(np.mean(fits) - ref["fit_mean"]) <= 4 * ref["fit_std"]
