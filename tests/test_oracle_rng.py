"""Pins for oracle/rng.py (the counter-based Gaussian test matrices of
sequential RandTucker, Alg. 2).

The generator's exact output values are parity unpinned: no printed values
of the published generator are used here.  What is pinned is that the code
does what its definition says, word by word, and that its outputs have the
distribution Alg. 2 needs (independent standard normal entries)."""

import numpy as np
from scipy import stats

from oracle import randtucker as RT
from oracle import rng as G
from oracle import tensor as T

MASK = (1 << 32) - 1


def round_by_words(c, k):
    """One round computed with Python integers (arbitrary precision), the
    64-bit products split into their high and low words."""
    p0 = 0xD2511F53 * c[0]
    p1 = 0xCD9E8D57 * c[2]
    return ((p1 >> 32) ^ c[1] ^ k[0], p1 & MASK, (p0 >> 32) ^ c[3] ^ k[1], p0 & MASK)


def test_round_matches_its_definition():
    rng = np.random.default_rng(1)
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        got = G.philox_round(tuple(np.uint64(x) for x in c), tuple(np.uint64(x) for x in k))
        assert tuple(int(x) for x in got) == round_by_words(c, k)


def test_ten_rounds_with_key_schedule():
    """Ten rounds: the key advances by (0x9E3779B9, 0xBB67AE85) mod 2^32
    before rounds 2..10."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        k = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        want = tuple(c)
        for r in range(10):
            kr = ((k[0] + r * 0x9E3779B9) & MASK, (k[1] + r * 0xBB67AE85) & MASK)
            want = round_by_words(want, kr)
        got = G.philox4x32_10(tuple(np.uint64(x) for x in c), tuple(np.uint64(x) for x in k))
        assert tuple(int(x) for x in got) == want


def test_round_is_a_bijection_on_samples():
    """A round is invertible (the odd multipliers make the products' low
    words bijective): distinct counters never collide."""
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2 ** 32, (4, 200000), dtype=np.uint64)
    c[0] = np.arange(200000, dtype=np.uint64)        # distinct inputs
    out = G.philox_round(tuple(c), (np.uint64(7), np.uint64(9)))
    assert len(np.unique(out[3])) == 200000         # lo0 is a bijection of c0


def test_words_are_uniform():
    x = G.philox4x32_10((np.arange(100000, dtype=np.uint64), np.zeros(100000, np.uint64),
                         np.zeros(100000, np.uint64), np.zeros(100000, np.uint64)),
                        (np.uint64(123), np.uint64(0)))
    for w in x:
        u = w.astype(np.float64) / 2.0 ** 32
        assert stats.kstest(u, "uniform").pvalue > 1e-3
        bits = np.unpackbits(w.astype(">u4").view(np.uint8))
        assert abs(bits.mean() - 0.5) < 0.005


def test_gaussian_matrix_is_standard_normal_and_uncorrelated():
    Om = G.gaussian_matrix(20000, 30, 2, 14121885)
    assert Om.shape == (20000, 30)
    v = Om.reshape(-1)
    assert abs(v.mean()) < 0.01 and abs(v.std() - 1.0) < 0.01
    assert stats.kstest(v, "norm").pvalue > 1e-3
    C = np.corrcoef(Om.T)
    assert np.max(np.abs(C - np.eye(30))) < 0.04
    # neighbouring rows, other modes and other seeds are unrelated
    B = G.gaussian_matrix(20000, 30, 3, 14121885)
    D = G.gaussian_matrix(20000, 30, 2, 14121886)
    for X in (B, D):
        assert abs(np.corrcoef(v, X.reshape(-1))[0, 1]) < 0.02
    assert abs(np.corrcoef(Om[:-1].reshape(-1), Om[1:].reshape(-1))[0, 1]) < 0.02


def test_entries_depend_only_on_their_counter():
    """Any block of a test matrix equals the same block of a larger one."""
    A = G.gaussian_matrix(500, 12, 1, 99)
    B = G.gaussian_matrix(300, 7, 1, 99)
    assert np.array_equal(A[:300, :7], B)


def test_sequential_randtucker_with_counter_gaussians_recovers_exact_rank():
    """Alg. 2 with these test matrices recovers a noise-free tensor of
    multilinear rank below the sketch widths exactly."""
    rng = np.random.default_rng(4)
    dims, ranks, rt = (20, 24, 28), (3, 4, 5), (6, 7, 8)
    Gc = rng.standard_normal(ranks)
    U = [np.linalg.qr(rng.standard_normal((I, r)))[0] for I, r in zip(dims, ranks)]
    Y = T.tucker_full(Gc, U)
    Om = G.sequential_omegas(dims, rt, 2024)
    assert [o.shape for o in Om] == [(24 * 28, 6), (6 * 28, 7), (6 * 7, 8)]
    Uh, Gh = RT.rand_tucker_sequential(Y, Om)
    assert np.linalg.norm(Y - T.tucker_full(Gh, Uh)) <= 1e-12 * np.linalg.norm(Y)
