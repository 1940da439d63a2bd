"""Counter-based Gaussian numbers for the dense test matrices of sequential
RandTucker (Alg. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The generator is Philox4x32 with 10 rounds, as defined by Salmon, Moraes,
Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): a
128-bit counter (four 32-bit words) and a 64-bit key (two words); a round
multiplies words 0 and 2 by two fixed odd constants into 64-bit products and
recombines their halves with words 1 and 3 and the key; the key is advanced
by two fixed constants (the golden ratio's and sqrt(3) - 1's 32-bit
fractions) before every round after the first.  Because each output depends
only on (counter, key), every entry of a test matrix can be produced where
it is needed, in any order, on any device (the parameter broadcast Section
IV-B describes for distributed generation).

Entry (r, k) of the test matrix of mode n (r the row, in the row-major order
of the other modes' indices):
    counter = (r mod 2^32, r div 2^32, k, n),  key = (seed mod 2^32, seed div 2^32)
    u1 = (x0 + 1) 2^-32 in (0, 1],  u2 = (x1 + 1/2) 2^-32 in (0, 1)
    value = sqrt(-2 ln u1) cos(2 pi u2)        (Box-Muller, FP64)
with x0, x1 the first two output words.

Pins: tests/test_oracle_rng.py (the round function against its definition
written out by words on single inputs; bijectivity of the round on sampled
inputs; distribution of the outputs: uniform words, standard normal values,
no correlation between neighbouring counters).
"""

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)


def philox_round(c, k):
    """One Philox4x32 round: c = (c0, c1, c2, c3), k = (k0, k1), arrays of
    uint64 holding 32-bit values."""
    c0, c1, c2, c3 = c
    k0, k1 = k
    p0 = _M0 * c0            # < 2^64: exact in uint64
    p1 = _M1 * c2
    hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
    hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
    return (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)


def philox4x32_10(c, k):
    """Ten rounds, the key advanced before every round after the first."""
    c = tuple(np.asarray(x, dtype=np.uint64) & _MASK for x in c)
    k0, k1 = (np.asarray(x, dtype=np.uint64) & _MASK for x in k)
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        c = philox_round(c, (k0, k1))
    return c


def gaussian_matrix(rows, cols, mode, seed):
    """The rows x cols test matrix of the given mode (FP64)."""
    r = np.arange(rows, dtype=np.uint64)[:, None] * np.ones((1, cols), dtype=np.uint64)
    kk = np.ones((rows, 1), dtype=np.uint64) * np.arange(cols, dtype=np.uint64)[None, :]
    seed = np.uint64(seed)
    x = philox4x32_10((r & _MASK, r >> np.uint64(32), kk,
                       np.full(r.shape, mode, dtype=np.uint64)),
                      (seed & _MASK, seed >> np.uint64(32)))
    u1 = (x[0].astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = (x[1].astype(np.float64) + 0.5) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def sequential_omegas(dims, ranks_tilde, seed):
    """The dense test matrices of Alg. 2 on a tensor of these dims: mode n
    sees the earlier modes already shrunk to R~_k, so its matrix has
    prod_{k<n} R~_k prod_{k>n} I_k rows and R~_n columns."""
    out = []
    for n in range(len(dims)):
        rows = 1
        for k in range(len(dims)):
            if k != n:
                rows *= ranks_tilde[k] if k < n else dims[k]
        out.append(gaussian_matrix(rows, ranks_tilde[n], n, seed))
    return out
