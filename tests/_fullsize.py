"""Host-side FP64 helpers of the full-size parity tests.

The library's streaming passes contract the last mode (TA = Y x_N B_N^T) and
the next-to-last mode (TB = Y x_{N-1} B_{N-1}^T) in one read of Y; every
mode's sketch is then finished on those shrunk tensors: X_n from TA for
n < N (the other modes contracted with their FP32 bases), X_N from TB.  In
the precision form the streamed operands are BF16 (Y's copy and the streamed
basis); everything after them is FP32.  The functions here recompute those
quantities in FP64 from given operands, with the BF16 rounding written here
(round to nearest even), independently of the library.
"""

import numpy as np

from oracle import tensor as T


def bf16_round(x):
    """FP32 values rounded to BF16 (nearest even), returned as FP64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def host_f64(Y, bf16=False, rows=50):
    """Device FP32 tensor -> host FP64 array, mode-1 slab by slab (optionally
    rounded to BF16 first)."""
    out = np.empty(tuple(Y.shape), dtype=np.float64)
    for a in range(0, Y.shape[0], rows):
        blk = Y[a:a + rows].cpu().numpy()
        out[a:a + rows] = bf16_round(blk) if bf16 else blk
    return out


def path_sketches(Y, bases, omt, bf16=False):
    """Z_n = X_(n) Omega~_n with X_n = Y x_{p != n} B_p^T contracted in the
    library's order: the streamed factor B_N (for n < N) or B_{N-1} (for
    n = N) first, rounded to BF16 when bf16 (Y must then hold the BF16
    values), the other modes with the given FP32 values.  All FP64."""
    N = Y.ndim
    last, second = N - 1, N - 2
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    TA = T.ttm_t(Y, rnd(bases[last]), last)
    TB = T.ttm_t(Y, rnd(bases[second]), second)
    Z = []
    for n in range(N):
        src, skip = (TA, (n, last)) if n != last else (TB, (last, second))
        X = T.multi_ttm_t(src, [None if p in skip else np.asarray(bases[p], np.float64)
                                for p in range(N)])
        Z.append(T.unfold(X, n) @ np.asarray(omt[n], np.float64))
    return Z


def path_core(Y, Q, bf16=False):
    """G~ = Y x_1 Q_1^T ... x_N Q_N^T with the last mode first (in BF16 when
    bf16, Y then holding the BF16 values), the rest with FP32 values."""
    N = Y.ndim
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    X = T.ttm_t(Y, rnd(Q[N - 1]), N - 1)
    return T.multi_ttm_t(X, [np.asarray(q, np.float64) for q in Q[:N - 1]] + [None])


def maxrel(a, b):
    """max |a - b| / max |b| (element-wise error over the result's scale)."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev64(t):
    return t.detach().cpu().numpy().astype(np.float64)
