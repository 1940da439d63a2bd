"""Plain FP64 CPU oracle for randomized Tucker compression and FFCP.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
helpers with the HIP library; both sides only consume the same seeded inputs
from ``synth``.

Everything here is written for readability against the paper (Zhou,
Cichocki, Xie, "Decomposition of Big Tensors With Low Multilinear Rank"):
unfoldings, mode products and Khatri-Rao products are spelled out with NumPy
library primitives (tensordot, reshape, matmul, LAPACK QR / symmetric eig),
with no blocking, fusion or reordering beyond what the paper states.

Layout convention: tensors are row-major (last index fastest).  The mode-n
unfolding Y_(n) has I_n rows; its columns run over the remaining indices in
increasing mode order with the last one fastest.  Every quantity is defined
index-wise, so this choice does not change any result.

Parity status per function is listed in each module header.
"""

from . import tensor, randtucker, ffcp, metrics, mlp, rng  # noqa: F401
