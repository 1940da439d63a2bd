"""C-ABI tests that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid descriptions on the host before any
device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1412_1885_amd as P
from paper_1412_1885_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f)
           for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(rt_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = declared_functions()
    assert "rt_tucker_rand" in names and "rt_ffcp" in names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_version_and_status_strings():
    assert "gfx950" in P.version()
    assert P.status_string(0) == "RT_OK"
    assert P.status_string(-1) == "RT_ERR_INVALID_ARG"
    assert P.status_string(-3) == "RT_ERR_WORKSPACE"


def _ws(desc):
    n = ctypes.c_size_t(0)
    rc = P.lib().rt_tucker_rand_workspace(ctypes.byref(desc), ctypes.byref(n))
    return rc, n.value


def test_tucker_workspace_validation():
    ok = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7], sweeps=2)
    rc, n = _ws(ok)
    assert rc == 0 and n > 0
    bad_cases = []
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7]); d.N = 1
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7]); d.sweeps = 3
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 13])   # R_n > R~_n
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 8], [10, 11, 12], [5, 6, 7])     # R~_n > I_n
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 60], [10, 11, 65], [5, 6, 7])    # R~ > 64
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7]); d.precision = 7
    bad_cases.append(d)
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7], precision="f32",
                      bf16_input=True)
    bad_cases.append(d)
    for d in bad_cases:
        rc, _ = _ws(d)
        assert rc == B.RT_F32 - 1, P.last_error()      # RT_ERR_INVALID_ARG
        assert P.last_error()


def test_bf16_shapes_checked_at_validation():
    """The BF16 streaming pass needs I_N % 4 == 0, I_{N-1} <= 1024 and the
    two streamed sketch widths <= 32: rejected before anything is launched."""
    n = ctypes.c_size_t(0)
    ok = P.tucker_desc([4, 20, 32], [4, 5, 5], [3, 3, 3], precision="bf16")
    assert P.lib().rt_tucker_rand_workspace(ctypes.byref(ok), ctypes.byref(n)) == 0
    for dims, rt in (([4, 20, 30], [4, 5, 5]),        # I_N % 4 != 0
                     ([4, 1100, 32], [4, 5, 5]),      # I_{N-1} > 1024
                     ([4, 40, 64], [4, 5, 33])):      # streamed width > 32
        d = P.tucker_desc(dims, rt, [3, 3, 3], precision="bf16")
        rc = P.lib().rt_tucker_rand_workspace(ctypes.byref(d), ctypes.byref(n))
        assert rc == -2, (dims, rt, rc)   # RT_ERR_UNSUPPORTED
        assert "BF16" in P.last_error()


def test_bf16_copy_length():
    """The BF16 copy's rows are padded to a multiple of 64 values; no copy in
    the other forms or for a caller's BF16 tensor."""
    n = ctypes.c_int64(-1)
    L = P.lib()
    for dims, want in (([1000, 1000, 1000], 1000 * 1000 * 1024),
                       ([6, 40, 56], 6 * 40 * 64), ([3, 5, 7, 128], 3 * 5 * 7 * 128),
                       ([2, 3, 68], 2 * 3 * 128)):
        d = P.tucker_desc(dims, [2] * len(dims), precision="bf16")
        assert L.rt_tucker_bf16_copy_elems(ctypes.byref(d), ctypes.byref(n)) == 0
        assert n.value == want, dims
        assert P.bf16_copy_shape(dims) == tuple(dims[:-1]) + (want // np.prod(dims[:-1]),)
    for d in (P.tucker_desc([6, 40, 56], [2, 2, 2], precision="f32"),
              P.tucker_desc([6, 40, 56], [2, 2, 2], precision="bf16", bf16_input=True)):
        assert L.rt_tucker_bf16_copy_elems(ctypes.byref(d), ctypes.byref(n)) == 0
        assert n.value == 0
    d = P.tucker_desc([6, 40, 56], [2, 2, 2], precision="bf16")
    assert L.rt_tucker_bf16_copy_elems(ctypes.byref(d), None) == -1
    d.N = 1
    assert L.rt_tucker_bf16_copy_elems(ctypes.byref(d), ctypes.byref(n)) == -1


def test_gauss_seidel_order_accepted():
    """RT_FLAG_GAUSS_SEIDEL selects the printed loop order of Algorithm 3;
    the workspace is the Jacobi form's (the same buffers, used in turn)."""
    d = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7], order="gauss_seidel")
    assert d.flags & B.RT_FLAG_GAUSS_SEIDEL
    rc, n_gs = _ws(d)
    rc2, n_j = _ws(P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7]))
    assert rc == 0 and rc2 == 0 and n_gs == n_j
    with pytest.raises(ValueError):
        P.tucker_desc([4, 5, 6], [2, 2, 2], order="random")


def test_tucker_rand_rejects_null_and_misaligned_pointers_before_launch():
    d = P.tucker_desc([4, 5, 6], [2, 2, 2], [1, 1, 1])
    vp = ctypes.c_void_p
    arr = (vp * 3)(16, 32, 48)
    rc = P.lib().rt_tucker_rand(ctypes.byref(d), None, arr, arr, vp(64), 1 << 20,
                                arr, vp(80), None, None, None, None)
    assert rc == -1 and "Y" in P.last_error()
    rc = P.lib().rt_tucker_rand(ctypes.byref(d), vp(8), arr, arr, vp(64), 1 << 20,
                                arr, vp(80), None, None, None, None)
    assert rc == -1 and "aligned" in P.last_error()


def test_ffcp_validation():
    n = ctypes.c_size_t(0)
    d = P.ffcp_desc([30, 40, 50], [5, 6, 7], 4, "hals")
    assert P.lib().rt_ffcp_workspace(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value > 0
    for mutate in (lambda d: setattr(d, "R", 0), lambda d: setattr(d, "R", 65),
                   lambda d: setattr(d, "update", 5), lambda d: setattr(d, "max_it", 0),
                   lambda d: setattr(d, "tol", -1.0)):
        d = P.ffcp_desc([30, 40, 50], [5, 6, 7], 4)
        mutate(d)
        assert P.lib().rt_ffcp_workspace(ctypes.byref(d), ctypes.byref(n)) == -1
    d = P.ffcp_desc([30, 4, 50], [5, 6, 7], 4)   # R_n > I_n
    assert P.lib().rt_ffcp_workspace(ctypes.byref(d), ctypes.byref(n)) == -1


def test_workspace_too_small_reported():
    d = P.tucker_desc([4, 5, 6], [2, 2, 2], [1, 1, 1])
    vp = ctypes.c_void_p
    arr = (vp * 6)(*[256 * (i + 1) for i in range(6)])
    rc = P.lib().rt_tucker_rand(ctypes.byref(d), vp(4096), arr, arr, vp(8192), 16,
                                arr, vp(12288), None, None, None, None)
    assert rc == -3 and "workspace" in P.last_error()


def test_mlp_descriptor_validation():
    n = ctypes.c_size_t(0)
    d = P.mlp_desc(16, (20, 20, 20), 20)
    assert P.lib().rt_mlp_workspace(ctypes.byref(d), ctypes.byref(n)) == 0 and n.value > 0
    d = P.mlp_desc(16, (20, 20, 20, 20), 20)          # order 4
    assert P.lib().rt_mlp_workspace(ctypes.byref(d), ctypes.byref(n)) == -2
    d = P.mlp_desc(16, (20, 20, 20), 40)              # R > 32
    assert P.lib().rt_mlp_workspace(ctypes.byref(d), ctypes.byref(n)) == -1
    d = P.mlp_desc(16, (20, 20, 20), 20, hidden=(100, 64))   # width not a multiple of 8
    assert P.lib().rt_mlp_workspace(ctypes.byref(d), ctypes.byref(n)) == -1


def test_bf16_slab_count_checked_at_validation():
    """The conversion's one-dimensional grid holds every (slab, block) pair:
    300^4 (90,000 slabs) is accepted; a shape needing more than 2^31 - 1
    blocks is rejected on the host before anything is launched."""
    n = ctypes.c_size_t(0)
    ok = P.tucker_desc([300, 300, 300, 300], [4, 4, 4, 4], [2, 2, 2, 2], precision="bf16")
    assert P.lib().rt_tucker_rand_workspace(ctypes.byref(ok), ctypes.byref(n)) == 0
    big = P.tucker_desc([2 ** 22, 2 ** 11, 1024, 4], [2, 2, 2, 2], [1, 1, 1, 1],
                        precision="bf16")
    assert P.lib().rt_tucker_rand_workspace(ctypes.byref(big), ctypes.byref(n)) == -2
    assert "blocks" in P.last_error()


def _dense_descs(**kw):
    td = P.tucker_desc([40, 50, 60], [10, 11, 12], [5, 6, 7], sweeps=2)
    fd = P.ffcp_desc([40, 50, 60], [5, 6, 7], 4, "als", "hosvd")
    for k, v in kw.items():
        setattr(td, k, v)
    return td, fd


def test_ffcp_dense_workspace_and_validation():
    """rt_ffcp_dense: its workspace holds both stages; the FFCP description
    must match the Tucker output and the compression must be FP32-output."""
    L = P.lib()
    n, nt, nf = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
    td, fd = _dense_descs()
    assert L.rt_ffcp_dense_workspace(ctypes.byref(td), ctypes.byref(fd), ctypes.byref(n)) == 0
    assert L.rt_tucker_rand_workspace(ctypes.byref(td), ctypes.byref(nt)) == 0
    assert L.rt_ffcp_workspace(ctypes.byref(fd), ctypes.byref(nf)) == 0
    assert n.value >= nt.value + nf.value
    td, fd = _dense_descs()
    fd.ranks[1] = 7                                   # not the Tucker output rank
    assert L.rt_ffcp_dense_workspace(ctypes.byref(td), ctypes.byref(fd), ctypes.byref(n)) == -1
    assert "differs" in P.last_error()
    td, fd = _dense_descs(precision=2)                # FP64 compression
    assert L.rt_ffcp_dense_workspace(ctypes.byref(td), ctypes.byref(fd), ctypes.byref(n)) == -2
    td, fd = _dense_descs()
    vp = ctypes.c_void_p
    arr = (vp * 6)(*[256 * (i + 1) for i in range(6)])
    # a NULL lambda is rejected before the compression is enqueued
    rc = L.rt_ffcp_dense(ctypes.byref(td), ctypes.byref(fd), vp(4096), arr, arr, None,
                         None, None, vp(1 << 20), n.value, arr, None, None, None, None,
                         None)
    assert rc == -1 and "lambda" in P.last_error()


def test_ffcp_noalloc_rejects_oversized_problems_on_the_host():
    """rt_ffcp_noalloc checks the description and the static scratch's size
    limit before touching a device."""
    L = P.lib()
    vp = ctypes.c_void_p
    arr = (vp * 4)(*[256 * (i + 1) for i in range(4)])
    big = P.ffcp_desc([40000] * 4, [20] * 4, 20, "hals")
    rc = L.rt_ffcp_noalloc(ctypes.byref(big), arr, vp(4096), arr, None, arr, vp(8192),
                           None, None, None)
    assert rc == -2 and "scratch" in P.last_error()
    bad = P.ffcp_desc([30, 40, 50], [5, 6, 7], 4)
    bad.R = 0
    rc = L.rt_ffcp_noalloc(ctypes.byref(bad), arr, vp(4096), arr, None, arr, vp(8192),
                           None, None, None)
    assert rc == -1
