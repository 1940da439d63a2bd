"""ctypes binding of librtucker (include/rtucker.h).

Argument marshalling only: every step of the method runs in the HIP library.
torch is used for device memory and the current stream.  If the library is
not built this module raises; there is no CPU fallback.
"""

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtucker.so")

RT_MAX_MODES = 8
RT_MAX_SKETCH = 64
RT_F32, RT_BF16_MIXED, RT_F64 = 0, 1, 2
RT_FLAG_NO_TRUNCATE, RT_FLAG_BF16_INPUT, RT_FLAG_GAUSS_SEIDEL = 1, 2, 4
RT_ALS, RT_HALS, RT_MU = 0, 1, 2
RT_INIT_USER, RT_INIT_HOSVD, RT_INIT_COEFF, RT_INIT_COEFF_GUARDED = 0, 1, 2, 3
INITS = {"user": RT_INIT_USER, "hosvd": RT_INIT_HOSVD, "coeff": RT_INIT_COEFF,
         "coeff_guarded": RT_INIT_COEFF_GUARDED}
PRECISIONS = {"f32": RT_F32, "bf16": RT_BF16_MIXED, "f64": RT_F64}
UPDATES = {"als": RT_ALS, "hals": RT_HALS, "mu": RT_MU}


class TuckerDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("dims", ctypes.c_int64 * RT_MAX_MODES),
                ("ranks", ctypes.c_int32 * RT_MAX_MODES),
                ("ranks_tilde", ctypes.c_int32 * RT_MAX_MODES)]


class TuckerTrace(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_void_p * (2 * RT_MAX_MODES)),
                ("Q", ctypes.c_void_p * (2 * RT_MAX_MODES)),
                ("Gt", ctypes.c_void_p)]


class FfcpDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("R", ctypes.c_int32),
                ("update", ctypes.c_int32), ("init", ctypes.c_int32),
                ("max_it", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double), ("l1", ctypes.c_double),
                ("normY2", ctypes.c_double),
                ("dims", ctypes.c_int64 * RT_MAX_MODES),
                ("ranks", ctypes.c_int32 * RT_MAX_MODES)]


TUCKER_INFO_DTYPE = np.dtype([("normY2", "<f8"), ("normG2", "<f8"),
                              ("nonfinite", "<i4"), ("rank_deficient", "<i4"),
                              ("reserved", "<i8", (2,))])
class MlpDesc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("N", ctypes.c_int32), ("R", ctypes.c_int32),
                ("hidden1", ctypes.c_int32), ("hidden2", ctypes.c_int32),
                ("core_dims", ctypes.c_int32 * 8)]


class SequentialDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64),
                ("dims", ctypes.c_int64 * RT_MAX_MODES),
                ("ranks_tilde", ctypes.c_int32 * RT_MAX_MODES)]


class MlpParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p * 3) for k in ("W", "b", "Wb", "mW", "vW", "mb", "vb")]


FFCP_INFO_DTYPE = np.dtype([("iterations", "<i4"), ("converged", "<i4"),
                            ("ridged", "<i4"), ("init_used", "<i4"),
                            ("fit", "<f8"), ("fit_prev", "<f8")])

_lib_handle = None


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


RT_ERR_NONFINITE = -4


class NonFiniteInput(RtError):
    """The device saw a NaN or Inf in Y (rt_tucker_info.nonfinite).  The
    call's outputs are attached as ``.out``."""

    def __init__(self, out):
        super().__init__(RT_ERR_NONFINITE, "Y holds a NaN or Inf value")
        self.out = out


def lib():
    """Load librtucker.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing; build it with "
                "`python -m paper_1412_1885_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.rt_tucker_rand_workspace.argtypes = [ctypes.POINTER(TuckerDesc), ctypes.POINTER(sz)]
        L.rt_tucker_bf16_copy_elems.argtypes = [ctypes.POINTER(TuckerDesc),
                                                ctypes.POINTER(i64)]
        L.rt_tucker_rand.argtypes = [ctypes.POINTER(TuckerDesc), vp, ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), vp, sz, ctypes.POINTER(vp), vp,
                                     vp, vp, ctypes.POINTER(TuckerTrace), vp]
        L.rt_ffcp_workspace.argtypes = [ctypes.POINTER(FfcpDesc), ctypes.POINTER(sz)]
        L.rt_ffcp.argtypes = [ctypes.POINTER(FfcpDesc), ctypes.POINTER(vp), vp,
                              ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz,
                              ctypes.POINTER(vp), vp, vp, vp, vp]
        L.rt_tucker_sequential_workspace.argtypes = [ctypes.POINTER(SequentialDesc),
                                                     ctypes.POINTER(sz)]
        L.rt_tucker_sequential.argtypes = [ctypes.POINTER(SequentialDesc), vp, vp, sz,
                                           ctypes.POINTER(vp), vp, ctypes.POINTER(vp), vp]
        L.rt_gaussian_matrix.argtypes = [i32, ctypes.c_uint64, i32, i64, i32, vp, vp]
        L.rt_ffcp_noalloc.argtypes = [ctypes.POINTER(FfcpDesc), ctypes.POINTER(vp), vp,
                                      ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), vp, vp, vp, vp]
        L.rt_ffcp_dense_workspace.argtypes = [ctypes.POINTER(TuckerDesc),
                                              ctypes.POINTER(FfcpDesc), ctypes.POINTER(sz)]
        L.rt_ffcp_dense.argtypes = [ctypes.POINTER(TuckerDesc), ctypes.POINTER(FfcpDesc), vp,
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                    ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz,
                                    ctypes.POINTER(vp), vp, vp, vp, vp, vp]
        L.rt_ttm.argtypes = [i32, i64, i64, i64, i32, vp, vp, vp, vp]
        L.rt_stream_pass.argtypes = [i32, i64, i64, i64, vp, vp, i32, vp, i32, vp, vp,
                                     vp, vp, sz, vp]
        L.rt_cp_fit_workspace.argtypes = [ctypes.POINTER(FfcpDesc), ctypes.POINTER(sz)]
        L.rt_cp_fit_dense.argtypes = [ctypes.POINTER(FfcpDesc), vp, ctypes.POINTER(vp),
                                      vp, vp, sz, vp, vp]
        L.rt_mlp_workspace.argtypes = [ctypes.POINTER(MlpDesc), ctypes.POINTER(sz)]
        L.rt_mlp_sync_bf16.argtypes = [ctypes.POINTER(MlpDesc), ctypes.POINTER(MlpParams), vp]
        L.rt_mlp_forward.argtypes = [ctypes.POINTER(MlpDesc), ctypes.POINTER(MlpParams), vp,
                                     vp, vp, sz, vp]
        L.rt_mlp_grad.argtypes = [ctypes.POINTER(MlpDesc), ctypes.POINTER(MlpParams), vp,
                                  ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, sz, vp]
        L.rt_mlp_train_step.argtypes = [ctypes.POINTER(MlpDesc), ctypes.POINTER(MlpParams),
                                        vp, ctypes.c_float, i32, vp, vp, sz, vp]
        L.rt_status_string.argtypes = [ctypes.c_int]
        L.rt_status_string.restype = ctypes.c_char_p
        L.rt_last_error.restype = ctypes.c_char_p
        L.rt_version.restype = ctypes.c_char_p
        for f in ("rt_tucker_rand_workspace", "rt_tucker_bf16_copy_elems",
                  "rt_tucker_rand", "rt_ffcp_workspace",
                  "rt_ffcp", "rt_ffcp_noalloc", "rt_tucker_sequential_workspace",
                  "rt_tucker_sequential", "rt_gaussian_matrix", "rt_ffcp_dense_workspace", "rt_ffcp_dense", "rt_ttm", "rt_cp_fit_workspace", "rt_cp_fit_dense",
                  "rt_stream_pass", "rt_profile_enable", "rt_profile_read",
                  "rt_mlp_workspace", "rt_mlp_sync_bf16", "rt_mlp_forward", "rt_mlp_grad",
                  "rt_mlp_train_step"):
            getattr(L, f).restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def status_string(status):
    return lib().rt_status_string(int(status)).decode()


def last_error():
    return lib().rt_last_error().decode()


def version():
    return lib().rt_version().decode()


def _check(rc):
    if rc != 0:
        raise RtError(rc, last_error())


# --------------------------------------------------------------- helpers

def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * max(1, len(tensors)))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr() if t is not None else 0
    return arr


def _require_device(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device=device)


# --------------------------------------------------------------- entry points

def tucker_desc(dims, ranks_tilde, ranks=None, sweeps=1, precision="f32",
                truncate=True, bf16_input=False, order="jacobi"):
    if order not in ("jacobi", "gauss_seidel"):
        raise ValueError(f"order must be 'jacobi' or 'gauss_seidel', not {order!r}")
    d = TuckerDesc()
    d.N = len(dims)
    d.sweeps = sweeps
    d.precision = PRECISIONS[precision]
    d.flags = (0 if truncate else RT_FLAG_NO_TRUNCATE) | \
        (RT_FLAG_BF16_INPUT if bf16_input else 0) | \
        (RT_FLAG_GAUSS_SEIDEL if order == "gauss_seidel" else 0)
    for n, I in enumerate(dims):
        d.dims[n] = int(I)
        d.ranks_tilde[n] = int(ranks_tilde[n])
        d.ranks[n] = int(ranks[n]) if ranks is not None else int(ranks_tilde[n])
    return d


def tucker_rand_workspace(desc):
    n = ctypes.c_size_t(0)
    _check(lib().rt_tucker_rand_workspace(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def bf16_copy_shape(dims, ranks_tilde=None):
    """Shape of the Ybf16 buffer of the precision form for a tensor of these
    dims (rt_tucker_bf16_copy_elems): dims[:-1] + (L,), L = dims[-1] rounded
    up to a multiple of 64; the copy of Y is buf[..., :dims[-1]]."""
    N = len(dims)
    rt = ranks_tilde if ranks_tilde is not None else [1] * N
    desc = tucker_desc(dims, rt, None, 1, "bf16")
    n = ctypes.c_int64(0)
    _check(lib().rt_tucker_bf16_copy_elems(ctypes.byref(desc), ctypes.byref(n)))
    lead = int(np.prod([int(d) for d in dims[:-1]]))
    return tuple(int(d) for d in dims[:-1]) + (n.value // lead,)


def tucker_rand(Y, omegas, omega_tildes, ranks=None, sweeps=1, precision="f32",
                truncate=True, trace=False, ybf16=None, bf16_input=False,
                dims=None, workspace=None, stream=None, sync=True,
                check_finite=True, order="jacobi"):
    """rt_tucker_rand.  Y: device tensor (float32 / float64, or int16/uint16
    BF16 bit patterns with bf16_input).  omegas: N device matrices I_n x R~_n.
    omega_tildes: list over sweeps of N device matrices.  Returns a dict with
    U (list), G, and when sync, info (numpy record) and the optional trace.
    With sync and check_finite, a NaN/Inf in Y raises NonFiniteInput."""
    torch = _torch()
    dims = list(Y.shape) if dims is None else list(dims)
    N = len(dims)
    rt = [int(o.shape[1]) for o in omegas]
    desc = tucker_desc(dims, rt, ranks, sweeps, precision, truncate, bf16_input, order)
    fdt = torch.float64 if precision == "f64" else torch.float32
    _require_device(Y, "Y")
    for n in range(N):
        _require_device(omegas[n], f"omegas[{n}]", fdt)
    for s in range(sweeps):
        for n in range(N):
            _require_device(omega_tildes[s][n], f"omega_tildes[{s}][{n}]", fdt)
    dev = Y.device
    out_r = [desc.ranks[n] if truncate else rt[n] for n in range(N)]
    U = [torch.empty((dims[n], out_r[n]), dtype=fdt, device=dev) for n in range(N)]
    G = torch.empty(out_r, dtype=fdt, device=dev)
    if precision == "bf16" and not bf16_input:
        shape = bf16_copy_shape(dims, rt)
        if ybf16 is None:
            ybf16 = torch.empty(shape, dtype=torch.int16, device=dev)
        _require_device(ybf16, "ybf16")
        if ybf16.numel() < int(np.prod(shape)) or ybf16.element_size() != 2:
            raise ValueError(f"ybf16 must hold {shape} 16-bit values")
    info = torch.zeros(TUCKER_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ws_bytes = tucker_rand_workspace(desc)
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes \
        else _workspace(ws_bytes, dev)
    tr = None
    trace_t = None
    if trace:
        tr = TuckerTrace()
        trace_t = {"Z": [], "Q": [], "Gt": torch.empty(rt, dtype=fdt, device=dev)}
        for s in range(sweeps):
            for n in range(N):
                z = torch.empty((dims[n], rt[n]), dtype=fdt, device=dev)
                q = torch.empty((dims[n], rt[n]), dtype=fdt, device=dev)
                trace_t["Z"].append(z)
                trace_t["Q"].append(q)
                tr.Z[s * N + n] = z.data_ptr()
                tr.Q[s * N + n] = q.data_ptr()
        tr.Gt = trace_t["Gt"].data_ptr()
    om = _ptr_array(omegas)
    omt = _ptr_array([omega_tildes[s][n] for s in range(sweeps) for n in range(N)])
    Uarr = _ptr_array(U)
    _check(lib().rt_tucker_rand(ctypes.byref(desc), _ptr(Y), om, omt, _ptr(ws),
                                ws.numel(), Uarr, _ptr(G), _ptr(ybf16), _ptr(info),
                                ctypes.byref(tr) if tr is not None else None,
                                _stream_handle(stream)))
    out = {"U": U, "G": G, "ybf16": ybf16, "info_dev": info, "workspace": ws}
    if trace:
        out["trace"] = trace_t
    if sync:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        out["info"] = np.frombuffer(info.cpu().numpy().tobytes(), TUCKER_INFO_DTYPE)[0]
        if check_finite and int(out["info"]["nonfinite"]) != 0:
            raise NonFiniteInput(out)
    return out


def ffcp_desc(dims, ranks, R, update="als", init="user", max_it=1000, tol=1e-6,
              l1=0.0, normY2=None):
    d = FfcpDesc()
    d.N = len(dims)
    d.R = int(R)
    d.update = UPDATES[update]
    d.init = INITS[init]
    d.max_it = int(max_it)
    d.tol = float(tol)
    d.l1 = float(l1)
    d.normY2 = float("nan") if normY2 is None else float(normY2)
    for n in range(d.N):
        d.dims[n] = int(dims[n])
        d.ranks[n] = int(ranks[n])
    return d


def ffcp_workspace(desc):
    n = ctypes.c_size_t(0)
    _check(lib().rt_ffcp_workspace(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def ffcp(U, G, R, update="als", A_init=None, init=None, pad=None, max_it=1000,
         tol=1e-6, l1=0.0, normY2=None, fit_trace=False, workspace=None,
         stream=None, sync=True):
    """rt_ffcp on a Tucker format.  U: N device float32 I_n x R_n; G: device
    float32 core.  A_init (list of device float32 I_n x R) selects the user
    init; init="coeff" / "coeff_guarded" takes A_init as R_n x R coefficient
    matrices (A_n = U_n V_n; the guarded form keeps them only if their
    initial fit is at least the HOSVD start's); init="hosvd" (pad: list of
    R_n x (R - R_n) matrices for modes with R > R_n)."""
    torch = _torch()
    N = len(U)
    dims = [int(u.shape[0]) for u in U]
    ranks = [int(u.shape[1]) for u in U]
    if init is None:
        init = "user" if A_init is not None else "hosvd"
    desc = ffcp_desc(dims, ranks, R, update, init, max_it, tol, l1, normY2)
    for n in range(N):
        _require_device(U[n], f"U[{n}]", torch.float32)
    _require_device(G, "G", torch.float32)
    if A_init is not None:
        for n, a in enumerate(A_init):
            if a is not None:
                _require_device(a, f"A_init[{n}]", torch.float32)
    dev = G.device
    A = [torch.empty((dims[n], R), dtype=torch.float32, device=dev) for n in range(N)]
    lam = torch.empty(R, dtype=torch.float32, device=dev)
    info = torch.zeros(FFCP_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ft = torch.zeros(max_it, dtype=torch.float64, device=dev) if fit_trace else None
    ws_bytes = ffcp_workspace(desc)
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes \
        else _workspace(ws_bytes, dev)
    ainit = _ptr_array(A_init) if A_init is not None else None
    padp = _ptr_array(pad) if pad is not None else None
    _check(lib().rt_ffcp(ctypes.byref(desc), _ptr_array(U), _ptr(G), ainit, padp,
                         _ptr(ws), ws.numel(), _ptr_array(A), _ptr(lam), _ptr(ft),
                         _ptr(info), _stream_handle(stream)))
    out = {"A": A, "lam": lam, "info_dev": info, "fit_trace_dev": ft, "workspace": ws}
    if sync:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        inf = np.frombuffer(info.cpu().numpy().tobytes(), FFCP_INFO_DTYPE)[0]
        if int(inf["converged"]) < 0:
            raise RtError(-1, "FFCP: a grid barrier of the multi-workgroup form gave up "
                              "(results undefined)")
        out["info"] = inf
        if ft is not None:
            out["fits"] = ft.cpu().numpy()[: int(inf["iterations"])]
    return out


def sequential_desc(dims, ranks_tilde, seed, precision="f32"):
    d = SequentialDesc()
    d.N = len(dims)
    d.precision = PRECISIONS[precision]
    d.seed = int(seed)
    for n, I in enumerate(dims):
        d.dims[n] = int(I)
        d.ranks_tilde[n] = int(ranks_tilde[n])
    return d


def tucker_sequential(Y, ranks_tilde, seed, keep_omegas=False, stream=None, sync=True):
    """rt_tucker_sequential: Algorithm 2 with the device's counter-based
    Gaussian test matrices.  Y: device float32 / float64 tensor.  Returns
    U (list), G and, with keep_omegas, the test matrices as used."""
    torch = _torch()
    dims = list(Y.shape)
    N = len(dims)
    precision = "f64" if Y.dtype == torch.float64 else "f32"
    desc = sequential_desc(dims, ranks_tilde, seed, precision)
    _require_device(Y, "Y")
    n = ctypes.c_size_t(0)
    _check(lib().rt_tucker_sequential_workspace(ctypes.byref(desc), ctypes.byref(n)))
    dev = Y.device
    ws = _workspace(n.value, dev)
    U = [torch.empty((dims[k], ranks_tilde[k]), dtype=Y.dtype, device=dev) for k in range(N)]
    G = torch.empty(list(ranks_tilde), dtype=Y.dtype, device=dev)
    oms = None
    if keep_omegas:
        oms = []
        for k in range(N):
            rows = 1
            for q in range(N):
                if q != k:
                    rows *= ranks_tilde[q] if q < k else dims[q]
            oms.append(torch.empty((rows, ranks_tilde[k]), dtype=Y.dtype, device=dev))
    _check(lib().rt_tucker_sequential(ctypes.byref(desc), _ptr(Y), _ptr(ws), ws.numel(),
                                      _ptr_array(U), _ptr(G),
                                      _ptr_array(oms) if oms is not None else None,
                                      _stream_handle(stream)))
    if sync:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return {"U": U, "G": G, "omegas": oms, "workspace": ws}


def gaussian_matrix(rows, cols, mode, seed, dtype=None, device="cuda", stream=None):
    """rt_gaussian_matrix: the counter-based Gaussian test matrix (device)."""
    torch = _torch()
    dtype = torch.float32 if dtype is None else dtype
    out = torch.empty((rows, cols), dtype=dtype, device=device)
    code = PRECISIONS["f64"] if dtype == torch.float64 else PRECISIONS["f32"]
    _check(lib().rt_gaussian_matrix(code, int(seed), int(mode), int(rows), int(cols),
                                    _ptr(out), _stream_handle(stream)))
    return out


def ffcp_noalloc(U, G, R, update="als", A_init=None, init=None, pad=None, max_it=1000,
                 tol=1e-6, l1=0.0, normY2=None, fit_trace=False, stream=None, sync=True):
    """rt_ffcp_noalloc: ffcp with the library's static scratch instead of a
    workspace (arguments and results as ffcp)."""
    torch = _torch()
    N = len(U)
    dims = [int(u.shape[0]) for u in U]
    ranks = [int(u.shape[1]) for u in U]
    if init is None:
        init = "user" if A_init is not None else "hosvd"
    desc = ffcp_desc(dims, ranks, R, update, init, max_it, tol, l1, normY2)
    for n in range(N):
        _require_device(U[n], f"U[{n}]", torch.float32)
    _require_device(G, "G", torch.float32)
    dev = G.device
    A = [torch.empty((dims[n], R), dtype=torch.float32, device=dev) for n in range(N)]
    lam = torch.empty(R, dtype=torch.float32, device=dev)
    info = torch.zeros(FFCP_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ft = torch.zeros(max_it, dtype=torch.float64, device=dev) if fit_trace else None
    _check(lib().rt_ffcp_noalloc(ctypes.byref(desc), _ptr_array(U), _ptr(G),
                                 _ptr_array(A_init) if A_init is not None else None,
                                 _ptr_array(pad) if pad is not None else None,
                                 _ptr_array(A), _ptr(lam), _ptr(ft), _ptr(info),
                                 _stream_handle(stream)))
    out = {"A": A, "lam": lam}
    if sync:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        inf = np.frombuffer(info.cpu().numpy().tobytes(), FFCP_INFO_DTYPE)[0]
        if int(inf["converged"]) < 0:
            raise RtError(-1, "FFCP: a grid barrier of the multi-workgroup form gave up "
                              "(results undefined)")
        out["info"] = inf
        if ft is not None:
            out["fits"] = ft.cpu().numpy()[: int(inf["iterations"])]
    return out


def ffcp_dense_workspace(tdesc, fdesc):
    n = ctypes.c_size_t(0)
    _check(lib().rt_ffcp_dense_workspace(ctypes.byref(tdesc), ctypes.byref(fdesc),
                                         ctypes.byref(n)))
    return n.value


def ffcp_dense(Y, omegas, omega_tildes, R, ranks=None, sweeps=1, precision="f32",
               update="als", A_init=None, init=None, pad=None, max_it=1000, tol=1e-6,
               l1=0.0, normY2=None, fit_trace=False, ybf16=None, stream=None,
               sync=True, check_finite=True):
    """rt_ffcp_dense: Algorithm 1 on the dense Y (RandTucker2i, then FFCP on
    its Tucker format, in one call).  Arguments as tucker_rand and ffcp;
    A_init / pad as ffcp's (I_n x R starts, or R_n x R coefficients)."""
    torch = _torch()
    dims = list(Y.shape)
    N = len(dims)
    rt = [int(o.shape[1]) for o in omegas]
    rk = list(ranks) if ranks is not None else rt
    tdesc = tucker_desc(dims, rt, rk, sweeps, precision)
    if init is None:
        init = "user" if A_init is not None else "hosvd"
    fdesc = ffcp_desc(dims, rk, R, update, init, max_it, tol, l1, normY2)
    _require_device(Y, "Y")
    for n in range(N):
        _require_device(omegas[n], f"omegas[{n}]", torch.float32)
        for s_ in range(sweeps):
            _require_device(omega_tildes[s_][n], f"omega_tildes[{s_}][{n}]", torch.float32)
    dev = Y.device
    if precision == "bf16" and ybf16 is None:
        ybf16 = torch.empty(bf16_copy_shape(dims, rt), dtype=torch.int16, device=dev)
    A = [torch.empty((dims[n], R), dtype=torch.float32, device=dev) for n in range(N)]
    lam = torch.empty(R, dtype=torch.float32, device=dev)
    tinfo = torch.zeros(TUCKER_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    finfo = torch.zeros(FFCP_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    ft = torch.zeros(max_it, dtype=torch.float64, device=dev) if fit_trace else None
    ws = _workspace(ffcp_dense_workspace(tdesc, fdesc), dev)
    om = _ptr_array(omegas)
    omt = _ptr_array([omega_tildes[s_][n] for s_ in range(sweeps) for n in range(N)])
    _check(lib().rt_ffcp_dense(ctypes.byref(tdesc), ctypes.byref(fdesc), _ptr(Y), om, omt,
                               _ptr(ybf16),
                               _ptr_array(A_init) if A_init is not None else None,
                               _ptr_array(pad) if pad is not None else None,
                               _ptr(ws), ws.numel(), _ptr_array(A), _ptr(lam), _ptr(ft),
                               _ptr(tinfo), _ptr(finfo), _stream_handle(stream)))
    out = {"A": A, "lam": lam, "workspace": ws}
    if sync:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        out["tucker_info"] = np.frombuffer(tinfo.cpu().numpy().tobytes(), TUCKER_INFO_DTYPE)[0]
        inf = np.frombuffer(finfo.cpu().numpy().tobytes(), FFCP_INFO_DTYPE)[0]
        out["info"] = inf
        if ft is not None:
            out["fits"] = ft.cpu().numpy()[: int(inf["iterations"])]
        if check_finite and int(out["tucker_info"]["nonfinite"]) != 0:
            raise NonFiniteInput(out)
    return out


def ttm(X, M, n, stream=None):
    """rt_ttm: X x_n M^T for a device tensor X and device matrix M (I_n x K)."""
    torch = _torch()
    _require_device(X, "X")
    _require_device(M, "M", X.dtype)
    shape = list(X.shape)
    A = int(np.prod(shape[:n])) if n > 0 else 1
    C = int(np.prod(shape[n + 1:])) if n + 1 < len(shape) else 1
    K = int(M.shape[1])
    out = torch.empty(shape[:n] + [K] + shape[n + 1:], dtype=X.dtype, device=X.device)
    dt = RT_F64 if X.dtype == torch.float64 else RT_F32
    _check(lib().rt_ttm(dt, A, shape[n], C, K, _ptr(X), _ptr(M), _ptr(out),
                        _stream_handle(stream)))
    return out


def stream_pass(Y3, B2, B1=None, stream=None):
    """rt_stream_pass on a device tensor viewed [A, I1, I2]: returns
    (TA, TB or None, ||Y||^2)."""
    torch = _torch()
    _require_device(Y3, "Y")
    A, I1, I2 = (int(x) for x in Y3.shape)
    K2 = int(B2.shape[1])
    TA = torch.empty((A, I1, K2), dtype=Y3.dtype, device=Y3.device)
    TB = None
    K1 = 0
    if B1 is not None:
        K1 = int(B1.shape[1])
        TB = torch.empty((A, K1, I2), dtype=Y3.dtype, device=Y3.device)
    nrm = torch.zeros(2, dtype=torch.float64, device=Y3.device)
    ws = _workspace(8192, Y3.device)
    dt = RT_F64 if Y3.dtype == torch.float64 else RT_F32
    _check(lib().rt_stream_pass(dt, A, I1, I2, _ptr(Y3), _ptr(B2), K2, _ptr(B1), K1,
                                _ptr(TA), _ptr(TB), _ptr(nrm), _ptr(ws), ws.numel(),
                                _stream_handle(stream)))
    torch.cuda.current_stream().synchronize()
    return TA, TB, float(nrm[0].item())


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("count", ctypes.c_int64 * 9)]


PROFILE_STAGES = ("first_pass", "sweep_pass", "core_pass", "contract", "qr",
                  "truncate", "ffcp", "stats", "convert")


def profile_enable(on=True):
    _check(lib().rt_profile_enable(1 if on else 0))


def profile_read():
    """Per-stage {name: (total_ms, launches)} of the bracketed stages."""
    p = Profile()
    _check(lib().rt_profile_read(ctypes.byref(p)))
    return {PROFILE_STAGES[i]: (p.ms[i], int(p.count[i])) for i in range(len(PROFILE_STAGES))}


def cp_fit_dense(Y, A, lam=None, stream=None):
    """rt_cp_fit_dense: (fit, ||Y||^2, <Y, Yhat>) of a CP model against Y."""
    torch = _torch()
    _require_device(Y, "Y", torch.float32)
    dims = list(Y.shape)
    R = int(A[0].shape[1])
    desc = ffcp_desc(dims, [1] * len(dims), R)
    n = ctypes.c_size_t(0)
    _check(lib().rt_cp_fit_workspace(ctypes.byref(desc), ctypes.byref(n)))
    ws = _workspace(n.value, Y.device)
    out3 = torch.zeros(4, dtype=torch.float64, device=Y.device)
    _check(lib().rt_cp_fit_dense(ctypes.byref(desc), _ptr(Y), _ptr_array(A), _ptr(lam),
                                 _ptr(ws), ws.numel(), _ptr(out3), _stream_handle(stream)))
    torch.cuda.current_stream().synchronize()
    v = out3.cpu().numpy()
    return float(v[0]), float(v[1]), float(v[2])


# names of the C ABI
rt_tucker_rand = tucker_rand
rt_ffcp = ffcp
rt_ttm = ttm
rt_cp_fit_dense = cp_fit_dense
rt_stream_pass = stream_pass


# ------------------------------------------------------------ learned init

def mlp_desc(batch, core_dims, R, hidden=(1024, 1024)):
    d = MlpDesc()
    d.batch = int(batch)
    d.N = len(core_dims)
    d.R = int(R)
    d.hidden1, d.hidden2 = int(hidden[0]), int(hidden[1])
    for n, c in enumerate(core_dims):
        d.core_dims[n] = int(c)
    return d


class MLP:
    """Device parameters of the learned FFCP initializer (rt_mlp_*): FP32
    master weights and biases, their BF16 copies and the Adam moments, all
    torch tensors on `device`.  Layer widths: (prod core_dims, hidden1,
    hidden2, R * sum core_dims)."""

    def __init__(self, core_dims, R, hidden=(1024, 1024), device="cuda"):
        torch = _torch()
        self.core_dims = [int(c) for c in core_dims]
        self.R = int(R)
        self.hidden = tuple(int(h) for h in hidden)
        d0 = int(np.prod(self.core_dims))
        d3 = self.R * sum(self.core_dims)
        self.dims = [d0, self.hidden[0], self.hidden[1], d3]
        f32 = dict(dtype=torch.float32, device=device)
        self.W = [torch.zeros(self.dims[l], self.dims[l + 1], **f32) for l in range(3)]
        self.b = [torch.zeros(self.dims[l + 1], **f32) for l in range(3)]
        self.Wb = [torch.zeros(self.dims[l], self.dims[l + 1], dtype=torch.int16,
                               device=device) for l in range(3)]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0
        self._ws = None

    def params(self):
        p = MlpParams()
        for name in ("W", "b", "Wb", "mW", "vW", "mb", "vb"):
            arr = getattr(p, name)
            for l, t in enumerate(getattr(self, name)):
                arr[l] = t.data_ptr()
        return p

    def desc(self, batch):
        return mlp_desc(batch, self.core_dims, self.R, self.hidden)

    def load(self, W, b):
        """Set the FP32 weights (host arrays, W[l]: d_l x d_{l+1}) and refresh
        the BF16 copies; resets the optimizer state."""
        torch = _torch()
        for l in range(3):
            self.W[l].copy_(torch.from_numpy(np.ascontiguousarray(W[l], np.float32)))
            self.b[l].copy_(torch.from_numpy(np.ascontiguousarray(b[l], np.float32)))
        for t in self.mW + self.vW + self.mb + self.vb:
            t.zero_()
        self.step = 0
        self.sync_bf16()

    def sync_bf16(self, stream=None):
        d = self.desc(1)
        p = self.params()
        _check(lib().rt_mlp_sync_bf16(ctypes.byref(d), ctypes.byref(p),
                                       _stream_handle(stream)))

    def _workspace(self, d, device):
        n = ctypes.c_size_t(0)
        _check(lib().rt_mlp_workspace(ctypes.byref(d), ctypes.byref(n)))
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = _workspace(n.value, device)
        return self._ws

    def forward(self, G, stream=None):
        """G: device float32 (batch, *core_dims) -> V (batch, d3) float32,
        the predicted factors scaled by ||G||^(1/N)."""
        torch = _torch()
        _require_device(G, "G", torch.float32)
        B = int(G.shape[0])
        d = self.desc(B)
        ws = self._workspace(d, G.device)
        V = torch.empty(B, self.dims[3], dtype=torch.float32, device=G.device)
        p = self.params()
        _check(lib().rt_mlp_forward(ctypes.byref(d), ctypes.byref(p), _ptr(G), _ptr(V),
                                    _ptr(ws), ws.numel(), _stream_handle(stream)))
        return V

    def split(self, V):
        """Per-core list of N coefficient matrices R_n x R from forward()."""
        out, off = [], 0
        for c in self.core_dims:
            out.append(V[:, off:off + c * self.R].reshape(-1, c, self.R))
            off += c * self.R
        return out

    def grad(self, G, stream=None):
        """(per-core losses, [gW], [gb]) without updating the parameters."""
        torch = _torch()
        _require_device(G, "G", torch.float32)
        B = int(G.shape[0])
        d = self.desc(B)
        ws = self._workspace(d, G.device)
        gW = [torch.empty_like(w) for w in self.W]
        gb = [torch.empty_like(b) for b in self.b]
        loss = torch.empty(B, dtype=torch.float32, device=G.device)
        p = self.params()
        _check(lib().rt_mlp_grad(ctypes.byref(d), ctypes.byref(p), _ptr(G),
                                 _ptr_array(gW), _ptr_array(gb), _ptr(loss), _ptr(ws),
                                 ws.numel(), _stream_handle(stream)))
        return loss, gW, gb

    def train_step(self, G, lr, stream=None):
        """One Adam step on the batch G; returns the device per-core losses."""
        torch = _torch()
        _require_device(G, "G", torch.float32)
        B = int(G.shape[0])
        d = self.desc(B)
        ws = self._workspace(d, G.device)
        loss = torch.empty(B, dtype=torch.float32, device=G.device)
        self.step += 1
        p = self.params()
        _check(lib().rt_mlp_train_step(ctypes.byref(d), ctypes.byref(p), _ptr(G),
                                       float(lr), self.step, _ptr(loss), _ptr(ws),
                                       ws.numel(), _stream_handle(stream)))
        return loss
