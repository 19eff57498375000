"""ctypes binding of the C ABI in include/jsvd.h (argument marshalling only).

Every step of the computation runs in the HIP library; torch supplies the
device memory and the current stream.  There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.

Matrices are column-major in the library.  A torch (m x n) matrix whose
strides are (1, m) is column-major already; the functions below take any
(m x n) tensor, copy it into column-major storage and return column-major
views.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libjsvd.so")

_i32, _i64, _dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

STRATEGIES = {"rrev": 0, "r": 1, "crev": 2, "c": 3, "rr": 4}
STATUS = {0: "ok", 1: "not converged", 3: "non-finite value", 4: "HIP error",
          5: "equal singular values", 6: "out of device memory"}


class Opts(ctypes.Structure):
    _fields_ = [("block_w", _i32), ("strategy", _i32), ("max_inner_sweeps", _i32),
                ("max_sweeps", _i32), ("want_v", _i32), ("sort", _i32), ("qr", _i32),
                ("scaled", _i32), ("factorize", _i32), ("fuse", _i32)]


class Info(ctypes.Structure):
    _fields_ = [("sweeps", _i32), ("converged", _i32), ("rotations", _i64),
                ("proper_rotations", _i64), ("inner_sweeps", _i64), ("pair_updates", _i64),
                ("chol_breakdowns", _i32), ("hyp_clamps", _i32), ("block_w", _i32),
                ("n_blocks", _i32), ("seconds", _dbl), ("preprocessed", _i32), ("scaled", _i32),
                ("rank", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("count", _i32), ("n_upper", _i64 * 8), ("block_w", _i32 * 8),
                ("gram_wg", _i32 * 8), ("update_wg", _i32 * 8),
                ("batch_g_groups", _i32), ("batch_block_min_n", _i32)]


TUNING_PATH = os.path.join(HERE, "tuning.json")


class JsvdError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code} ({STATUS.get(code, 'invalid argument' if code < 0 else '?')})")
        self.code = code


_LIB = None
EXPORTS = ["jsvd_default_opts", "jsvd_create", "jsvd_set_stream", "jsvd_destroy", "jsvd_gesvd",
           "jsvd_hsvd", "jsvd_strategy_table", "jsvd_inner_table", "jsvd_quad_table",
           "jsvd_strategy_order",
           "jsvd_error_string",
           "jsvd_diag_fp64", "jsvd_kernel_timing", "jsvd_kernel_times", "jsvd_gesvd_batched",
           "jsvd_svd_backward", "jsvd_set_tuning", "jsvd_batched_block_min_n",
           "jsvd_workspace_size", "jsvd_workspace_size_batched", "jsvd_reserve_batched",
           "jsvd_diag_refined", "jsvd_gesvd_batched_noalloc", "jsvd_gesvd_full",
           "jsvd_colnorms", "jsvd_rdssq_bounds"]


def lib():
    """Load libjsvd.so (raises if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1401_2720_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.jsvd_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.jsvd_create.argtypes = [ctypes.POINTER(_vp), _vp]
    L.jsvd_set_stream.argtypes = [_vp, _vp]
    L.jsvd_destroy.argtypes = [_vp]
    L.jsvd_gesvd.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(Opts),
                             ctypes.POINTER(Info)]
    L.jsvd_gesvd_full.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64,
                                  ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.jsvd_hsvd.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _i64,
                            ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.jsvd_strategy_table.argtypes = [_i32, _i32, _vp]
    L.jsvd_inner_table.argtypes = [_i32, _i32, _vp]
    L.jsvd_quad_table.argtypes = [_i32, _i32, _vp]
    L.jsvd_strategy_order.argtypes = [_i32]
    L.jsvd_strategy_order.restype = _i32
    L.jsvd_batched_block_min_n.argtypes = [_vp]
    L.jsvd_batched_block_min_n.restype = _i32
    L.jsvd_error_string.argtypes = [ctypes.c_int]
    L.jsvd_error_string.restype = ctypes.c_char_p
    L.jsvd_diag_fp64.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp]
    L.jsvd_gesvd_batched.argtypes = [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     _vp, ctypes.POINTER(Opts), _vp, _vp]
    L.jsvd_gesvd_batched_noalloc.argtypes = L.jsvd_gesvd_batched.argtypes
    L.jsvd_svd_backward.argtypes = [_vp, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.jsvd_set_tuning.argtypes = [_vp, ctypes.POINTER(Tuning)]
    L.jsvd_workspace_size.argtypes = [_vp, _i64, _i64, ctypes.POINTER(Opts),
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.jsvd_workspace_size_batched.argtypes = [_vp, _i64, _i32, _i32, ctypes.POINTER(Opts),
                                              ctypes.POINTER(ctypes.c_size_t)]
    L.jsvd_reserve_batched.argtypes = [_vp, _i64, _i32, _i32, ctypes.POINTER(Opts)]
    L.jsvd_diag_refined.argtypes = [_vp, _i64, _vp, _vp, _vp]
    L.jsvd_colnorms.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp]
    L.jsvd_rdssq_bounds.argtypes = [_i32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.jsvd_kernel_timing.argtypes = [_vp, ctypes.c_int]
    L.jsvd_kernel_times.argtypes = [_vp, _vp, _vp]
    for f in ("jsvd_default_opts", "jsvd_create", "jsvd_set_stream", "jsvd_destroy",
              "jsvd_gesvd", "jsvd_hsvd", "jsvd_strategy_table", "jsvd_diag_fp64",
              "jsvd_kernel_timing", "jsvd_kernel_times", "jsvd_gesvd_batched",
              "jsvd_svd_backward", "jsvd_workspace_size", "jsvd_workspace_size_batched",
              "jsvd_reserve_batched", "jsvd_diag_refined", "jsvd_gesvd_batched_noalloc",
              "jsvd_gesvd_full", "jsvd_colnorms", "jsvd_rdssq_bounds"):
        getattr(L, f).restype = ctypes.c_int
    _LIB = L
    return L


# ------------------------------------------------------------------ handles
_HANDLES = {}


def _handle(device_index, stream_ptr):
    L = lib()
    h = _HANDLES.get(device_index)
    if h is None:
        import torch
        with torch.cuda.device(device_index):
            hp = _vp()
            rc = L.jsvd_create(ctypes.byref(hp), _vp(stream_ptr))
            if rc:
                raise JsvdError(rc, "jsvd_create")
        h = hp
        _HANDLES[device_index] = h
        table = load_tuning(device_index)
        if table is not None:
            set_tuning(device_index, table, handle=h)
    rc = L.jsvd_set_stream(h, _vp(stream_ptr))
    if rc:
        raise JsvdError(rc, "jsvd_set_stream")
    return h


def tuning_struct(table):
    """The jsvd_tuning of a table {"n_upper": [...], "block_w": [...],
    "gram_wg": [...], "update_wg": [...] (optional, 0 = built-in),
    "batch_g_groups": int, "batch_block_min_n": int} (raises ValueError if it
    cannot be one)."""
    nu, bw = list(table.get("n_upper", [])), list(table.get("block_w", []))
    gw = list(table.get("gram_wg", [0] * len(nu)))
    uw = list(table.get("update_wg", [0] * len(nu)))
    if len(nu) != len(bw) or len(nu) > 8 or len(gw) != len(nu) or len(uw) != len(nu):
        raise ValueError("n_upper, block_w, gram_wg and update_wg must have the same length, "
                         "at most 8")
    t = Tuning()
    t.count = len(nu)
    for i, (a, b) in enumerate(zip(nu, bw)):
        t.n_upper[i] = int(a)
        t.block_w[i] = int(b)
        t.gram_wg[i] = int(gw[i])
        t.update_wg[i] = int(uw[i])
    t.batch_g_groups = int(table.get("batch_g_groups", 0))
    t.batch_block_min_n = int(table.get("batch_block_min_n", 0))
    return t


def load_tuning(device_index=None, path=None):
    """The tuned table of the autotuner's file for this device's architecture,
    or None (no file, or tuned on another architecture)."""
    import json
    path = path or TUNING_PATH
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if device_index is not None:
        import torch
        arch = torch.cuda.get_device_properties(device_index).gcnArchName.split(":")[0]
        if rec.get("arch") != arch:
            return None
    return rec.get("table")


def set_tuning(device_index, table, handle=None):
    """Install a tuned table on the device's handle (None removes it)."""
    h = handle if handle is not None else _HANDLES.get(device_index)
    if h is None:
        import torch
        h = _handle(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    t = tuning_struct(table) if table is not None else None
    rc = lib().jsvd_set_tuning(h, ctypes.byref(t) if t is not None else None)
    if rc:
        raise JsvdError(rc, "jsvd_set_tuning")


QR_MODES = {"auto": 0, "off": 1, "on": 2}  # also the scaled-mode choices


FACTORIZE = {"cholesky": 0, "qr": 1}


def make_opts(block_w=0, strategy="rrev", max_inner_sweeps=0, max_sweeps=30, want_v=True,
              sort=True, qr="auto", scaled="auto", factorize="cholesky", fuse=False):
    o = Opts()
    lib().jsvd_default_opts(ctypes.byref(o))
    o.block_w = int(block_w)
    o.strategy = STRATEGIES[strategy] if isinstance(strategy, str) else int(strategy)
    o.max_inner_sweeps = int(max_inner_sweeps)
    o.max_sweeps = int(max_sweeps)
    o.want_v = 1 if want_v else 0
    o.sort = 1 if sort else 0
    o.qr = QR_MODES[qr] if isinstance(qr, str) else int(qr)
    o.scaled = QR_MODES[scaled] if isinstance(scaled, str) else int(scaled)
    o.factorize = FACTORIZE[factorize] if isinstance(factorize, str) else int(factorize)
    o.fuse = 1 if fuse else 0
    return o


def _colmajor_copy(A):
    """A fresh (n x m) contiguous tensor whose memory is A (m x n) column-major."""
    import torch
    if not (A.is_cuda and A.dtype == torch.float64 and A.dim() == 2):
        raise ValueError("expected a 2-D float64 CUDA tensor")
    return A.t().clone(memory_format=torch.contiguous_format)


def _raise_on(rc, what, allow):
    if rc < 0 or (rc > 0 and rc not in allow):
        raise JsvdError(rc, what)


def gesvd(A, block_w=0, strategy="rrev", max_inner_sweeps=0, max_sweeps=30, want_v=True,
          sort=True, allow=(1,), qr="auto", scaled="auto", factorize="cholesky", fuse=False):
    """SVD A = U diag(S) V^T of a float64 CUDA tensor (m >= n).

    Returns (U, S, V, info): U (m x n) and V (n x n) column-major views, S (n),
    info a dict (sweeps, rotations, ... and 'status').  Status codes listed
    in ``allow`` are returned in info instead of raised.
    """
    import torch
    m, n = A.shape
    work = _colmajor_copy(A)
    dev = A.device
    S = torch.empty(n, dtype=torch.float64, device=dev)
    Vb = torch.empty((n, n), dtype=torch.float64, device=dev) if want_v else None
    stream = torch.cuda.current_stream(dev)
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                stream.cuda_stream)
    o = make_opts(block_w, strategy, max_inner_sweeps, max_sweeps, want_v, sort, qr, scaled,
                  factorize, fuse)
    info = Info()
    rc = lib().jsvd_gesvd(h, m, n, _vp(work.data_ptr()), m, _vp(S.data_ptr()),
                          _vp(Vb.data_ptr()) if want_v else None, n, ctypes.byref(o),
                          ctypes.byref(info))
    _raise_on(rc, "jsvd_gesvd", allow)
    d = info.as_dict()
    d["status"] = rc
    return work.t(), S, (Vb.t() if want_v else None), d


def gesvd_full(A, block_w=0, strategy="rrev", max_inner_sweeps=0, max_sweeps=30, want_v=True,
               allow=(1,), qr="auto", scaled="auto", factorize="cholesky", fuse=False):
    """Full SVD A = U [diag(S); 0] V^T of a float64 CUDA tensor (m >= n) with
    U of order m.  Returns (U, S, V, info): U (m x m) and V (n x n) views of
    column-major buffers."""
    import torch
    m, n = A.shape
    work = _colmajor_copy(A)
    dev = A.device
    Ub = torch.empty((m, m), dtype=torch.float64, device=dev)
    S = torch.empty(n, dtype=torch.float64, device=dev)
    Vb = torch.empty((n, n), dtype=torch.float64, device=dev) if want_v else None
    stream = torch.cuda.current_stream(dev)
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                stream.cuda_stream)
    o = make_opts(block_w, strategy, max_inner_sweeps, max_sweeps, want_v, True, qr, scaled,
                  factorize, fuse)
    info = Info()
    rc = lib().jsvd_gesvd_full(h, m, n, _vp(work.data_ptr()), m, _vp(Ub.data_ptr()), m,
                               _vp(S.data_ptr()), _vp(Vb.data_ptr()) if want_v else None, n,
                               ctypes.byref(o), ctypes.byref(info))
    _raise_on(rc, "jsvd_gesvd_full", allow)
    d = info.as_dict()
    d["status"] = rc
    return Ub.t(), S, (Vb.t() if want_v else None), d


def hsvd(G, J, block_w=0, strategy="rrev", max_inner_sweeps=0, max_sweeps=30, want_v=True,
         sort=True, allow=(1,), scaled="auto", factorize="cholesky", fuse=False):
    """Hyperbolic SVD G V = U diag(S), V^T J V = diag(J_out).

    J: sequence of n values, each +1 or -1.  Returns (U, S, V, J_out, info)
    with J_out a numpy int8 array.
    """
    import numpy as np
    import torch
    m, n = G.shape
    Jh = np.ascontiguousarray(np.asarray(J, dtype=np.int8))
    if Jh.shape != (n,):
        raise ValueError("J must have n entries")
    Jout = np.zeros(n, dtype=np.int8)
    work = _colmajor_copy(G)
    dev = G.device
    S = torch.empty(n, dtype=torch.float64, device=dev)
    Vb = torch.empty((n, n), dtype=torch.float64, device=dev) if want_v else None
    stream = torch.cuda.current_stream(dev)
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                stream.cuda_stream)
    o = make_opts(block_w, strategy, max_inner_sweeps, max_sweeps, want_v, sort, scaled=scaled,
                  factorize=factorize, fuse=fuse)
    info = Info()
    rc = lib().jsvd_hsvd(h, m, n, _vp(work.data_ptr()), m, _vp(Jh.ctypes.data),
                         _vp(Jout.ctypes.data), _vp(S.data_ptr()),
                         _vp(Vb.data_ptr()) if want_v else None, n, ctypes.byref(o),
                         ctypes.byref(info))
    _raise_on(rc, "jsvd_hsvd", allow)
    d = info.as_dict()
    d["status"] = rc
    return work.t(), S, (Vb.t() if want_v else None), Jout, d


def strategy_table(order, kind="rrev"):
    """(order-1, order/2, 2) int32 array of one-based pivot pairs (host only)."""
    import numpy as np
    out = np.zeros((order - 1) * (order // 2) * 2, dtype=np.int32)
    k = STRATEGIES[kind] if isinstance(kind, str) else int(kind)
    rc = lib().jsvd_strategy_table(int(order), k, _vp(out.ctypes.data))
    if rc:
        raise JsvdError(rc, "jsvd_strategy_table")
    return out.reshape(order - 1, order // 2, 2)


def inner_table(order, kind="rrev"):
    """The inner kernels' table for 2w = order (32 or 64): strategy_table's
    with each step's pairs reordered for the LDS banks (host only)."""
    import numpy as np
    out = np.zeros((order - 1) * (order // 2) * 2, dtype=np.int32)
    k = STRATEGIES[kind] if isinstance(kind, str) else int(kind)
    rc = lib().jsvd_inner_table(int(order), k, _vp(out.ctypes.data))
    if rc:
        raise JsvdError(rc, "jsvd_inner_table")
    return out.reshape(order - 1, order // 2, 2)


def quad_table(order, kind="rrev"):
    """(order - 2, order / 4, 8) int32 array of the step-to-step groups of
    the fused update-and-Gram launch, or None when the ordering has none
    (host only)."""
    import numpy as np
    out = np.zeros(max(order - 2, 0) * (order // 4) * 8, dtype=np.int32)
    k = STRATEGIES[kind] if isinstance(kind, str) else int(kind)
    rc = lib().jsvd_quad_table(int(order), k, _vp(out.ctypes.data))
    if rc == 1:
        return None
    if rc:
        raise JsvdError(rc, "jsvd_quad_table")
    return out.reshape(order - 2, order // 4, 8)


def strategy_order(nb):
    return int(lib().jsvd_strategy_order(int(nb)))


def batched_block_min_n(device_index=None):
    """Smallest n that the batched call blocks on this device's handle."""
    import torch
    dev = torch.cuda.current_device() if device_index is None else device_index
    h = _handle(dev, torch.cuda.current_stream(dev).cuda_stream)
    return int(lib().jsvd_batched_block_min_n(h))


def diag_fp64(a, b):
    """Device a/b and sqrt(a) for float64 CUDA tensors (rounding check)."""
    import torch
    a = a.contiguous()
    b = b.contiguous()
    q = torch.empty_like(a)
    r = torch.empty_like(a)
    dev = a.device
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                torch.cuda.current_stream(dev).cuda_stream)
    rc = lib().jsvd_diag_fp64(h, a.numel(), _vp(a.data_ptr()), _vp(b.data_ptr()),
                              _vp(q.data_ptr()), _vp(r.data_ptr()))
    if rc:
        raise JsvdError(rc, "jsvd_diag_fp64")
    return q, r


def colnorms(A):
    """DRDSSQ (Appendix A) of every column of a 2-D float64 CUDA tensor (any
    strides are copied to column-major first): returns (exps, ssq, norms),
    the sum of squares 2^exps ssq in the common form and the norm."""
    import torch
    m, n = A.shape
    X = _colmajor_copy(A)
    exps = torch.empty(n, dtype=torch.int32, device=A.device)
    ssq = torch.empty(n, dtype=torch.float64, device=A.device)
    norms = torch.empty(n, dtype=torch.float64, device=A.device)
    dev = A.device
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                torch.cuda.current_stream(dev).cuda_stream)
    rc = lib().jsvd_colnorms(h, m, n, _vp(X.data_ptr()), m, _vp(exps.data_ptr()),
                             _vp(ssq.data_ptr()), _vp(norms.data_ptr()))
    if rc:
        raise JsvdError(rc, "jsvd_colnorms")
    return exps, ssq, norms


def rdssq_bounds(lg):
    """(t_lo, t_hi) of DRDSSQ for vectors with ceil(lg n) = lg (host only)."""
    lo, hi = ctypes.c_double(), ctypes.c_double()
    rc = lib().jsvd_rdssq_bounds(int(lg), ctypes.byref(lo), ctypes.byref(hi))
    if rc:
        raise JsvdError(rc, "jsvd_rdssq_bounds")
    return lo.value, hi.value


def diag_refined(a, b):
    """The kernels' refined reciprocal, quotient and square roots on the
    device: returns (rcp(b), a/b, sqrt(a), 1/sqrt(a), sqrt(a)) as float64
    CUDA tensors (the last two from the Cholesky's scaled pair)."""
    import torch
    a = a.contiguous()
    b = b.contiguous()
    out = torch.empty(5 * a.numel(), dtype=torch.float64, device=a.device)
    dev = a.device
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                torch.cuda.current_stream(dev).cuda_stream)
    rc = lib().jsvd_diag_refined(h, a.numel(), _vp(a.data_ptr()), _vp(b.data_ptr()),
                                 _vp(out.data_ptr()))
    if rc:
        raise JsvdError(rc, "jsvd_diag_refined")
    return tuple(out.view(5, -1)[k] for k in range(5))


def workspace_size(m, n, device_index=None, **opts):
    """Device workspace bytes of jsvd_gesvd / jsvd_hsvd for an m x n problem."""
    import torch
    dev = torch.cuda.current_device() if device_index is None else device_index
    h = _handle(dev, torch.cuda.current_stream(dev).cuda_stream)
    o = make_opts(**opts)
    out = ctypes.c_size_t(0)
    rc = lib().jsvd_workspace_size(h, int(m), int(n), ctypes.byref(o), ctypes.byref(out))
    if rc:
        raise JsvdError(rc, "jsvd_workspace_size")
    return int(out.value)


def workspace_size_batched(batch, device_index=None, max_sweeps=30):
    """Device workspace bytes of jsvd_gesvd_batched for a Batch."""
    import torch
    dev = torch.cuda.current_device() if device_index is None else device_index
    h = _handle(dev, torch.cuda.current_stream(dev).cuda_stream)
    o = make_opts(max_sweeps=max_sweeps, want_v=batch.want_v)
    out = ctypes.c_size_t(0)
    rc = lib().jsvd_workspace_size_batched(h, batch.count, batch.max_m, batch.max_n,
                                           ctypes.byref(o), ctypes.byref(out))
    if rc:
        raise JsvdError(rc, "jsvd_workspace_size_batched")
    return int(out.value)


def reserve_batched(batch, max_sweeps=30):
    """Allocate the batched workspace for a Batch now, so that the next
    gesvd_batched on it allocates nothing (and can be captured first)."""
    import torch
    dev = batch.A.device
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                torch.cuda.current_stream(dev).cuda_stream)
    o = make_opts(max_sweeps=max_sweeps, want_v=batch.want_v)
    rc = lib().jsvd_reserve_batched(h, batch.count, batch.max_m, batch.max_n, ctypes.byref(o))
    if rc:
        raise JsvdError(rc, "jsvd_reserve_batched")


def kernel_timing(device_index, enable=True, stride=1):
    """Turn per-kernel event timing on (and zero it) or off for a device's
    handle; with stride k only every k-th p-step of a sweep is timed."""
    import torch
    h = _handle(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    rc = lib().jsvd_kernel_timing(h, int(stride) if enable else 0)
    if rc:
        raise JsvdError(rc, "jsvd_kernel_timing")


def kernel_times(device_index):
    """{'gram'|'inner'|'update'|'fused': (total_ms, launches)} since the last
    reset ('fused': the update fused with the next p-step's Gram kernel)."""
    import numpy as np
    import torch
    h = _handle(device_index, torch.cuda.current_stream(device_index).cuda_stream)
    ms = np.zeros(4, np.float64)
    cnt = np.zeros(4, np.int64)
    rc = lib().jsvd_kernel_times(h, _vp(ms.ctypes.data), _vp(cnt.ctypes.data))
    if rc:
        raise JsvdError(rc, "jsvd_kernel_times")
    return {k: (float(ms[i]), int(cnt[i]))
            for i, k in enumerate(("gram", "inner", "update", "fused"))}


class Batch:
    """Uneven problems packed column-major into one device buffer.

    Built from a list of (m_i x n_i) arrays (numpy or torch); holds the
    device buffers A (in: G, out: U), S, V, the int32 sizes and the int64
    offsets that jsvd_gesvd_batched takes.
    """

    def __init__(self, mats, device="cuda", want_v=True):
        import numpy as np
        import torch
        ms = np.array([a.shape[0] for a in mats], np.int32)
        ns = np.array([a.shape[1] for a in mats], np.int32)
        if np.any(ms < ns) or np.any(ns < 1):
            raise ValueError("every problem needs 1 <= n <= m")
        count = len(mats)
        a_off = np.zeros(count, np.int64)
        s_off = np.zeros(count, np.int64)
        v_off = np.zeros(count, np.int64)
        if count:
            a_off[1:] = np.cumsum(ms.astype(np.int64) * ns)[:-1]
            s_off[1:] = np.cumsum(ns.astype(np.int64))[:-1]
            v_off[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
        host = np.concatenate([np.asarray(a if not hasattr(a, "cpu") else a.cpu(),
                                          np.float64).ravel(order="F") for a in mats])
        self.count = count
        self.max_m = int(ms.max()) if count else 1
        self.max_n = int(ns.max()) if count else 1
        self.m_host, self.n_host = ms, ns
        self.a_off_host, self.s_off_host, self.v_off_host = a_off, s_off, v_off
        dev = torch.device(device)
        self.A0 = torch.from_numpy(host).to(dev)
        self.A = self.A0.clone()
        self.S = torch.zeros(int(ns.sum()), dtype=torch.float64, device=dev)
        self.V = torch.zeros(int((ns.astype(np.int64) ** 2).sum()), dtype=torch.float64,
                             device=dev) if want_v else None
        self.m = torch.from_numpy(ms).to(dev)
        self.n = torch.from_numpy(ns).to(dev)
        self.a_off = torch.from_numpy(a_off).to(dev)
        self.s_off = torch.from_numpy(s_off).to(dev)
        self.v_off = torch.from_numpy(v_off).to(dev)
        self.status = torch.zeros(count, dtype=torch.int32, device=dev)
        self.sweeps = torch.zeros(count, dtype=torch.int32, device=dev)
        self.want_v = want_v

    @classmethod
    def from_uniform(cls, A, want_v=True):
        """A batch of equally sized problems from a (b, m, n) float64 CUDA tensor,
        packed on the device (no host round trip)."""
        import numpy as np
        import torch
        b, m, n = A.shape
        self = cls.__new__(cls)
        dev = A.device
        self.count = b
        self.max_m, self.max_n = m, n
        self.m_host = np.full(b, m, np.int32)
        self.n_host = np.full(b, n, np.int32)
        self.a_off_host = np.arange(b, dtype=np.int64) * m * n
        self.s_off_host = np.arange(b, dtype=np.int64) * n
        self.v_off_host = np.arange(b, dtype=np.int64) * n * n
        self.A0 = A.transpose(-1, -2).contiguous().view(-1)
        self.A = self.A0.clone()
        self.S = torch.zeros(b * n, dtype=torch.float64, device=dev)
        self.V = torch.zeros(b * n * n, dtype=torch.float64, device=dev) if want_v else None
        self.m = torch.from_numpy(self.m_host).to(dev)
        self.n = torch.from_numpy(self.n_host).to(dev)
        self.a_off = torch.from_numpy(self.a_off_host).to(dev)
        self.s_off = torch.from_numpy(self.s_off_host).to(dev)
        self.v_off = torch.from_numpy(self.v_off_host).to(dev)
        self.status = torch.zeros(b, dtype=torch.int32, device=dev)
        self.sweeps = torch.zeros(b, dtype=torch.int32, device=dev)
        self.want_v = want_v
        return self

    def results(self, i):
        """(U, S, V) of problem i as numpy arrays (after a synchronised run)."""
        m, n = int(self.m_host[i]), int(self.n_host[i])
        a, s, v = int(self.a_off_host[i]), int(self.s_off_host[i]), int(self.v_off_host[i])
        U = self.A[a:a + m * n].cpu().numpy().reshape((m, n), order="F")
        S = self.S[s:s + n].cpu().numpy()
        V = self.V[v:v + n * n].cpu().numpy().reshape((n, n), order="F") if self.want_v else None
        return U, S, V


def gesvd_batched(batch, max_sweeps=30, restore=True, noalloc=False, scaled="auto"):
    """Run jsvd_gesvd_batched (noalloc=True: jsvd_gesvd_batched_noalloc) on a
    Batch on the current stream (asynchronous).

    restore=True first copies the original inputs back into batch.A.
    scaled="on": DDRJAC pairs and DRDSSQ norms for badly scaled problems.
    """
    import torch
    dev = batch.A.device
    stream = torch.cuda.current_stream(dev)
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                stream.cuda_stream)
    if restore:
        batch.A.copy_(batch.A0)
    o = make_opts(max_sweeps=max_sweeps, want_v=batch.want_v, scaled=scaled)
    name = "jsvd_gesvd_batched_noalloc" if noalloc else "jsvd_gesvd_batched"
    rc = getattr(lib(), name)(
        h, batch.count, batch.max_m, batch.max_n, _vp(batch.m.data_ptr()),
        _vp(batch.n.data_ptr()), _vp(batch.a_off.data_ptr()), _vp(batch.s_off.data_ptr()),
        _vp(batch.v_off.data_ptr()) if batch.want_v else None, _vp(batch.A.data_ptr()),
        _vp(batch.S.data_ptr()), _vp(batch.V.data_ptr()) if batch.want_v else None,
        ctypes.byref(o), _vp(batch.status.data_ptr()), _vp(batch.sweeps.data_ptr()))
    if rc:
        raise JsvdError(rc, name)


def svd_backward(U, S, V, dU=None, dS=None, dV=None):
    """dA from the SVD adjoint for (b, m, n) / (m, n) float64 CUDA tensors.

    U (.., m, n), S (.., n), V (.., n, n) as matrices (any strides); dU, dS,
    dV of the same shapes or None.  Returns dA (.., m, n).
    """
    import torch
    batched = U.dim() == 3
    if not batched:
        U, S, V = U[None], S[None], V[None]
        dU = None if dU is None else dU[None]
        dS = None if dS is None else dS[None]
        dV = None if dV is None else dV[None]
    b, m, n = U.shape

    def cm(X):  # contiguous batch of column-major matrices
        return None if X is None else X.transpose(-1, -2).contiguous()

    Uc, Vc, dUc, dVc = cm(U), cm(V), cm(dU), cm(dV)
    Sc = S.contiguous()
    dSc = None if dS is None else dS.contiguous()
    dA = torch.empty((b, n, m), dtype=torch.float64, device=U.device)
    dev = U.device
    h = _handle(dev.index if dev.index is not None else torch.cuda.current_device(),
                torch.cuda.current_stream(dev).cuda_stream)
    p = lambda X: None if X is None else _vp(X.data_ptr())  # noqa: E731
    rc = lib().jsvd_svd_backward(h, b, m, n, p(Uc), p(Sc), p(Vc), p(dUc), p(dSc), p(dVc),
                                 p(dA))
    if rc:
        raise JsvdError(rc, "jsvd_svd_backward")
    dA = dA.transpose(-1, -2)
    return dA if batched else dA[0]
