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

STRATEGIES = {"rrev": 0, "r": 1, "crev": 2, "c": 3}
STATUS = {0: "ok", 1: "not converged", 2: "Cholesky breakdown", 3: "non-finite value",
          4: "HIP error", 5: "out of device memory"}


class Opts(ctypes.Structure):
    _fields_ = [("block_w", _i32), ("strategy", _i32), ("max_inner_sweeps", _i32),
                ("max_sweeps", _i32), ("want_v", _i32), ("sort", _i32)]


class Info(ctypes.Structure):
    _fields_ = [("sweeps", _i32), ("converged", _i32), ("rotations", _i64),
                ("proper_rotations", _i64), ("inner_sweeps", _i64), ("pair_updates", _i64),
                ("chol_breakdowns", _i32), ("hyp_clamps", _i32), ("block_w", _i32),
                ("n_blocks", _i32), ("seconds", _dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class JsvdError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: status {code} ({STATUS.get(code, 'invalid argument' if code < 0 else '?')})")
        self.code = code


_LIB = None
EXPORTS = ["jsvd_default_opts", "jsvd_create", "jsvd_set_stream", "jsvd_destroy", "jsvd_gesvd",
           "jsvd_hsvd", "jsvd_strategy_table", "jsvd_strategy_order", "jsvd_error_string",
           "jsvd_diag_fp64"]


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
    L.jsvd_hsvd.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _i64,
                            ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    L.jsvd_strategy_table.argtypes = [_i32, _i32, _vp]
    L.jsvd_strategy_order.argtypes = [_i32]
    L.jsvd_strategy_order.restype = _i32
    L.jsvd_error_string.argtypes = [ctypes.c_int]
    L.jsvd_error_string.restype = ctypes.c_char_p
    L.jsvd_diag_fp64.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp]
    for f in ("jsvd_default_opts", "jsvd_create", "jsvd_set_stream", "jsvd_destroy",
              "jsvd_gesvd", "jsvd_hsvd", "jsvd_strategy_table", "jsvd_diag_fp64"):
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
    rc = L.jsvd_set_stream(h, _vp(stream_ptr))
    if rc:
        raise JsvdError(rc, "jsvd_set_stream")
    return h


def make_opts(block_w=0, strategy="rrev", max_inner_sweeps=30, max_sweeps=30, want_v=True,
              sort=True):
    o = Opts()
    lib().jsvd_default_opts(ctypes.byref(o))
    o.block_w = int(block_w)
    o.strategy = STRATEGIES[strategy] if isinstance(strategy, str) else int(strategy)
    o.max_inner_sweeps = int(max_inner_sweeps)
    o.max_sweeps = int(max_sweeps)
    o.want_v = 1 if want_v else 0
    o.sort = 1 if sort else 0
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


def gesvd(A, block_w=0, strategy="rrev", max_inner_sweeps=30, max_sweeps=30, want_v=True,
          sort=True, allow=(1,)):
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
    o = make_opts(block_w, strategy, max_inner_sweeps, max_sweeps, want_v, sort)
    info = Info()
    rc = lib().jsvd_gesvd(h, m, n, _vp(work.data_ptr()), m, _vp(S.data_ptr()),
                          _vp(Vb.data_ptr()) if want_v else None, n, ctypes.byref(o),
                          ctypes.byref(info))
    _raise_on(rc, "jsvd_gesvd", allow)
    d = info.as_dict()
    d["status"] = rc
    return work.t(), S, (Vb.t() if want_v else None), d


def hsvd(G, J, block_w=0, strategy="rrev", max_inner_sweeps=30, max_sweeps=30, want_v=True,
         sort=True, allow=(1,)):
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
    o = make_opts(block_w, strategy, max_inner_sweeps, max_sweeps, want_v, sort)
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


def strategy_order(nb):
    return int(lib().jsvd_strategy_order(int(nb)))


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
