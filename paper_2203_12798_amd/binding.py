"""ctypes binding of libdpar2 (include/dpar2.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory and the stream; nothing here computes on the host or falls back
to another implementation -- a missing library is an error."""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpar2.so")

DPAR2_OK = 0
DPAR2_EINVAL = -1
DPAR2_ESHAPE = -2
DPAR2_ENUMERIC = -3
DPAR2_ENOCONV = -4
DPAR2_EHIP = -5
DPAR2_EWORKSPACE = -6
DPAR2_F32 = 0
DPAR2_BF16 = 1
DPAR2_FP8_E4M3 = 2
DPAR2_FLAG_NO_GRAPH = 0x1
DPAR2_FLAG_WIDE_SLAB = 0x2
DPAR2_FLAG_DETERMINISTIC = 0x4

WARN_JACOBI_CAP = 0x1
WARN_RANK_DEFICIENT = 0x2
WARN_NONFINITE = 0x4


class Dpar2Error(RuntimeError):
    """A non-OK status.  For DPAR2_ENUMERIC raised by the report readers
    and by decompose(report=True), `report` holds the report(s) the library
    filled anyway."""

    def __init__(self, status: int, message: str, report=None):
        super().__init__(f"libdpar2 status {status}: {message}")
        self.status = status
        self.report = report


class c_tensor(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("J", ctypes.c_int64),
                ("row_offsets", ctypes.c_void_p), ("row_offsets_host", ctypes.c_void_p),
                ("slab", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("slice_scale", ctypes.c_void_p)]


class c_opts(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("sketch", ctypes.c_int32), ("sketch2", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("power_iters", ctypes.c_int32), ("item_rows", ctypes.c_int32)]


class c_factors(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("V", ctypes.c_void_p), ("W", ctypes.c_void_p)]


class c_compressed(ctypes.Structure):
    _fields_ = [("Mt", ctypes.c_void_p), ("D", ctypes.c_void_p), ("E", ctypes.c_void_p),
                ("F", ctypes.c_void_p), ("Phi", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("xnorm2", ctypes.c_void_p)]


class c_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("err_last", ctypes.c_double),
                ("fit_compressed", ctypes.c_double), ("fit_true", ctypes.c_double),
                ("xnorm2", ctypes.c_double), ("warn_bits", ctypes.c_uint32)]


EXPORTS = ["dpar2_workspace_bytes", "dpar2_workspace_size", "dpar2_compress", "dpar2_als_step", "dpar2_fitness",
           "dpar2_output_U", "dpar2_output_A", "dpar2_decompose", "dpar2_decompose_noalloc", "dpar2_append_workspace_bytes",
           "dpar2_append", "dpar2_release",
           "dpar2_release_all", "dpar2_plain_workspace_bytes", "dpar2_als_plain", "dpar2_feature_pcc",
           "dpar2_slice_similarity", "dpar2_top_k", "dpar2_rwr", "dpar2_compressed_view", "dpar2_report_read",
           "dpar2_batch_workspace_size", "dpar2_decompose_batch", "dpar2_batch_report_read",
           "dpar2_warm_param_count", "dpar2_warm_features", "dpar2_warm_targets", "dpar2_warm_apply",
           "dpar2_warm_forward", "dpar2_warm_backward", "dpar2_warm_adam", "dpar2_autotune_item_rows",
           "dpar2_autotune_slab",
           "dpar2_profile_enable", "dpar2_profile_read", "dpar2_status_string", "dpar2_last_error"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libdpar2.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not found: build it with paper_2203_12798_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    for name in ("dpar2_workspace_bytes", "dpar2_workspace_size"):
        getattr(lib, name).restype = ctypes.c_size_t
        getattr(lib, name).argtypes = [P(c_tensor), P(c_opts)]
    lib.dpar2_compress.restype = ctypes.c_int32
    lib.dpar2_compress.argtypes = [P(c_tensor), P(c_opts), vp, vp, vp, ctypes.c_size_t, vp]
    lib.dpar2_als_step.restype = ctypes.c_int32
    lib.dpar2_als_step.argtypes = [P(c_tensor), P(c_opts), P(c_factors), ctypes.c_int32, vp, vp,
                                   ctypes.c_size_t, vp]
    lib.dpar2_fitness.restype = ctypes.c_int32
    lib.dpar2_fitness.argtypes = [P(c_tensor), P(c_opts), P(c_factors), vp, vp, ctypes.c_size_t, vp]
    lib.dpar2_output_U.restype = ctypes.c_int32
    lib.dpar2_output_U.argtypes = [P(c_tensor), P(c_opts), P(c_factors), vp, vp, ctypes.c_size_t, vp]
    lib.dpar2_output_A.restype = ctypes.c_int32
    lib.dpar2_output_A.argtypes = [P(c_tensor), P(c_opts), vp, vp, ctypes.c_size_t, vp]
    lib.dpar2_decompose.restype = ctypes.c_int32
    lib.dpar2_decompose.argtypes = [P(c_tensor), P(c_opts), vp, vp, P(c_factors), vp, P(c_report), vp,
                                    ctypes.c_size_t, vp]
    lib.dpar2_decompose_noalloc.restype = ctypes.c_int32
    lib.dpar2_decompose_noalloc.argtypes = [P(c_tensor), P(c_opts), vp, vp, P(c_factors), vp, P(c_report), vp]
    lib.dpar2_append_workspace_bytes.restype = ctypes.c_size_t
    lib.dpar2_append_workspace_bytes.argtypes = [P(c_tensor), ctypes.c_int64, P(c_opts)]
    lib.dpar2_append.restype = ctypes.c_int32
    lib.dpar2_append.argtypes = [P(c_tensor), ctypes.c_int64, P(c_opts), vp, vp, vp, ctypes.c_size_t,
                                 P(c_factors), vp, P(c_report), vp, ctypes.c_size_t, vp]
    lib.dpar2_plain_workspace_bytes.restype = ctypes.c_size_t
    lib.dpar2_plain_workspace_bytes.argtypes = [P(c_tensor), P(c_opts)]
    lib.dpar2_als_plain.restype = ctypes.c_int32
    lib.dpar2_als_plain.argtypes = [P(c_tensor), P(c_opts), P(c_factors), vp, vp, P(c_report), vp,
                                    ctypes.c_size_t, vp]
    lib.dpar2_feature_pcc.restype = ctypes.c_int32
    lib.dpar2_feature_pcc.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, vp, vp]
    lib.dpar2_slice_similarity.restype = ctypes.c_int32
    lib.dpar2_slice_similarity.argtypes = [P(c_tensor), ctypes.c_int32, vp, ctypes.c_int32, vp, vp, ctypes.c_double,
                                           vp, vp]
    lib.dpar2_top_k.restype = ctypes.c_int32
    lib.dpar2_top_k.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp]
    lib.dpar2_rwr.restype = ctypes.c_int32
    lib.dpar2_rwr.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    lib.dpar2_release.restype = ctypes.c_int32
    lib.dpar2_release.argtypes = [vp]
    lib.dpar2_release_all.restype = ctypes.c_int32
    lib.dpar2_release_all.argtypes = []
    lib.dpar2_compressed_view.restype = ctypes.c_int32
    lib.dpar2_compressed_view.argtypes = [P(c_tensor), P(c_opts), vp, ctypes.c_size_t, P(c_compressed)]
    lib.dpar2_report_read.restype = ctypes.c_int32
    lib.dpar2_report_read.argtypes = [P(c_tensor), P(c_opts), vp, P(c_report), vp]
    lib.dpar2_batch_workspace_size.restype = ctypes.c_size_t
    lib.dpar2_batch_workspace_size.argtypes = [ctypes.c_int32, P(c_tensor), P(c_opts)]
    lib.dpar2_decompose_batch.restype = ctypes.c_int32
    lib.dpar2_decompose_batch.argtypes = [ctypes.c_int32, P(c_tensor), P(c_opts), P(vp), P(vp), P(c_factors), vp,
                                          ctypes.c_size_t, vp]
    lib.dpar2_batch_report_read.restype = ctypes.c_int32
    lib.dpar2_batch_report_read.argtypes = [ctypes.c_int32, P(c_tensor), P(c_opts), vp, P(c_report), vp]
    i32, f32 = ctypes.c_int32, ctypes.c_float
    lib.dpar2_warm_param_count.restype = ctypes.c_int64
    lib.dpar2_warm_param_count.argtypes = [i32]
    for name, n_dev in (("dpar2_warm_features", 1), ("dpar2_warm_targets", 4), ("dpar2_warm_apply", 4)):
        fn = getattr(lib, name)
        fn.restype = i32
        if name == "dpar2_warm_features":
            fn.argtypes = [P(c_tensor), P(c_opts), vp, ctypes.c_size_t, vp, vp]
        elif name == "dpar2_warm_targets":
            fn.argtypes = [P(c_tensor), P(c_opts), vp, ctypes.c_size_t, P(c_factors), vp, vp, vp, vp]
        else:
            fn.argtypes = [P(c_tensor), P(c_opts), vp, ctypes.c_size_t, vp, vp, vp, P(c_factors), vp]
    lib.dpar2_warm_forward.restype = i32
    lib.dpar2_warm_forward.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dpar2_warm_backward.restype = i32
    lib.dpar2_warm_backward.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.dpar2_warm_adam.restype = i32
    lib.dpar2_warm_adam.argtypes = [i32, vp, vp, vp, vp, i32, f32, f32, f32, f32, f32, vp]
    lib.dpar2_autotune_item_rows.restype = i32
    lib.dpar2_autotune_item_rows.argtypes = [P(c_tensor), P(c_opts), vp, P(i32), i32, vp, ctypes.c_size_t,
                                             P(i32), P(f32), vp]
    lib.dpar2_autotune_slab.restype = i32
    lib.dpar2_autotune_slab.argtypes = [P(c_tensor), P(c_opts), vp, P(i32), P(i32), i32, vp, ctypes.c_size_t,
                                        P(i32), P(f32), vp]
    lib.dpar2_profile_enable.restype = ctypes.c_int32
    lib.dpar2_profile_enable.argtypes = [ctypes.c_int32]
    lib.dpar2_profile_read.restype = ctypes.c_int32
    lib.dpar2_profile_read.argtypes = [P(ctypes.c_int32), P(ctypes.c_double)]
    lib.dpar2_status_string.restype = ctypes.c_char_p
    lib.dpar2_status_string.argtypes = [ctypes.c_int32]
    lib.dpar2_last_error.restype = ctypes.c_char_p
    lib.dpar2_last_error.argtypes = []
    _lib = lib
    return lib


def _check(st: int, report=None):
    if st != DPAR2_OK:
        msg = load().dpar2_last_error().decode(errors="replace")
        raise Dpar2Error(st, msg, report)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream)


@dataclasses.dataclass
class Options:
    rank: int
    sketch: int
    sketch2: int
    max_iter: int
    tol: float = -1.0
    power_iters: int = 0
    graph: bool = True      # False sets DPAR2_FLAG_NO_GRAPH
    item_rows: int = 0      # 0: the library's default work-item size
    wide_slab: bool = False  # True sets DPAR2_FLAG_WIDE_SLAB (128-column-chunk slab pass)
    deterministic: bool = False  # True sets DPAR2_FLAG_DETERMINISTIC (resumable bit for bit)

    def c(self) -> c_opts:
        flags = ((0 if self.graph else DPAR2_FLAG_NO_GRAPH) | (DPAR2_FLAG_WIDE_SLAB if self.wide_slab else 0)
                 | (DPAR2_FLAG_DETERMINISTIC if self.deterministic else 0))
        return c_opts(self.rank, self.sketch, self.sketch2, self.max_iter, float(self.tol),
                      flags, self.power_iters, self.item_rows)


class Tensor:
    """An irregular tensor resident on the GPU: slab (N x J, row-major) of
    float32, of bfloat16 bit patterns (uint16 storage, torch.int16) or of fp8
    e4m3 bytes (torch.uint8) with per-slice float32 scales, and int64 row
    offsets (device copy + host copy)."""

    def __init__(self, slab, offsets_dev, offsets_host: np.ndarray, dtype: int = DPAR2_F32, scale=None):
        import torch
        want = {DPAR2_F32: torch.float32, DPAR2_BF16: torch.int16, DPAR2_FP8_E4M3: torch.uint8}[dtype]
        assert slab.is_cuda and slab.dtype == want and slab.is_contiguous() and slab.dim() == 2
        assert offsets_dev.is_cuda and offsets_dev.dtype == torch.int64 and offsets_dev.is_contiguous()
        if dtype == DPAR2_FP8_E4M3:
            assert scale is not None and scale.is_cuda and scale.dtype == torch.float32
        self.slab = slab
        self.dtype = dtype
        self.scale = scale
        self.offsets_dev = offsets_dev
        self.offsets_host = np.ascontiguousarray(offsets_host, dtype=np.int64)
        self.K = int(self.offsets_host.shape[0] - 1)
        self.J = int(slab.shape[1])

    @classmethod
    def from_numpy(cls, slab: np.ndarray, offsets: np.ndarray, device="cuda:0", dtype: int = DPAR2_F32,
                   scale: np.ndarray | None = None):
        """slab: float32 values, or for DPAR2_BF16 the uint16 bit patterns,
        for DPAR2_FP8_E4M3 the uint8 codes (then scale: K float32)."""
        import torch
        if dtype == DPAR2_F32:
            s = torch.from_numpy(np.ascontiguousarray(slab, dtype=np.float32)).to(device)
        elif dtype == DPAR2_BF16:
            s = torch.from_numpy(np.ascontiguousarray(slab, dtype=np.uint16).view(np.int16)).to(device)
        else:
            s = torch.from_numpy(np.ascontiguousarray(slab, dtype=np.uint8)).to(device)
        o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(device)
        sc = None
        if scale is not None:
            sc = torch.from_numpy(np.ascontiguousarray(scale, dtype=np.float32)).to(device)
        return cls(s, o, offsets, dtype, sc)

    def c(self) -> c_tensor:
        return c_tensor(self.K, self.J, _ptr(self.offsets_dev),
                        self.offsets_host.ctypes.data_as(ctypes.c_void_p).value,
                        _ptr(self.slab), self.dtype, _ptr(self.scale) if self.scale is not None else None)


class Factors:
    """H (R x R), V (J x R), W (K x R) float64 device tensors, row-major."""

    def __init__(self, H, V, W):
        import torch
        for t in (H, V, W):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        self.H, self.V, self.W = H, V, W

    @classmethod
    def from_numpy(cls, H, V, W, device="cuda:0"):
        import torch
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
        return cls(f(H), f(V), f(W))

    def c(self) -> c_factors:
        return c_factors(_ptr(self.H), _ptr(self.V), _ptr(self.W))

    def numpy(self):
        return self.H.cpu().numpy(), self.V.cpu().numpy(), self.W.cpu().numpy()


def workspace_size(X: Tensor, o: Options) -> int:
    """Bytes of workspace for (X, o); raises on invalid arguments."""
    lib = load()
    tc, oc = X.c(), o.c()
    n = lib.dpar2_workspace_bytes(ctypes.byref(tc), ctypes.byref(oc))
    if n == 0:
        raise Dpar2Error(DPAR2_EINVAL, last_error())
    return int(n)


def alloc_workspace(X: Tensor, o: Options, device="cuda:0"):
    import torch
    n = workspace_size(X, o)
    return torch.empty(n + 256, dtype=torch.uint8, device=device)


def _ws(ws):
    p = int(ws.data_ptr())
    off = (-p) % 256
    return p + off, int(ws.numel()) - off


def compress(X: Tensor, o: Options, omega1, omega2, ws, stream=None):
    lib = load()
    p, n = _ws(ws)
    _check(lib.dpar2_compress(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(omega1), _ptr(omega2),
                              p, n, _stream(stream)))


def als_step(X: Tensor, o: Options, f: Factors, n_steps: int, ws, err_trace=None, stream=None):
    lib = load()
    p, n = _ws(ws)
    fc = f.c()
    _check(lib.dpar2_als_step(ctypes.byref(X.c()), ctypes.byref(o.c()), ctypes.byref(fc), int(n_steps),
                              _ptr(err_trace), p, n, _stream(stream)))


def fitness(X: Tensor, o: Options, f: Factors, ws, fit=None, stream=None):
    lib = load()
    p, n = _ws(ws)
    fc = f.c()
    _check(lib.dpar2_fitness(ctypes.byref(X.c()), ctypes.byref(o.c()), ctypes.byref(fc), _ptr(fit),
                             p, n, _stream(stream)))


def output_U(X: Tensor, o: Options, f: Factors, U, ws, stream=None):
    lib = load()
    p, n = _ws(ws)
    fc = f.c()
    _check(lib.dpar2_output_U(ctypes.byref(X.c()), ctypes.byref(o.c()), ctypes.byref(fc), _ptr(U),
                              p, n, _stream(stream)))


def decompose(X: Tensor, o: Options, omega1, omega2, f: Factors, ws, U=None, stream=None, report=False):
    """Enqueues the decomposition.  report=True synchronises and returns the
    report dict (with "status": 0 or DPAR2_ENOCONV); a NaN/Inf slab raises
    Dpar2Error(DPAR2_ENUMERIC)."""
    lib = load()
    p, n = _ws(ws)
    fc = f.c()
    r = c_report() if report else None
    st = lib.dpar2_decompose(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(omega1), _ptr(omega2),
                             ctypes.byref(fc), _ptr(U), ctypes.byref(r) if report else None, p, n,
                             _stream(stream))
    d = None
    if report and st in (DPAR2_OK, DPAR2_ENOCONV, DPAR2_ENUMERIC):
        d = _report_dict(r)
        d["status"] = st
    if st == DPAR2_ENOCONV and report:
        return d
    _check(st, d)
    return d


def decompose_noalloc(X: Tensor, o: Options, omega1, omega2, f: Factors, U=None, stream=None, report=False):
    """decompose() on the library's static device scratch (no workspace, no
    allocation); same report convention as decompose()."""
    lib = load()
    fc = f.c()
    r = c_report() if report else None
    st = lib.dpar2_decompose_noalloc(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(omega1), _ptr(omega2),
                                     ctypes.byref(fc), _ptr(U), ctypes.byref(r) if report else None,
                                     _stream(stream))
    d = None
    if report and st in (DPAR2_OK, DPAR2_ENOCONV, DPAR2_ENUMERIC):
        d = _report_dict(r)
        d["status"] = st
    if st == DPAR2_ENOCONV and report:
        return d
    _check(st, d)
    return d


NOALLOC_SCRATCH_BYTES = 64 << 20


def append_workspace_size(X: Tensor, k_prev: int, o: Options) -> int:
    """Bytes of workspace of append(X, k_prev, o, ...); raises on invalid
    arguments."""
    n = load().dpar2_append_workspace_bytes(ctypes.byref(X.c()), int(k_prev), ctypes.byref(o.c()))
    if n == 0:
        raise Dpar2Error(DPAR2_EINVAL, last_error())
    return int(n)


def alloc_append_workspace(X: Tensor, k_prev: int, o: Options, device="cuda:0"):
    import torch
    return torch.empty(append_workspace_size(X, k_prev, o) + 256, dtype=torch.uint8, device=device)


def append(X: Tensor, k_prev: int, o: Options, omega1, omega2, ws_prev, f: Factors, ws, U=None, stream=None,
           report=False):
    """DPar2 after appending slices k_prev.. of X to a tensor whose first
    k_prev slices were decomposed with workspace ws_prev (dpar2_append); same
    report convention as decompose().  ws (from alloc_append_workspace) then
    serves as ws_prev of the next append."""
    lib = load()
    p, n = _ws(ws)
    pp, npv = _ws(ws_prev)
    fc = f.c()
    r = c_report() if report else None
    st = lib.dpar2_append(ctypes.byref(X.c()), int(k_prev), ctypes.byref(o.c()), _ptr(omega1), _ptr(omega2),
                          pp, npv, ctypes.byref(fc), _ptr(U), ctypes.byref(r) if report else None, p, n,
                          _stream(stream))
    d = None
    if report and st in (DPAR2_OK, DPAR2_ENOCONV, DPAR2_ENUMERIC):
        d = _report_dict(r)
        d["status"] = st
    if st == DPAR2_ENOCONV and report:
        return d
    _check(st, d)
    return d


def plain_workspace_size(X: Tensor, o: Options) -> int:
    n = load().dpar2_plain_workspace_bytes(ctypes.byref(X.c()), ctypes.byref(o.c()))
    if n == 0:
        raise Dpar2Error(DPAR2_EINVAL, last_error())
    return int(n)


def alloc_plain_workspace(X: Tensor, o: Options, device="cuda:0"):
    import torch
    return torch.empty(plain_workspace_size(X, o) + 256, dtype=torch.uint8, device=device)


def als_plain(X: Tensor, o: Options, f: Factors, ws, err_trace=None, U=None, stream=None, report=False):
    """PARAFAC2-ALS on the uncompressed slices (Alg. 2), o.max_iter
    iterations from the factors in f (updated in place); same report
    convention as decompose()."""
    lib = load()
    p, n = _ws(ws)
    fc = f.c()
    r = c_report() if report else None
    st = lib.dpar2_als_plain(ctypes.byref(X.c()), ctypes.byref(o.c()), ctypes.byref(fc), _ptr(err_trace), _ptr(U),
                             ctypes.byref(r) if report else None, p, n, _stream(stream))
    d = None
    if report and st in (DPAR2_OK, DPAR2_ENOCONV, DPAR2_ENUMERIC):
        d = _report_dict(r)
        d["status"] = st
    if st == DPAR2_ENOCONV and report:
        return d
    _check(st, d)
    return d


def output_A(X: Tensor, o: Options, A, ws, stream=None):
    """A: float64 device (N, R) receives the first-stage factors A_k."""
    lib = load()
    p, n = _ws(ws)
    _check(lib.dpar2_output_A(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(A), p, n, _stream(stream)))


def release(ws):
    """Frees the library's host-side state (staging, graphs) kept for ws."""
    p, _ = _ws(ws)
    _check(load().dpar2_release(p))


def release_all():
    _check(load().dpar2_release_all())


def compressed_view(X: Tensor, o: Options, ws) -> dict:
    """Copies of the compressed representation (numpy float64): Mt ((KR) x J),
    D (J x R), E (R), F ((KR) x R), Phi (K x L x R), sigma (K x R), xnorm2 (K)."""
    import torch
    lib = load()
    p, n = _ws(ws)
    c = c_compressed()
    _check(lib.dpar2_compressed_view(ctypes.byref(X.c()), ctypes.byref(o.c()), p, n, ctypes.byref(c)))
    torch.cuda.synchronize()
    K, J, R, L = X.K, X.J, o.rank, o.sketch
    shapes = {"Mt": (K * R, J), "D": (J, R), "E": (R,), "F": (K * R, R), "Phi": (K, L, R),
              "sigma": (K, R), "xnorm2": (K,)}
    out = {}
    base = int(ws.data_ptr())
    for name, shp in shapes.items():
        addr = getattr(c, name)
        nel = int(np.prod(shp))
        off = (addr - base) // 8
        assert (addr - base) % 8 == 0
        out[name] = ws[off * 8:(off + nel) * 8].view(torch.float64).cpu().numpy().reshape(shp).copy()
    return out


def report_read(X: Tensor, o: Options, ws, stream=None) -> dict:
    lib = load()
    p, _ = _ws(ws)
    r = c_report()
    st = lib.dpar2_report_read(ctypes.byref(X.c()), ctypes.byref(o.c()), p, ctypes.byref(r), _stream(stream))
    _check(st, _report_dict(r) if st == DPAR2_ENUMERIC else None)
    return _report_dict(r)


def _report_dict(r) -> dict:
    return {"iters": r.iters, "converged": bool(r.converged), "err_last": r.err_last,
            "fit_compressed": r.fit_compressed, "fit_true": r.fit_true, "xnorm2": r.xnorm2,
            "warn_bits": r.warn_bits}


class _Batch:
    """ctypes arrays describing a batch of tensors (kept alive by the caller
    for the duration of a call)."""

    def __init__(self, Xs, os_, omega1s=None, omega2s=None, fs=None):
        n = len(Xs)
        assert n >= 1 and len(os_) == n
        self.n = n
        self.X = (c_tensor * n)(*[x.c() for x in Xs])
        self.o = (c_opts * n)(*[o.c() for o in os_])
        if omega1s is not None:
            self.om1 = (ctypes.c_void_p * n)(*[_ptr(w) for w in omega1s])
            self.om2 = (ctypes.c_void_p * n)(*[_ptr(w) for w in omega2s])
        if fs is not None:
            self.f = (c_factors * n)(*[f.c() for f in fs])


def batch_workspace_size(Xs, os_) -> int:
    b = _Batch(Xs, os_)
    n = load().dpar2_batch_workspace_size(b.n, b.X, b.o)
    if n == 0:
        raise Dpar2Error(DPAR2_EINVAL, last_error())
    return int(n)


def alloc_batch_workspace(Xs, os_, device="cuda:0"):
    import torch
    return torch.empty(batch_workspace_size(Xs, os_) + 256, dtype=torch.uint8, device=device)


def decompose_batch(Xs, os_, omega1s, omega2s, fs, ws, stream=None):
    """Decomposes every tensor of the batch (factors fs updated in place)."""
    b = _Batch(Xs, os_, omega1s, omega2s, fs)
    p, n = _ws(ws)
    _check(load().dpar2_decompose_batch(b.n, b.X, b.o, b.om1, b.om2, b.f, p, n, _stream(stream)))


def batch_report_read(Xs, os_, ws, stream=None) -> list:
    b = _Batch(Xs, os_)
    p, _ = _ws(ws)
    r = (c_report * b.n)()
    st = load().dpar2_batch_report_read(b.n, b.X, b.o, p, r, _stream(stream))
    _check(st, [_report_dict(r[i]) for i in range(b.n)] if st == DPAR2_ENUMERIC else None)
    return [_report_dict(r[i]) for i in range(b.n)]


def autotune_item_rows(X: Tensor, o: Options, omega1, ws, candidates=(2048, 4096, 8192, 16384), stream=None):
    """(best item_rows, {candidate: median slab-pass ms}); ws must fit the
    smallest candidate (see workspace_size with Options.item_rows)."""
    lib = load()
    p, n = _ws(ws)
    c = (ctypes.c_int32 * len(candidates))(*candidates)
    t = (ctypes.c_float * len(candidates))()
    best = ctypes.c_int32()
    _check(lib.dpar2_autotune_item_rows(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(omega1), c, len(candidates),
                                        p, n, ctypes.byref(best), t, _stream(stream)))
    return int(best.value), {int(k): float(v) for k, v in zip(candidates, t)}


def autotune_slab(X: Tensor, o: Options, omega1, ws, candidates, stream=None):
    """candidates: sequence of (item_rows, wide) pairs.  Returns (the fastest
    pair, [median slab-pass ms of each]); ws must fit every candidate (see
    workspace_size with Options.wide_slab=True if any candidate is wide)."""
    lib = load()
    p, n = _ws(ws)
    m = len(candidates)
    rows = (ctypes.c_int32 * m)(*[int(r) for r, _ in candidates])
    wide = (ctypes.c_int32 * m)(*[1 if w else 0 for _, w in candidates])
    t = (ctypes.c_float * m)()
    best = ctypes.c_int32()
    _check(lib.dpar2_autotune_slab(ctypes.byref(X.c()), ctypes.byref(o.c()), _ptr(omega1), rows, wide, m,
                                   p, n, ctypes.byref(best), t, _stream(stream)))
    return candidates[int(best.value)], [float(v) for v in t]


# --- learned warm start ----------------------------------------------------

WARM_WIDTH = 128


def warm_param_count(rank: int) -> int:
    n = int(load().dpar2_warm_param_count(int(rank)))
    if n == 0:
        raise Dpar2Error(DPAR2_EINVAL, "rank must be in 1..32")
    return n


def warm_features(X: Tensor, o: Options, ws, tok, stream=None):
    """tok: float32 device (K, R(R+1)/2)."""
    p, n = _ws(ws)
    _check(load().dpar2_warm_features(ctypes.byref(X.c()), ctypes.byref(o.c()), p, n, _ptr(tok), _stream(stream)))


def warm_targets(X: Tensor, o: Options, ws, f: Factors, tH, tV, tW, stream=None):
    p, n = _ws(ws)
    fc = f.c()
    _check(load().dpar2_warm_targets(ctypes.byref(X.c()), ctypes.byref(o.c()), p, n, ctypes.byref(fc),
                                     _ptr(tH), _ptr(tV), _ptr(tW), _stream(stream)))


def warm_apply(X: Tensor, o: Options, ws, pH, pV, pW, f: Factors, stream=None):
    p, n = _ws(ws)
    fc = f.c()
    _check(load().dpar2_warm_apply(ctypes.byref(X.c()), ctypes.byref(o.c()), p, n, _ptr(pH), _ptr(pV),
                                   _ptr(pW), ctypes.byref(fc), _stream(stream)))


def _tok_off(tok_off):
    """(device int32 tensor, host int32 array kept alive) of token offsets."""
    import torch
    host = np.ascontiguousarray(np.asarray(tok_off, dtype=np.int32))
    return torch.from_numpy(host).cuda(), host


def warm_forward(rank, tok_off, tok, theta, act, pH, pV, pW, stream=None):
    """tok_off: host sequence of n + 1 token offsets (copied to the device)."""
    dev, host = _tok_off(tok_off)
    _check(load().dpar2_warm_forward(int(rank), len(host) - 1, _ptr(dev), host.ctypes.data, _ptr(tok),
                                     _ptr(theta), _ptr(act), _ptr(pH), _ptr(pV), _ptr(pW), _stream(stream)))


def warm_backward(rank, tok_off, tok, theta, act, pH, pV, pW, tH, tV, tW, grad_part, grad, loss, stream=None):
    dev, host = _tok_off(tok_off)
    _check(load().dpar2_warm_backward(int(rank), len(host) - 1, _ptr(dev), host.ctypes.data, _ptr(tok),
                                      _ptr(theta), _ptr(act), _ptr(pH), _ptr(pV), _ptr(pW), _ptr(tH), _ptr(tV),
                                      _ptr(tW), _ptr(grad_part), _ptr(grad), _ptr(loss), _stream(stream)))


def warm_adam(rank, theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0,
              stream=None):
    _check(load().dpar2_warm_adam(int(rank), _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                  float(beta1), float(beta2), float(eps), float(grad_scale), _stream(stream)))


def profile_enable(on: bool = True):
    _check(load().dpar2_profile_enable(1 if on else 0))


def profile_read():
    """(launches, total_ms) of the slab-pass kernel since the last read."""
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(load().dpar2_profile_read(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def last_error() -> str:
    return load().dpar2_last_error().decode(errors="replace")


def status_string(st: int) -> str:
    return load().dpar2_status_string(int(st)).decode()


# --- post-processing of the factors (Sec. IV-E) ------------------------------

def feature_pcc(V, C, stream=None):
    """C (J x J float64) <- Pearson correlations between the rows of V (J x R)."""
    J, R = int(V.shape[0]), int(V.shape[1])
    _check(load().dpar2_feature_pcc(J, R, _ptr(V), _ptr(C), _stream(stream)))


def slice_similarity(X: Tensor, U, idx, gamma, S, stream=None):
    """S (n x n) <- exp(-gamma ||U_i - U_j||_F^2) over the slices idx (host
    sequence; copied to the device), all of one length."""
    import torch
    host = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    dev = torch.from_numpy(host).to(U.device)
    R = int(U.shape[1])
    _check(load().dpar2_slice_similarity(ctypes.byref(X.c()), R, _ptr(U), len(host), _ptr(dev), host.ctypes.data,
                                         float(gamma), _ptr(S), _stream(stream)))
    return dev


def top_k(v, exclude, k, out, stream=None):
    _check(load().dpar2_top_k(_ptr(v), int(v.numel()), int(exclude), int(k), _ptr(out), _stream(stream)))


def rwr(S, target, r, work, c=0.15, iters=100, stream=None):
    _check(load().dpar2_rwr(_ptr(S), int(S.shape[0]), int(target), float(c), int(iters), _ptr(r), _ptr(work),
                            _stream(stream)))
