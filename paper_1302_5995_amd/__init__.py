"""Python binding of the gfx950 DtN library (libdtn.so).

Argument marshalling only: every step of the build and of the apply runs in
the library's HIP kernels.  PyTorch is used for device memory and streams
when device tensors are passed.  There is no fallback: if the shared library
is missing or no gfx950 device is present, the calls raise.

Layout conventions follow include/dtn.h: node (i, j) of the n x n grid has
index i + n*j; matrices are column-major; the boundary ring (nb = 4(n-1)
nodes) is listed counter-clockwise from the corner (0, 0).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdtn.so")

DTN_OK, DTN_EINVAL, DTN_ENOMEM, DTN_ESINGULAR, DTN_EDEVICE, DTN_EBUSY, DTN_ENOTSUP, DTN_ERANK = 0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
FUSED, PLAIN = 0, 1
CONV_CENTRAL, CONV_PAPER = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
PIVOT_RTOL = 1e-11
PIVOT_AUTO, PIVOT_PARTIAL = 0, 1
RING_R1, RING_R2, RING_R3 = 0, 1, 2
COEF_PDE, COEF_NETWORK = 0, 1

# every symbol include/dtn.h declares
EXPORTS = [
    "dtn_build_desc_init", "dtn_build", "dtn_build_ex", "dtn_build_many", "dtn_apply", "dtn_apply_device",
    "dtn_apply_device_noalloc", "dtn_hbs_compress", "dtn_hbs_get", "dtn_apply_hbs_device",
    "dtn_hbs_invert", "dtn_hbs_inverse_get", "dtn_apply_hbs_inverse_device", "dtn_level_count", "dtn_level_box",
    "dtn_nb", "dtn_export_dense", "dtn_import_dense", "dtn_body_count", "dtn_body_get", "dtn_body_ptr",
    "dtn_apply_body_device", "dtn_body_plan_check", "dtn_device_ptr", "dtn_stats_get", "dtn_free", "dtn_last_error",
    "dtn_version", "dtn_profile_enable", "dtn_profile_select", "dtn_profile_reset", "dtn_profile_read",
    "dtn_plan_check", "dtn_plan_footprint", "dtn_last_build_code", "dtn_plan_check_tiles", "dtn_tune",
    "dtn_tune_enable", "dtn_tune_clear", "dtn_tune_save", "dtn_tune_load", "dtn_tune_size",
    "dtn_srv_create", "dtn_srv_add_op", "dtn_srv_remove_op", "dtn_srv_op_nb", "dtn_srv_submit_apply",
    "dtn_srv_submit_build", "dtn_srv_poll", "dtn_srv_wait", "dtn_srv_replay", "dtn_srv_stats_get",
    "dtn_srv_stats_reset", "dtn_srv_now_ns", "dtn_srv_destroy",
]


class BuildDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("b", C.c_void_p), ("c", C.c_void_p), ("d", C.c_void_p),
        ("coeff_mem", C.c_int), ("leaf", C.c_int), ("tol", C.c_double), ("hbs_min_level", C.c_int),
        ("precision", C.c_int), ("batching", C.c_int), ("conv", C.c_int), ("device", C.c_int),
        ("stream", C.c_void_p), ("pivoting", C.c_int), ("ring_rows", C.c_int), ("coef_form", C.c_int),
        ("capture_level", C.c_int), ("pad0", C.c_int), ("budget_bytes", C.c_size_t), ("kii_tol", C.c_double),
        ("n_body", C.c_int), ("pad1", C.c_int), ("body_nodes", C.c_void_p),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("nb", C.c_int), ("leaf", C.c_int), ("levels", C.c_int),
        ("precision", C.c_int), ("batching", C.c_int),
        ("build_ms", C.c_double), ("flops", C.c_double),
        ("level_ms", C.c_double * 32), ("level_flops", C.c_double * 32), ("max_rank", C.c_int * 32),
        ("min_pivot_ratio", C.c_double), ("pivoting_used", C.c_int),
        ("op_bytes", C.c_size_t), ("peak_workspace_bytes", C.c_size_t), ("structured_merges", C.c_int),
        ("max_growth", C.c_double),
    ]

    def as_dict(self) -> dict:
        L = self.levels
        return {
            "n": self.n, "nb": self.nb, "leaf": self.leaf, "levels": L, "precision": self.precision,
            "batching": self.batching, "build_ms": self.build_ms, "flops": self.flops,
            "level_ms": list(self.level_ms[: L + 1]), "level_flops": list(self.level_flops[: L + 1]),
            "max_rank": list(self.max_rank[: L + 1]),
            "min_pivot_ratio": self.min_pivot_ratio, "pivoting_used": self.pivoting_used,
            "op_bytes": self.op_bytes,
            "peak_workspace_bytes": self.peak_workspace_bytes, "structured_merges": self.structured_merges,
            "max_growth": self.max_growth,
        }


class HbsInfo(C.Structure):
    _fields_ = [("leaf", C.c_int), ("levels", C.c_int), ("nodes", C.c_int), ("launches", C.c_int),
                ("tol", C.c_double), ("bytes", C.c_size_t), ("max_rank", C.c_int * 32)]

    def as_dict(self) -> dict:
        return {"leaf": self.leaf, "levels": self.levels, "nodes": self.nodes, "launches": self.launches,
                "tol": self.tol, "bytes": self.bytes, "max_rank": list(self.max_rank[: self.levels + 1])}


class ProfEntry(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_longlong), ("total_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


class SrvResult(C.Structure):
    _fields_ = [("status", C.c_int), ("op_id", C.c_int), ("k", C.c_int), ("batch_cols", C.c_int),
                ("t_arrival_ns", C.c_longlong), ("t_start_ns", C.c_longlong), ("t_done_ns", C.c_longlong)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class SrvStats(C.Structure):
    _fields_ = [("applies_done", C.c_longlong), ("builds_done", C.c_longlong), ("solves_done", C.c_longlong),
                ("batches", C.c_longlong), ("refused", C.c_longlong), ("budget_bytes", C.c_size_t),
                ("resident_bytes", C.c_size_t), ("resident_ops", C.c_int), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("mean_batch_cols", C.c_double),
                ("span_s", C.c_double), ("solves_per_s", C.c_double), ("build_p50_ms", C.c_double),
                ("build_p99_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class SrvRequest(C.Structure):
    _fields_ = [("t_offset_ns", C.c_longlong), ("op_id", C.c_int), ("k", C.c_int), ("G", C.c_void_p),
                ("Y", C.c_void_p), ("build", C.c_void_p)]


class DtnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dtn error {code}: {msg}")
        self.code = code


_lib: Optional[C.CDLL] = None


def lib_path() -> str:
    return LIB_PATH


def load() -> C.CDLL:
    """Load libdtn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1302_5995_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "dtn_build_desc_init": (None, [C.POINTER(BuildDesc)]),
        "dtn_build": (P, [C.c_int, P, P, P, C.c_int, C.c_double]),
        "dtn_build_ex": (P, [C.POINTER(BuildDesc)]),
        "dtn_build_many": (C.c_int, [C.c_int, C.POINTER(BuildDesc), C.POINTER(P)]),
        "dtn_apply": (C.c_int, [P, P, C.c_int, P]),
        "dtn_apply_device": (C.c_int, [P, P, C.c_int, C.c_int, P, C.c_int, P]),
        "dtn_apply_device_noalloc": (C.c_int, [P, P, C.c_int, C.c_int, P, C.c_int, P]),
        "dtn_hbs_compress": (C.c_int, [P, C.c_double, C.c_int, C.c_int]),
        "dtn_hbs_get": (C.c_int, [P, C.POINTER(HbsInfo)]),
        "dtn_apply_hbs_device": (C.c_int, [P, P, C.c_int, C.c_int, P, C.c_int, P]),
        "dtn_hbs_invert": (C.c_int, [P, C.c_double, C.c_int]),
        "dtn_level_count": (C.c_int, [P]),
        "dtn_level_box": (C.c_int, [P, C.c_int, C.POINTER(C.c_int), P, C.c_int]),
        "dtn_hbs_inverse_get": (C.c_int, [P, C.POINTER(HbsInfo)]),
        "dtn_apply_hbs_inverse_device": (C.c_int, [P, P, C.c_int, C.c_int, P, C.c_int, P]),
        "dtn_nb": (C.c_int, [P]),
        "dtn_export_dense": (C.c_int, [P, P, C.c_int]),
        "dtn_import_dense": (P, [C.c_int, P, C.c_int, C.c_int]),
        "dtn_body_plan_check": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]),
        "dtn_body_count": (C.c_int, [P]),
        "dtn_body_get": (C.c_int, [P, P, C.c_int]),
        "dtn_body_ptr": (P, [P]),
        "dtn_apply_body_device": (C.c_int, [P, P, C.c_int, P, C.c_int, C.c_int, P, C.c_int, P]),
        "dtn_device_ptr": (P, [P]),
        "dtn_stats_get": (C.c_int, [P, C.POINTER(Stats)]),
        "dtn_free": (None, [P]),
        "dtn_last_error": (C.c_char_p, []),
        "dtn_last_build_code": (C.c_int, []),
        "dtn_version": (C.c_char_p, []),
        "dtn_profile_enable": (C.c_int, [C.c_int]),
        "dtn_profile_select": (C.c_int, [C.c_char_p]),
        "dtn_plan_check": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int]),
        "dtn_plan_footprint": (C.c_int, [C.POINTER(BuildDesc), C.POINTER(C.c_size_t), C.c_char_p, C.c_int]),
        "dtn_plan_check_tiles": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int]),
        "dtn_tune": (C.c_int, [C.POINTER(BuildDesc), C.c_int, C.c_char_p, C.c_int]),
        "dtn_tune_enable": (C.c_int, [C.c_int]),
        "dtn_tune_clear": (C.c_int, []),
        "dtn_tune_save": (C.c_int, [C.c_char_p]),
        "dtn_tune_load": (C.c_int, [C.c_char_p]),
        "dtn_tune_size": (C.c_int, []),
        "dtn_profile_reset": (C.c_int, []),
        "dtn_profile_read": (C.c_int, [C.POINTER(ProfEntry), C.c_int]),
        "dtn_srv_create": (P, [C.c_size_t, C.c_int, C.c_int]),
        "dtn_srv_add_op": (C.c_int, [P, P]),
        "dtn_srv_remove_op": (C.c_int, [P, C.c_int]),
        "dtn_srv_op_nb": (C.c_int, [P, C.c_int]),
        "dtn_srv_submit_apply": (C.c_longlong, [P, C.c_int, P, C.c_int, P]),
        "dtn_srv_submit_build": (C.c_longlong, [P, C.POINTER(BuildDesc)]),
        "dtn_srv_poll": (C.c_int, [P, C.c_longlong]),
        "dtn_srv_wait": (C.c_int, [P, C.c_longlong, C.POINTER(SrvResult)]),
        "dtn_srv_replay": (C.c_int, [P, C.c_int, C.POINTER(SrvRequest), C.POINTER(C.c_longlong)]),
        "dtn_srv_stats_get": (C.c_int, [P, C.POINTER(SrvStats)]),
        "dtn_srv_stats_reset": (C.c_int, [P]),
        "dtn_srv_now_ns": (C.c_longlong, []),
        "dtn_srv_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().dtn_last_error().decode()


def _check(code: int):
    if code != DTN_OK:
        raise DtnError(code, last_error())


def _host_field(f, n):
    if f is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
    if a.size != n * n:
        raise ValueError("coefficient field must have n*n entries")
    return a, a.ctypes.data


def _dev_field(f, n):
    if f is None:
        return None, None
    if f.dtype != __import__("torch").float64 or not f.is_contiguous() or f.numel() != n * n:
        raise ValueError("device coefficient must be a contiguous float64 tensor with n*n entries")
    return f, f.data_ptr()


_side_streams = {}


def _on_torch_stream(device, stream, launch):
    """Run launch(hipStream) ordered with torch's current stream on `device`.

    The C ABI reads a NULL stream as the library's own (non-blocking) stream, so torch's legacy
    default stream (handle 0) cannot be named directly: the work then goes to a side stream of
    default priority that first waits for torch's current stream, and torch's current stream waits
    for it afterwards (inputs produced and outputs consumed in torch's order)."""
    import torch
    if stream is not None:
        return launch(stream)
    cur = torch.cuda.current_stream(device)
    if cur.cuda_stream != 0:
        return launch(cur.cuda_stream)
    key = torch.device(device).index
    side = _side_streams.get(key)
    if side is None:
        side = _side_streams[key] = torch.cuda.Stream(device=device)
    side.wait_stream(cur)
    rc = launch(side.cuda_stream)
    cur.wait_stream(side)
    return rc


class Operator:
    """A built DtN operator resident on the GPU (owns its device memory)."""

    def __init__(self, handle: int):
        self._h = handle
        self.nb = load().dtn_nb(handle)

    @property
    def handle(self) -> int:
        return self._h

    def apply(self, G: np.ndarray) -> np.ndarray:
        """Y = T G for host data (nb x k, or length nb)."""
        G = np.asarray(G, dtype=np.float64)
        vec = G.ndim == 1
        G2 = np.asfortranarray(G.reshape(self.nb, -1))
        k = G2.shape[1]
        Y = np.empty((self.nb, k), dtype=np.float64, order="F")
        _check(load().dtn_apply(self._h, G2.ctypes.data, k, Y.ctypes.data))
        return Y[:, 0] if vec else Y

    def apply_device(self, G, Y=None, stream=None, noalloc=False):
        """Y = T G for torch CUDA float64 tensors of shape (nb, k) stored column-major.
        noalloc: call dtn_apply_device_noalloc (no device allocation; Y must be given)."""
        import torch
        if G.dim() != 2 or G.shape[0] != self.nb or G.dtype != torch.float64 or not G.is_cuda:
            raise ValueError("G must be a CUDA float64 tensor of shape (nb, k)")
        if G.stride(0) != 1:
            raise ValueError("G must be column-major (stride(0) == 1)")
        k = G.shape[1]
        if Y is None:
            if noalloc:
                raise ValueError("the allocation-free apply needs a caller-provided Y")
            Y = torch.empty((k, self.nb), dtype=torch.float64, device=G.device).t()
        if Y.dim() != 2 or tuple(Y.shape) != (self.nb, k) or Y.dtype != torch.float64 or Y.stride(0) != 1:
            raise ValueError("Y must be a column-major CUDA float64 tensor of shape (nb, k)")
        ldg = G.stride(1) if k > 1 else self.nb
        ldy = Y.stride(1) if k > 1 else self.nb
        fn = load().dtn_apply_device_noalloc if noalloc else load().dtn_apply_device
        _check(_on_torch_stream(G.device, stream,
                                lambda s: fn(self._h, G.data_ptr(), ldg, k, Y.data_ptr(), ldy, s)))
        return Y

    def hbs_compress(self, tol: float, leaf: int = 64, drop_dense: bool = False) -> dict:
        """Compress T into HBS form (Section 4); returns the factors' description."""
        _check(load().dtn_hbs_compress(self._h, float(tol), int(leaf), int(bool(drop_dense))))
        return self.hbs_info()

    def hbs_info(self) -> dict:
        info = HbsInfo()
        _check(load().dtn_hbs_get(self._h, C.byref(info)))
        return info.as_dict()

    def apply_hbs_device(self, G, Y=None, stream=None):
        """Y = T_HBS G through the telescoping factorisation (torch CUDA float64, column-major)."""
        import torch
        k = G.shape[1]
        if Y is None:
            Y = torch.empty((k, self.nb), dtype=torch.float64, device=G.device).t()
        ldg = G.stride(1) if k > 1 else self.nb
        ldy = Y.stride(1) if k > 1 else self.nb
        _check(_on_torch_stream(G.device, stream,
                                lambda s: load().dtn_apply_hbs_device(self._h, G.data_ptr(), ldg, k, Y.data_ptr(),
                                                                      ldy, s)))
        return Y

    def hbs_invert(self, tol: float, leaf: int = 64) -> dict:
        """Factors of T^{-1} by Algorithm 1 (Section 5.1) from equal-rank HBS factors of T; returns
        their description."""
        _check(load().dtn_hbs_invert(self._h, float(tol), int(leaf)))
        return self.hbs_inverse_info()

    def hbs_inverse_info(self) -> dict:
        info = HbsInfo()
        _check(load().dtn_hbs_inverse_get(self._h, C.byref(info)))
        return info.as_dict()

    def apply_hbs_inverse_device(self, X, Y=None, stream=None):
        """Y = T^{-1} X through Algorithm 2 (torch CUDA float64, column-major)."""
        import torch
        k = X.shape[1]
        if Y is None:
            Y = torch.empty((k, self.nb), dtype=torch.float64, device=X.device).t()
        ldx = X.stride(1) if k > 1 else self.nb
        ldy = Y.stride(1) if k > 1 else self.nb
        _check(_on_torch_stream(X.device, stream,
                                lambda s: load().dtn_apply_hbs_inverse_device(self._h, X.data_ptr(), ldx, k,
                                                                              Y.data_ptr(), ldy, s)))
        return Y

    def level_boxes(self, with_schur: bool = True) -> list:
        """The captured level (capture_level): [(rect (x0, x1, y0, y1), S or None), ...], S in ring order."""
        lib = load()
        cnt = lib.dtn_level_count(self._h)
        if cnt < 0:
            raise DtnError(cnt, last_error())
        out = []
        rect = (C.c_int * 4)()
        for q in range(cnt):
            _check(lib.dtn_level_box(self._h, q, rect, None, 0))
            x0, x1, y0, y1 = rect
            S = None
            if with_schur:
                m = 2 * (x1 - x0 - 1) + 2 * (y1 - y0 - 1)
                S = np.empty((m, m), dtype=np.float64, order="F")
                _check(lib.dtn_level_box(self._h, q, rect, S.ctypes.data, m))
            out.append(((x0, x1, y0, y1), S))
        return out

    def dense(self) -> np.ndarray:
        T = np.empty((self.nb, self.nb), dtype=np.float64, order="F")
        _check(load().dtn_export_dense(self._h, T.ctypes.data, self.nb))
        return T

    @property
    def body_count(self) -> int:
        return load().dtn_body_count(self._h)

    def body(self) -> np.ndarray:
        """F (nb x n_body) of a build with body loads: boundary fluxes per unit load (Section 7.3)."""
        F = np.empty((self.nb, self.body_count), dtype=np.float64, order="F")
        _check(load().dtn_body_get(self._h, F.ctypes.data, self.nb))
        return F

    def apply_body_device(self, G, Q, stream=None):
        """Y = T G + F Q for torch CUDA float64 tensors (nb x k and n_body x k, column-major)."""
        import torch
        k = G.shape[1]
        for X, rows in ((G, self.nb), (Q, self.body_count)):
            if X.dim() != 2 or X.shape != (rows, k) or X.dtype != torch.float64 or not X.is_cuda or X.stride(0) != 1:
                raise ValueError("G (nb x k) and Q (n_body x k) must be column-major CUDA float64 tensors")
        Y = torch.empty((k, self.nb), dtype=torch.float64, device=G.device).t()
        _check(load().dtn_apply_body_device(self._h, G.data_ptr(), G.stride(1), Q.data_ptr(), Q.stride(1), k,
                                            Y.data_ptr(), Y.stride(1), stream))
        return Y

    def device_ptr(self) -> int:
        return load().dtn_device_ptr(self._h)

    def stats(self) -> dict:
        st = Stats()
        _check(load().dtn_stats_get(self._h, C.byref(st)))
        return st.as_dict()

    def free(self):
        if self._h:
            load().dtn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def make_desc(n, b=None, c=None, d=None, leaf=32, tol=0.0, precision=FP64, batching=FUSED,
              conv=CONV_CENTRAL, device=0, stream=None, hbs_min_level=-1, pivoting=PIVOT_AUTO,
              ring_rows=RING_R1, coef_form=COEF_PDE, capture_level=-1, budget_bytes=0, kii_tol=0.0,
              body_nodes=None):
    """Fill a BuildDesc; returns (desc, keepalive) - keepalive holds the arrays referenced."""
    lib = load()
    D = BuildDesc()
    lib.dtn_build_desc_init(C.byref(D))
    D.n, D.leaf, D.tol = n, leaf, float(tol)
    D.precision, D.batching, D.conv, D.device = precision, batching, conv, device
    D.hbs_min_level = hbs_min_level
    D.stream = stream
    D.pivoting = pivoting
    D.ring_rows = ring_rows
    D.coef_form = coef_form
    D.capture_level = capture_level
    D.budget_bytes = int(budget_bytes)
    D.kii_tol = float(kii_tol)
    keep = []
    on_dev = any(f is not None and hasattr(f, "is_cuda") and f.is_cuda for f in (b, c, d))
    D.coeff_mem = MEM_DEVICE if on_dev else MEM_HOST
    conv_f = _dev_field if on_dev else _host_field
    ptrs = []
    for f in (b, c, d):
        a, p = conv_f(f, n)
        keep.append(a)
        ptrs.append(p)
    D.b, D.c, D.d = ptrs
    if body_nodes is not None:
        # loads at nodes (i, j): node index i + n j
        nodes = np.asarray(body_nodes, dtype=np.int64).reshape(-1, 2)
        idx = np.ascontiguousarray(nodes[:, 0] + n * nodes[:, 1], dtype=np.int32)
        keep.append(idx)
        D.n_body = int(idx.size)
        D.body_nodes = idx.ctypes.data
    return D, keep


def build(n, b=None, c=None, d=None, leaf=32, tol=0.0, **opts) -> Operator:
    """Build the DtN operator (host numpy or device torch coefficient fields; None = 0)."""
    D, keep = make_desc(n, b, c, d, leaf, tol, **opts)
    h = load().dtn_build_ex(C.byref(D))
    del keep
    if not h:
        code = load().dtn_last_build_code()
        raise DtnError(code if code != DTN_OK else DTN_EINVAL, last_error())
    return Operator(h)


def import_dense(T: np.ndarray, device: int = 0) -> Operator:
    """A handle holding the square matrix T (host), e.g. an operator saved with Operator.dense()."""
    T = np.asfortranarray(np.asarray(T, dtype=np.float64))
    if T.ndim != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    h = load().dtn_import_dense(T.shape[0], T.ctypes.data, T.shape[0], device)
    if not h:
        raise DtnError(DTN_EINVAL, last_error())
    return Operator(h)


def build_many(problems: Sequence[dict]) -> list:
    """Build several problems together (dicts of build() keyword arguments)."""
    lib = load()
    descs = (BuildDesc * len(problems))()
    keep = []
    for q, p in enumerate(problems):
        p = dict(p)
        D, k = make_desc(p.pop("n"), p.pop("b", None), p.pop("c", None), p.pop("d", None), **p)
        descs[q] = D
        keep.append(k)
    out = (C.c_void_p * len(problems))()
    _check(lib.dtn_build_many(len(problems), descs, out))
    return [Operator(out[q]) for q in range(len(problems))]


def version() -> str:
    return load().dtn_version().decode()


def profile_enable(on: bool = True):
    _check(load().dtn_profile_enable(1 if on else 0))


def profile_select(families=None):
    """Record only the named kernel families while profiling (None or empty: all)."""
    arg = ",".join(families).encode() if families else None
    _check(load().dtn_profile_select(arg))


def profile_reset():
    _check(load().dtn_profile_reset())


def plan_check(n, leaf=32, tol=0.0, mixed=False, fast=True, sym=0):
    """Host-only check that every device descriptor of the build plan stays inside its buffers
    (sym: 0 convection, 1 symmetric definite, 2 symmetric indefinite)."""
    _check(load().dtn_plan_check(int(n), int(leaf), float(tol), int(bool(mixed)), int(bool(fast)), int(sym)))


def body_plan_check(n, nodes, leaf=32, fast=True, sym=0):
    """Host-only check of the body-load plan for loads at nodes (i, j) (Section 7.3)."""
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 2)
    idx = np.ascontiguousarray(nodes[:, 0] + n * nodes[:, 1], dtype=np.int32)
    _check(load().dtn_body_plan_check(int(n), int(leaf), int(bool(fast)), int(sym), int(idx.size), idx.ctypes.data))


def plan_check_tiles(n, leaf=32, tol=0.0, mixed=False, fast=True, sym=0, tile=-1):
    """plan_check with every FP64 product launch that can take it forced to one tile configuration."""
    _check(load().dtn_plan_check_tiles(int(n), int(leaf), float(tol), int(bool(mixed)), int(bool(fast)), int(sym),
                                       int(tile)))


def tune(n, b=None, c=None, d=None, leaf=32, tol=0.0, reps=3, **opts) -> dict:
    """Time the build's product launches under each tile configuration and record the fastest per
    launch shape (see dtn_tune); returns {signature: {"tile": t, "ms": {tile: ms per build}}}."""
    import json
    D, keep = make_desc(n, b, c, d, leaf, tol, **opts)
    buf = C.create_string_buffer(1 << 20)
    rc = load().dtn_tune(C.byref(D), int(reps), buf, len(buf))
    del keep
    if rc < 0:
        raise DtnError(rc, last_error())
    return json.loads(buf.value.decode() or "{}")


def tune_enable(on: bool = True):
    _check(load().dtn_tune_enable(1 if on else 0))


def tune_clear():
    _check(load().dtn_tune_clear())


def tune_save(path: str):
    _check(load().dtn_tune_save(path.encode()))


def tune_load(path: str):
    _check(load().dtn_tune_load(path.encode()))


def tune_size() -> int:
    return load().dtn_tune_size()


def plan_footprint(n, b=None, c=None, d=None, leaf=32, tol=0.0, **opts):
    """Host-only: (device bytes of the plans a build with these options may allocate, plan-cache key)."""
    D, keep = make_desc(n, b, c, d, leaf, tol, **opts)
    nbytes = C.c_size_t(0)
    key = C.create_string_buffer(512)
    _check(load().dtn_plan_footprint(C.byref(D), C.byref(nbytes), key, 512))
    del keep
    return int(nbytes.value), key.value.decode()


def profile_read() -> dict:
    """Per kernel family: launches, total_ms, flops, bytes (from HIP events around each launch)."""
    lib = load()
    cnt = lib.dtn_profile_read(None, 0)
    arr = (ProfEntry * max(cnt, 1))()
    got = lib.dtn_profile_read(arr, cnt)
    return {arr[q].name.decode(): {"launches": arr[q].launches, "total_ms": arr[q].total_ms,
                                   "flops": arr[q].flops, "bytes": arr[q].bytes} for q in range(got)}


class Server:
    """Serving loop on one GPU: resident operators, continuous batching of applies, builds
    interleaved, admission by HBM footprint (see include/dtn.h).  Host arrays handed to
    submit_apply / submit_build are kept alive here until their ticket is waited for."""

    def __init__(self, budget_bytes: int, device: int = 0, max_batch_cols: int = 64):
        h = load().dtn_srv_create(int(budget_bytes), device, max_batch_cols)
        if not h:
            raise DtnError(DTN_EINVAL, last_error())
        self._h = h
        self.max_batch_cols = max_batch_cols
        self._keep = {}
        self._nb = {}

    def add_op(self, op: Operator) -> int:
        r = load().dtn_srv_add_op(self._h, op.handle)
        if r < 0:
            raise DtnError(r, last_error())
        self._nb[r] = op.nb
        return r

    def remove_op(self, op_id: int):
        _check(load().dtn_srv_remove_op(self._h, op_id))
        self._nb.pop(op_id, None)

    def op_nb(self, op_id: int) -> int:
        r = load().dtn_srv_op_nb(self._h, op_id)
        if r < 0:
            raise DtnError(r, last_error())
        return r

    def submit_apply(self, op_id: int, G: np.ndarray) -> int:
        nb = self.op_nb(op_id)
        G2 = np.asfortranarray(np.asarray(G, dtype=np.float64).reshape(nb, -1))
        Y = np.empty_like(G2, order="F")
        t = load().dtn_srv_submit_apply(self._h, op_id, G2.ctypes.data, G2.shape[1], Y.ctypes.data)
        if t < 0:
            raise DtnError(int(t), last_error())
        self._keep[t] = (G2, Y)
        return t

    def submit_build(self, n, b=None, c=None, d=None, leaf=32, **opts) -> int:
        D, keep = make_desc(n, b, c, d, leaf, **opts)
        t = load().dtn_srv_submit_build(self._h, C.byref(D))
        if t < 0:
            raise DtnError(int(t), last_error())
        self._keep[t] = (keep, None)
        return t

    def poll(self, ticket: int) -> bool:
        r = load().dtn_srv_poll(self._h, ticket)
        if r < 0:
            raise DtnError(r, last_error())
        return r == 1

    def wait(self, ticket: int):
        """Wait for a ticket: returns (Y or None, result dict); raises on a failed request."""
        res = SrvResult()
        st = load().dtn_srv_wait(self._h, ticket, C.byref(res))
        keep = self._keep.pop(ticket, (None, None))
        if st != DTN_OK:
            raise DtnError(st, f"request {ticket} failed")
        return keep[1], res.as_dict()

    def replay(self, schedule):
        """schedule: list of (t_offset_s, op_id, G) or (t_offset_s, op_id, G, Y) with Y a
        Fortran-ordered float64 output of G's shape, or (t_offset_s, "build", kwargs) for a build
        request (dtn.build keyword arguments, host coefficient arrays); submits each request at its
        time (open loop).  Returns the tickets in schedule order."""
        reqs = (SrvRequest * len(schedule))()
        for q, item in enumerate(schedule):
            if isinstance(item[1], str) and item[1] == "build":
                p = dict(item[2])
                D, keep = make_desc(p.pop("n"), p.pop("b", None), p.pop("c", None), p.pop("d", None), **p)
                Dp = C.pointer(D)
                reqs[q] = SrvRequest(int(item[0] * 1e9), -1, 0, None, None, C.cast(Dp, C.c_void_p))
                self._keep[("pending", q)] = ((D, Dp, keep), None)
                continue
            t, op_id, G = item[:3]
            nb = self._nb.get(op_id) or self.op_nb(op_id)
            G2 = np.asfortranarray(np.asarray(G, dtype=np.float64).reshape(nb, -1))
            Y = item[3] if len(item) > 3 else np.empty_like(G2, order="F")
            if Y.shape != G2.shape or Y.dtype != np.float64 or not Y.flags.f_contiguous:
                raise ValueError("Y must be a Fortran-ordered float64 array of G's shape")
            reqs[q] = SrvRequest(int(t * 1e9), op_id, G2.shape[1], G2.ctypes.data, Y.ctypes.data, None)
            self._keep[("pending", q)] = (G2, Y)
        tickets = (C.c_longlong * len(schedule))()
        rc = load().dtn_srv_replay(self._h, len(schedule), reqs, tickets)
        out = []
        for q in range(len(schedule)):
            kp = self._keep.pop(("pending", q))
            if tickets[q] >= 0:
                self._keep[tickets[q]] = kp
            out.append(int(tickets[q]))
        _check(rc)
        return out

    def stats(self) -> dict:
        st = SrvStats()
        _check(load().dtn_srv_stats_get(self._h, C.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        _check(load().dtn_srv_stats_reset(self._h))

    def close(self):
        if self._h:
            load().dtn_srv_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_ns() -> int:
    return load().dtn_srv_now_ns()
