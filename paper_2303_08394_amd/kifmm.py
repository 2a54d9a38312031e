"""Python binding of libkifmm.so (include/kifmm.h): argument marshalling only.

Every step of the evaluation runs in the HIP library; PyTorch supplies the
device memory and the stream.  Importing this module never falls back to a
CPU path: if the library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkifmm.so")

FP64, FP32, M2L_BF16X3, M2L_BF16X5, M2L_F16X3, FP64_M2L_FP32, FP64_M2L_F16X3 = range(7)
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": M2L_BF16X3, "bf16x5": M2L_BF16X5,
              "f16x3": M2L_F16X3, "fp64+m2l_fp32": FP64_M2L_FP32, "fp64+m2l_f16x3": FP64_M2L_F16X3}
LIST_U, LIST_V, LIST_W, LIST_X = 0, 1, 2, 3
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSUPPORTED"}


class KifmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class TreeParams(C.Structure):
    _fields_ = [("uniform_depth", C.c_int32), ("ncrit", C.c_int32), ("max_depth", C.c_int32),
                ("balance", C.c_int32), ("root_center", C.c_double * 3),
                ("root_halfwidth", C.c_double)]


class TreeInfo(C.Structure):
    _fields_ = [("n_src", C.c_int64), ("n_tgt", C.c_int64), ("depth", C.c_int32),
                ("n_boxes", C.c_int32), ("n_leaves", C.c_int32), ("reserved", C.c_int32),
                ("n_u", C.c_int64), ("n_v", C.c_int64), ("n_w", C.c_int64), ("n_x", C.c_int64),
                ("root_center", C.c_double * 3), ("root_halfwidth", C.c_double)]


_lib = None
EXPORTED = [
    "kifmm_build_tree", "kifmm_build_tree_device", "kifmm_tree_get_info", "kifmm_tree_export_boxes",
    "kifmm_tree_export_list", "kifmm_tree_export_perm", "kifmm_tree_update_points",
    "kifmm_precompute_operators", "kifmm_precompute_operators_ex", "kifmm_precompute_operators_screened",
    "kifmm_ops_save", "kifmm_ops_load",
    "kifmm_ops_export", "kifmm_ops_n", "kifmm_ops_levels", "kifmm_evaluate", "kifmm_evaluate_noalloc",
    "kifmm_evaluate_gradient", "kifmm_evaluate_batch",
    "kifmm_evaluate_simple", "kifmm_set_profiling", "kifmm_n_phases", "kifmm_phase_name",
    "kifmm_get_phase_times", "kifmm_graph_captures", "kifmm_debug_fail_allocations", "kifmm_debug_buffer", "kifmm_set_tuning", "kifmm_get_tuning", "kifmm_tree_destroy", "kifmm_ops_destroy", "kifmm_last_error",
]


def lib():
    """Loads libkifmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2303_08394_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    P, D, I32, I64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    L.kifmm_build_tree.argtypes = [D, I64, D, I64, C.POINTER(TreeParams), C.POINTER(P)]
    L.kifmm_build_tree_device.argtypes = [P, I64, P, I64, C.POINTER(TreeParams), P, C.POINTER(P)]
    L.kifmm_tree_get_info.argtypes = [P, C.POINTER(TreeInfo)]
    L.kifmm_tree_export_boxes.argtypes = [P, P, P, P, P, P, P]
    L.kifmm_tree_export_list.argtypes = [P, I32, P, P]
    L.kifmm_tree_export_perm.argtypes = [P, P, P]
    L.kifmm_tree_update_points.argtypes = [P, P, P, P]
    L.kifmm_precompute_operators.argtypes = [I32, C.c_double, C.POINTER(P)]
    L.kifmm_precompute_operators_ex.argtypes = [I32, C.c_double, I32, C.POINTER(P)]
    L.kifmm_precompute_operators_screened.argtypes = [I32, C.c_double, C.c_double, C.c_double, I32, I32,
                                                      C.POINTER(P)]
    L.kifmm_ops_save.argtypes = [P, C.c_char_p]
    L.kifmm_ops_load.argtypes = [C.c_char_p, I32, C.c_double, C.POINTER(P)]
    L.kifmm_ops_export.argtypes = [P, I32, D, I64]
    L.kifmm_ops_n.argtypes = [P]
    L.kifmm_ops_n.restype = I32
    L.kifmm_ops_levels.argtypes = [P]
    L.kifmm_ops_levels.restype = I32
    L.kifmm_evaluate.argtypes = [P, P, P, I32, P, I32, C.c_int, P]
    L.kifmm_evaluate_noalloc.argtypes = [P, P, P, I32, P, I32, C.c_int, P]
    L.kifmm_evaluate_gradient.argtypes = [P, P, P, I32, P, I32, C.c_int, P]
    L.kifmm_evaluate_batch.argtypes = [I32, C.POINTER(P), P, C.POINTER(P), C.POINTER(P), I32,
                                       C.c_int, P]
    L.kifmm_evaluate_simple.argtypes = [D, D, I64, D, I64, I32, D]
    L.kifmm_set_profiling.argtypes = [I32]
    L.kifmm_n_phases.restype = I32
    L.kifmm_phase_name.argtypes = [I32]
    L.kifmm_phase_name.restype = C.c_char_p
    L.kifmm_get_phase_times.argtypes = [D, C.POINTER(I64)]
    L.kifmm_graph_captures.argtypes = []
    L.kifmm_graph_captures.restype = I64
    L.kifmm_debug_fail_allocations.argtypes = [I64]
    L.kifmm_debug_fail_allocations.restype = None
    L.kifmm_debug_buffer.argtypes = [P, I32, I32, I32, D, I64]
    L.kifmm_set_tuning.argtypes = [C.c_char_p, I32]
    L.kifmm_get_tuning.argtypes = [C.c_char_p, C.POINTER(I32)]
    L.kifmm_tree_destroy.argtypes = [P]
    L.kifmm_tree_destroy.restype = None
    L.kifmm_ops_destroy.argtypes = [P]
    L.kifmm_ops_destroy.restype = None
    L.kifmm_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("kifmm_ops_n", "kifmm_n_phases", "kifmm_phase_name", "kifmm_last_error",
                        "kifmm_graph_captures", "kifmm_debug_fail_allocations",
                        "kifmm_tree_destroy", "kifmm_ops_destroy"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise KifmmError(st, lib().kifmm_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _params(uniform_depth, ncrit, max_depth, balance, center, halfwidth) -> TreeParams:
    prm = TreeParams()
    prm.uniform_depth = uniform_depth
    prm.ncrit = ncrit
    prm.max_depth = max_depth
    prm.balance = 1 if balance else 0
    if halfwidth and halfwidth > 0:
        prm.root_center[:] = [float(v) for v in center]
        prm.root_halfwidth = float(halfwidth)
    return prm


class Tree:
    """Octree + interaction lists built by the library (host)."""

    def __init__(self, src, tgt=None, *, uniform_depth: int = -1, ncrit: int = 64,
                 max_depth: int = 12, balance: bool = True, center=None, halfwidth: float = 0.0,
                 _handle=None):
        if _handle is not None:
            self._h = _handle
            return
        L = lib()
        src = np.ascontiguousarray(src, dtype=np.float64)
        tgt = src if tgt is None else np.ascontiguousarray(tgt, dtype=np.float64)
        prm = _params(uniform_depth, ncrit, max_depth, balance, center, halfwidth)
        h = C.c_void_p()
        _check(L.kifmm_build_tree(_dptr(src), len(src), _dptr(tgt), len(tgt), C.byref(prm), C.byref(h)))
        self._h = h

    @classmethod
    def on_device(cls, src, tgt=None, *, stream=None, uniform_depth: int = -1, ncrit: int = 64,
                  max_depth: int = 12, balance: bool = True, center=None, halfwidth: float = 0.0):
        """The same tree built on the GPU (kifmm_build_tree_device) from
        contiguous float64 CUDA tensors [n][3]; tgt None: the sources."""
        import torch
        for a in (src, tgt):
            if a is not None and (not a.is_cuda or a.dtype != torch.float64 or a.dim() != 2
                                  or a.shape[1] != 3 or not a.is_contiguous()):
                raise ValueError("on_device: contiguous float64 CUDA tensors of shape [n, 3]")
        t = src if tgt is None else tgt
        prm = _params(uniform_depth, ncrit, max_depth, balance, center, halfwidth)
        h = C.c_void_p()
        _check(lib().kifmm_build_tree_device(C.c_void_p(src.data_ptr()), src.shape[0], C.c_void_p(t.data_ptr()),
                                             t.shape[0], C.byref(prm), _stream_ptr(stream), C.byref(h)))
        return cls(None, _handle=h)

    @property
    def handle(self):
        return self._h

    def info(self) -> TreeInfo:
        inf = TreeInfo()
        _check(lib().kifmm_tree_get_info(self._h, C.byref(inf)))
        return inf

    def boxes(self) -> dict:
        nb = self.info().n_boxes
        out = dict(level=np.zeros(nb, np.int32), anchor=np.zeros((nb, 3), np.int32),
                   parent=np.zeros(nb, np.int32), is_leaf=np.zeros(nb, np.int32),
                   src_range=np.zeros((nb, 2), np.int64), tgt_range=np.zeros((nb, 2), np.int64))
        _check(lib().kifmm_tree_export_boxes(self._h, *[_vptr(out[k]) for k in
                                                       ("level", "anchor", "parent", "is_leaf",
                                                        "src_range", "tgt_range")]))
        return out

    def list(self, which: int):
        nb = self.info().n_boxes
        off = np.zeros(nb + 1, np.int64)
        _check(lib().kifmm_tree_export_list(self._h, which, _vptr(off), None))
        items = np.zeros(max(int(off[-1]), 1), np.int32)
        _check(lib().kifmm_tree_export_list(self._h, which, _vptr(off), _vptr(items)))
        return off, items[:int(off[-1])]

    def perm(self):
        inf = self.info()
        s, t = np.zeros(inf.n_src, np.int64), np.zeros(inf.n_tgt, np.int64)
        _check(lib().kifmm_tree_export_perm(self._h, _vptr(s), _vptr(t)))
        return s, t

    def update_points(self, src, tgt=None, stream=None):
        """New positions of the points of a uniform tree, re-sorted on the GPU
        (kifmm_tree_update_points).  src, tgt: float64 CUDA tensors [n][3];
        tgt None if the tree's targets are its sources."""
        import torch
        for a in (src, tgt):
            if a is not None and (not a.is_cuda or a.dtype != torch.float64 or a.dim() != 2
                                  or a.shape[1] != 3 or not a.is_contiguous()):
                raise ValueError("update_points: contiguous float64 CUDA tensors of shape [n, 3]")
        _check(lib().kifmm_tree_update_points(self._h, C.c_void_p(src.data_ptr()),
                                              None if tgt is None else C.c_void_p(tgt.data_ptr()),
                                              _stream_ptr(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kifmm_tree_destroy(h)
            self._h = None


class Operators:
    """Operator tables of order p (host FP64; uploaded on first use)."""

    def __init__(self, p: int, rcond: float = 1e-9, *, device_svd: bool = False, _handle=None):
        h = C.c_void_p()
        if _handle is not None:
            h = _handle
        elif device_svd:
            _check(lib().kifmm_precompute_operators_ex(p, rcond, 1, C.byref(h)))
        else:
            _check(lib().kifmm_precompute_operators(p, rcond, C.byref(h)))
        self._h = h
        self.p = p
        self.rcond = rcond
        self.n = lib().kifmm_ops_n(h)

    def save(self, path: str):
        """Writes the operator cache file (kifmm_ops_save)."""
        _check(lib().kifmm_ops_save(self._h, os.fsencode(path)))

    @classmethod
    def screened(cls, p: int, kappa: float, tree, rcond: float = 1e-9, device_svd: bool = False,
                 max_level=None) -> "Operators":
        """Operators of the screened kernel exp(-kappa r) / (4 pi r) for trees
        with the root box of `tree` and at most max_level levels (default: the
        tree's depth) (kifmm_precompute_operators_screened)."""
        inf = tree.info()
        lev = inf.depth if max_level is None else max_level
        h = C.c_void_p()
        _check(lib().kifmm_precompute_operators_screened(p, rcond, float(kappa), inf.root_halfwidth,
                                                         max(2, lev), 1 if device_svd else 0, C.byref(h)))
        ops = cls(p, rcond, _handle=h)
        ops.kappa = float(kappa)
        return ops

    @classmethod
    def load(cls, path: str, p: int, rcond: float = 1e-9) -> "Operators":
        """Reads an operator cache file of exactly (p, rcond) (kifmm_ops_load)."""
        h = C.c_void_p()
        _check(lib().kifmm_ops_load(os.fsencode(path), p, rcond, C.byref(h)))
        return cls(p, rcond, _handle=h)

    @classmethod
    def cached(cls, p: int, rcond: float = 1e-9, cache_dir: str = ".", device_svd: bool = False) -> "Operators":
        """Loads the operators of (p, rcond) from cache_dir, or computes and
        saves them there."""
        path = os.path.join(cache_dir, f"kifmm_ops_p{p}_rcond{rcond:.3e}.bin")
        if os.path.exists(path):
            try:
                return cls.load(path, p, rcond)
            except KifmmError:
                pass  # damaged or foreign: computed again below
        ops = cls(p, rcond, device_svd=device_svd)
        ops.save(path)
        return ops

    @property
    def handle(self):
        return self._h

    def export(self, which: int) -> np.ndarray:
        """A table (kifmm_ops_export); screened-kernel tables 1..5 come as
        [levels][...] (set l for boxes of half-width r0 / 2^l)."""
        n = self.n
        shapes = {0: (n, 3), 1: (n, n), 2: (n, n), 3: (8, n, n), 4: (8, n, n),
                  5: (316, n, n), 6: (316, 3)}
        lev = lib().kifmm_ops_levels(self._h)
        shape = (lev,) + shapes[which] if lev > 1 and 1 <= which <= 5 else shapes[which]
        out = np.zeros(shape)
        _check(lib().kifmm_ops_export(self._h, which, _dptr(out), out.size))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kifmm_ops_destroy(h)
            self._h = None


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def evaluate(tree: Tree, ops: Operators, charges, precision="fp32", out=None, stream=None):
    """Potentials at the tree's targets for device charges [n_rhs][n_src] (or [n_src]).

    charges: torch CUDA tensor, float64 or float32 (the output takes its dtype).
    Runs asynchronously on `stream` (default: torch's current stream)."""
    import torch
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if not charges.is_cuda:
        raise ValueError("charges must be a CUDA (HIP) tensor")
    one = charges.dim() == 1
    q = charges.reshape(1, -1) if one else charges
    q = q.contiguous()
    if q.dtype not in (torch.float64, torch.float32):
        raise ValueError("charges must be float64 or float32")
    inf = tree.info()
    if q.shape[1] != inf.n_src:
        raise ValueError(f"charges have {q.shape[1]} columns, the tree {inf.n_src} sources")
    n_rhs = q.shape[0]
    if out is None:
        out = torch.empty((n_rhs, inf.n_tgt), dtype=q.dtype, device=q.device)
    _check_out(out, n_rhs * inf.n_tgt, q)
    _check(lib().kifmm_evaluate(tree.handle, ops.handle, C.c_void_p(q.data_ptr()), n_rhs,
                                C.c_void_p(out.data_ptr()), 1 if q.dtype == torch.float64 else 0,
                                prec, _stream_ptr(stream)))
    return out.reshape(inf.n_tgt) if one else out.reshape(n_rhs, inf.n_tgt)


def evaluate_noalloc(tree: Tree, ops: Operators, charges, out, precision="fp32", stream=None):
    """kifmm_evaluate_noalloc: like evaluate, with every work buffer taken from
    the library's fixed device array; allocates nothing, so `charges`
    ([n_rhs][n_src]) and `out` ([n_rhs][n_tgt], same dtype) must be given
    contiguous.  Needs one evaluate() of the same tree, operators, n_rhs and
    precision on this device first."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if not charges.is_cuda or not charges.is_contiguous():
        raise ValueError("charges must be a contiguous CUDA (HIP) tensor")
    inf = tree.info()
    n_rhs = charges.numel() // max(inf.n_src, 1)
    if n_rhs * inf.n_src != charges.numel():
        raise ValueError(f"charges hold {charges.numel()} values, not a multiple of {inf.n_src} sources")
    _check_out(out, n_rhs * inf.n_tgt, charges)
    import torch
    _check(lib().kifmm_evaluate_noalloc(tree.handle, ops.handle, C.c_void_p(charges.data_ptr()), n_rhs,
                                        C.c_void_p(out.data_ptr()), 1 if charges.dtype == torch.float64 else 0,
                                        prec, _stream_ptr(stream)))
    return out


def _check_out(out, numel, q):
    if (not out.is_cuda or out.dtype != q.dtype or not out.is_contiguous()
            or out.numel() != numel or out.device != q.device):
        raise ValueError(f"out must be a contiguous {q.dtype} tensor of {numel} elements on {q.device}")


def evaluate_gradient(tree: Tree, ops: Operators, charges, precision="fp32", out=None, stream=None):
    """Potentials and gradients at the tree's targets (kifmm_evaluate_gradient).

    charges: torch CUDA tensor [n_rhs][n_src] (or [n_src]), float64 or float32.
    Returns [n_rhs][4][n_tgt] (or [4][n_tgt]): potential, d/dx, d/dy, d/dz."""
    import torch
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if not charges.is_cuda:
        raise ValueError("charges must be a CUDA (HIP) tensor")
    one = charges.dim() == 1
    q = (charges.reshape(1, -1) if one else charges).contiguous()
    if q.dtype not in (torch.float64, torch.float32):
        raise ValueError("charges must be float64 or float32")
    inf = tree.info()
    if q.shape[1] != inf.n_src:
        raise ValueError(f"charges have {q.shape[1]} columns, the tree {inf.n_src} sources")
    n_rhs = q.shape[0]
    if out is None:
        out = torch.empty((n_rhs, 4, inf.n_tgt), dtype=q.dtype, device=q.device)
    _check_out(out, n_rhs * 4 * inf.n_tgt, q)
    _check(lib().kifmm_evaluate_gradient(tree.handle, ops.handle, C.c_void_p(q.data_ptr()), n_rhs,
                                         C.c_void_p(out.data_ptr()), 1 if q.dtype == torch.float64 else 0,
                                         prec, _stream_ptr(stream)))
    return out.reshape(4, inf.n_tgt) if one else out.reshape(n_rhs, 4, inf.n_tgt)


def evaluate_batch(trees, ops: Operators, charges, precision="fp32", outs=None, stream=None):
    """One pass over several independent problems (one charge vector each)."""
    import torch
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = len(trees)
    qs = [c.contiguous() for c in charges]
    dt = qs[0].dtype
    if len(qs) != n:
        raise ValueError("one charge vector per tree")
    for t, q in zip(trees, qs):
        if not q.is_cuda or q.dtype != dt or q.numel() != t.info().n_src:
            raise ValueError("charges: one CUDA vector per tree, of its source count and one dtype")
    if outs is None:
        outs = [torch.empty(t.info().n_tgt, dtype=dt, device=qs[0].device) for t in trees]
    if len(outs) != n:
        raise ValueError("one output per tree")
    for t, o, q in zip(trees, outs, qs):
        _check_out(o, t.info().n_tgt, q)
    th = (C.c_void_p * n)(*[t.handle.value for t in trees])
    qp = (C.c_void_p * n)(*[q.data_ptr() for q in qs])
    op = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(lib().kifmm_evaluate_batch(n, th, ops.handle, qp, op,
                                      1 if dt == torch.float64 else 0, prec, _stream_ptr(stream)))
    return outs


def debug_buffer(tree: Tree, which: int, n: int, fp64: bool, n_rhs: int = 1) -> np.ndarray:
    """Intermediate buffer of the last evaluate on `tree` (see kifmm_debug_buffer):
    which 0..3 -> [n_boxes][n_rhs][n], 4 -> [n_rhs][n_tgt]."""
    inf = tree.info()
    shape = (n_rhs, inf.n_tgt) if which == 4 else (inf.n_boxes, n_rhs, n)
    out = np.zeros(shape)
    _check(lib().kifmm_debug_buffer(tree.handle, which, 1 if fp64 else 0, n_rhs, _dptr(out), out.size))
    return out


def evaluate_simple(src, q, tgt, p: int) -> np.ndarray:
    """Host arrays in, host FP64 potentials out (adaptive tree, FP32 evaluation)."""
    src = np.ascontiguousarray(src, np.float64)
    tgt = np.ascontiguousarray(tgt, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    pot = np.zeros(len(tgt))
    _check(lib().kifmm_evaluate_simple(_dptr(src), _dptr(q), len(src), _dptr(tgt), len(tgt), p,
                                       _dptr(pot)))
    return pot


def set_tuning(key: str, value: int):
    """Process-wide kernel tuning knob (see kifmm_set_tuning)."""
    _check(lib().kifmm_set_tuning(key.encode(), int(value)))


def get_tuning(key: str) -> int:
    """Current value of a tuning knob (see kifmm_get_tuning)."""
    v = C.c_int32(0)
    _check(lib().kifmm_get_tuning(key.encode(), C.byref(v)))
    return int(v.value)


def set_profiling(on: bool):
    _check(lib().kifmm_set_profiling(1 if on else 0))


def fail_allocations_after(n: int):
    """Test hook: the allocation after n more successful ones fails with
    ENOMEM (kifmm_debug_fail_allocations); n < 0 disarms it."""
    lib().kifmm_debug_fail_allocations(int(n))


def graph_captures() -> int:
    """Evaluation graphs captured so far in this process."""
    return int(lib().kifmm_graph_captures())


def phase_times() -> dict:
    """{phase: (ms, launches)} accumulated since the last call (synchronises)."""
    L = lib()
    n = L.kifmm_n_phases()
    ms = np.zeros(n)
    la = np.zeros(n, np.int64)
    _check(L.kifmm_get_phase_times(_dptr(ms), la.ctypes.data_as(C.POINTER(C.c_int64))))
    return {L.kifmm_phase_name(i).decode(): (float(ms[i]), int(la[i])) for i in range(n)}
