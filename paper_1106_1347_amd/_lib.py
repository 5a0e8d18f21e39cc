"""ctypes binding of libmmm.so (the C ABI declared in include/mmm.h)."""
import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmmm.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError("libmmm.so is not built (%s); run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1106_1347_amd/build.py`" % _LIB_PATH)

_lib = ctypes.CDLL(_LIB_PATH)

METHODS = {
    "naive": 0,
    "kahan": 1,
    "winograd": 2,
    "winograd_scaled": 3,
    "strassen_naive": 4,
    "strassen_winograd": 5,
    "dgemm": 6,
    "split": 7,
    "naive_on_array": 8,
    "naive_unroll2": 9,
    "naive_unroll3": 10,
    "naive_unroll4": 11,
    "dot2": 12,
}
PAD_MODES = {"paper": 0, "levels": 1}
LEAVES = {"dgemm": 0, "naive": 1}
SLICE_TYPES = {"bf16": 0, "fp16": 1, "int8": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "alias", 3: "workspace", 4: "unsupported", 5: "launch",
          6: "out of memory"}


class _CConfig(ctypes.Structure):
    _fields_ = [("strassen_levels", ctypes.c_int32), ("pad_mode", ctypes.c_int32),
                ("strassen_leaf", ctypes.c_int32), ("split_slices", ctypes.c_int32),
                ("split_type", ctypes.c_int32), ("split_scale_lambda", ctypes.c_int32),
                ("naive_fma", ctypes.c_int32), ("split_bits", ctypes.c_int32), ("reserved", ctypes.c_int32 * 8)]


class _CProblem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("P", ctypes.c_int64), ("M", ctypes.c_int64),
                ("method", ctypes.c_int32), ("slices", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_sigs = {
    "mmm_config_default": (_CConfig, []),
    "mmm_workspace_bytes": (_sz, [ctypes.c_int, _i64, _i64, _i64, ctypes.POINTER(_CConfig)]),
    "mmm_multiply": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_int, ctypes.POINTER(_CConfig), _vp,
                                    _sz, _vp]),
    "mmm_multiply_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_int,
                                            ctypes.POINTER(_CConfig), _vp]),
    "mmm_noalloc_scratch_bytes": (_sz, []),
    "mmm_plus": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "mmm_minus": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "mmm_multiply_with_scalar": (ctypes.c_int, [ctypes.c_double, _vp, _vp, _i64, _i64, _vp]),
    "mmm_norm_inf": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp]),
    "mmm_winograd_lambda": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mmm_batch_create": (ctypes.c_int, [ctypes.POINTER(_CProblem), _i32, ctypes.POINTER(_CConfig), _vp,
                                        ctypes.POINTER(_vp)]),
    "mmm_batch_launch": (ctypes.c_int, [_vp, _vp]),
    "mmm_batch_destroy": (ctypes.c_int, [_vp]),
    "mmm_timer_start": (ctypes.c_int, []),
    "mmm_timer_stop": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]),
    "mmm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mmm_last_error": (ctypes.c_char_p, []),
    "mmm_version": (_i32, []),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib_path() -> str:
    return _LIB_PATH


def version() -> int:
    return int(_lib.mmm_version())


class MmmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.mmm_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), msg))


def _check(st: int, where: str) -> None:
    if st != 0:
        raise MmmError(st, where)


@dataclasses.dataclass
class Config:
    """Mirror of mmm_config (include/mmm.h)."""
    strassen_levels: int = 2
    pad_mode: str = "levels"
    strassen_leaf: str = "dgemm"
    split_slices: int = 6
    split_type: str = "bf16"
    split_scale_lambda: bool = True
    naive_fma: bool = False
    split_bits: int = 0  # 0: the digit type's default width (bf16 8, fp16 9, int8 7); int8 8: byte digits

    def _c(self) -> _CConfig:
        c = _CConfig()
        c.strassen_levels = int(self.strassen_levels)
        c.pad_mode = PAD_MODES[self.pad_mode]
        c.strassen_leaf = LEAVES[self.strassen_leaf]
        c.split_slices = int(self.split_slices)
        c.split_type = SLICE_TYPES[self.split_type]
        c.split_scale_lambda = int(bool(self.split_scale_lambda))
        c.naive_fma = int(bool(self.naive_fma))
        c.split_bits = int(self.split_bits)
        return c


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous 2-D tensor" % name)
    return t


def workspace_bytes(method: str, N: int, P: int, M: int, config: Optional[Config] = None) -> int:
    c = (config or Config())._c()
    r = _lib.mmm_workspace_bytes(METHODS[method], N, P, M, ctypes.byref(c))
    if r == ctypes.c_size_t(-1).value:
        raise ValueError("invalid arguments for workspace_bytes(%s, %d, %d, %d)" % (method, N, P, M))
    return int(r)


def multiply(A: torch.Tensor, B: torch.Tensor, method: str = "dgemm", config: Optional[Config] = None,
             out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None, stream=None):
    """C = A B by `method` (see METHODS); asynchronous on `stream`."""
    _dev(A, "A")
    _dev(B, "B")
    N, P = A.shape
    P2, M = B.shape
    if P != P2:
        raise ValueError("inner dimensions differ: %d vs %d" % (P, P2))
    if out is None:
        out = torch.empty((N, M), dtype=torch.float64, device=A.device)
    else:
        _dev(out, "out")
        if tuple(out.shape) != (N, M):
            raise ValueError("out has shape %s, expected %s" % (tuple(out.shape), (N, M)))
    c = (config or Config())._c()
    need = _lib.mmm_workspace_bytes(METHODS[method], N, P, M, ctypes.byref(c))
    if need == ctypes.c_size_t(-1).value:
        raise ValueError("no plan for %s at (%d, %d, %d) with this config" % (method, N, P, M))
    if need > 0 and (workspace is None or workspace.numel() * workspace.element_size() < need):
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    wptr = workspace.data_ptr() if (workspace is not None and need > 0) else None
    wbytes = workspace.numel() * workspace.element_size() if wptr else 0
    st = _lib.mmm_multiply(A.data_ptr(), B.data_ptr(), out.data_ptr(), N, P, M, METHODS[method], ctypes.byref(c),
                           wptr, wbytes, _stream(stream))
    _check(st, "mmm_multiply(%s)" % method)
    return out


def noalloc_scratch_bytes() -> int:
    """Bytes of the library-owned workspace array used by multiply_noalloc."""
    return int(_lib.mmm_noalloc_scratch_bytes())


def multiply_noalloc(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor, method: str = "dgemm",
                     config: Optional[Config] = None, stream=None):
    """out = A B by `method` with the library's static workspace array
    (mmm_multiply_noalloc): nothing is allocated, by the library or here."""
    _dev(A, "A")
    _dev(B, "B")
    _dev(out, "out")
    N, P = A.shape
    P2, M = B.shape
    if P != P2 or tuple(out.shape) != (N, M):
        raise ValueError("shapes do not match: A %s, B %s, out %s" % (tuple(A.shape), tuple(B.shape),
                                                                      tuple(out.shape)))
    c = (config or Config())._c()
    st = _lib.mmm_multiply_noalloc(A.data_ptr(), B.data_ptr(), out.data_ptr(), N, P, M, METHODS[method],
                                   ctypes.byref(c), _stream(stream))
    _check(st, "mmm_multiply_noalloc(%s)" % method)
    return out


def plus(A, B, out=None, stream=None):
    _dev(A, "A")
    _dev(B, "B")
    out = torch.empty_like(A) if out is None else out
    _check(_lib.mmm_plus(A.data_ptr(), B.data_ptr(), out.data_ptr(), A.shape[0], A.shape[1], _stream(stream)),
           "mmm_plus")
    return out


def minus(A, B, out=None, stream=None):
    _dev(A, "A")
    _dev(B, "B")
    out = torch.empty_like(A) if out is None else out
    _check(_lib.mmm_minus(A.data_ptr(), B.data_ptr(), out.data_ptr(), A.shape[0], A.shape[1], _stream(stream)),
           "mmm_minus")
    return out


def multiply_with_scalar(alpha, A, out=None, stream=None):
    _dev(A, "A")
    out = torch.empty_like(A) if out is None else out
    _check(_lib.mmm_multiply_with_scalar(float(alpha), A.data_ptr(), out.data_ptr(), A.shape[0], A.shape[1],
                                         _stream(stream)), "mmm_multiply_with_scalar")
    return out


def norm_inf(A, out=None, stream=None):
    """Device 0-d float64 tensor holding max_i sum_j |A_ij|."""
    _dev(A, "A")
    out = torch.empty((), dtype=torch.float64, device=A.device) if out is None else out
    _check(_lib.mmm_norm_inf(A.data_ptr(), A.shape[0], A.shape[1], out.data_ptr(), _stream(stream)), "mmm_norm_inf")
    return out


def winograd_lambda(normA: torch.Tensor, normB: torch.Tensor, stream=None):
    """Device 0-d int32 tensor holding the scaling exponent of WinogradScaled."""
    out = torch.empty((), dtype=torch.int32, device=normA.device)
    _check(_lib.mmm_winograd_lambda(normA.data_ptr(), normB.data_ptr(), out.data_ptr(), _stream(stream)),
           "mmm_winograd_lambda")
    return out


def timer_start() -> None:
    """Start bracketing each call's dominant kernel with HIP events (this thread)."""
    _check(_lib.mmm_timer_start(), "mmm_timer_start")


def timer_stop():
    """Stop the kernel timer: (summed milliseconds, number of bracketed launches)."""
    ms = ctypes.c_double()
    n = _i64()
    _check(_lib.mmm_timer_stop(ctypes.byref(ms), ctypes.byref(n)), "mmm_timer_stop")
    return float(ms.value), int(n.value)


TILES = {"auto": 0, "128x128": 1, "64x64": 2, "128x64": 3}
SPLIT_TILES = {"auto": 0, "wide": 1, "narrow": 2}


class Batch:
    """Plan for many independent products launched as one HIP graph (mmm_batch_*).

    problems: sequence of (A, B, C, method[, slices[, tile]]) with CUDA
    float64 tensors; method is "dgemm" or "split"; slices 0 = the config's
    digit count; tile a key of TILES (DGEMM) or SPLIT_TILES (split), or an int.
    """

    def __init__(self, problems: Sequence[tuple], config: Optional[Config] = None, stream=None):
        arr = (_CProblem * len(problems))()
        self._keep = []
        for i, p in enumerate(problems):
            A, B, C, method = p[0], p[1], p[2], p[3]
            slices = p[4] if len(p) > 4 else 0
            tile = p[5] if len(p) > 5 else 0
            for t, n in ((A, "A"), (B, "B"), (C, "C")):
                _dev(t, n)
            if A.shape[1] != B.shape[0] or tuple(C.shape) != (A.shape[0], B.shape[1]):
                raise ValueError("problem %d: shapes do not match" % i)
            arr[i].A, arr[i].B, arr[i].C = A.data_ptr(), B.data_ptr(), C.data_ptr()
            arr[i].N, arr[i].P = A.shape
            arr[i].M = B.shape[1]
            arr[i].method = METHODS[method]
            arr[i].slices = int(slices)
            names = SPLIT_TILES if method == "split" else TILES
            arr[i].tile = names[tile] if isinstance(tile, str) else int(tile)
            self._keep.append((A, B, C))
        c = (config or Config())._c()
        h = ctypes.c_void_p()
        _check(_lib.mmm_batch_create(arr, len(problems), ctypes.byref(c), _stream(stream), ctypes.byref(h)),
               "mmm_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(_lib.mmm_batch_launch(self._h, _stream(stream)), "mmm_batch_launch")

    def close(self):
        if getattr(self, "_h", None):
            _lib.mmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
