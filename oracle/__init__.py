"""CPU FP64 oracle for "Methods of Matrix Multiplication" (Hedtke, arXiv:1106.1347).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library
never does, and this package never imports the GPU library: the two share
no code.  Each wrapper below calls the C routine of the same name in
``oracle.c``, which cites the passage of the paper it follows.

All functions take and return numpy float64 arrays, row-major.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("MMM_ORACLE_LIB")  # the sanitizer build, for the checking run
    if not path:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
    lib = ctypes.CDLL(path)
    dp, i64 = ctypes.c_void_p, _i64
    sig = {
        "oracle_set_threads": (None, [ctypes.c_int]),
        "oracle_get_threads": (ctypes.c_int, []),
        "oracle_max_threads": (ctypes.c_int, []),
        "oracle_plus": (None, [dp, dp, dp, i64, i64]),
        "oracle_minus": (None, [dp, dp, dp, i64, i64]),
        "oracle_max_int": (i64, [i64, i64]),
        "oracle_max_double": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "oracle_norm_inf": (ctypes.c_double, [dp, i64, i64]),
        "oracle_scale": (None, [ctypes.c_double, dp, dp, i64, i64]),
        "oracle_naive": (None, [dp, dp, dp, i64, i64, i64]),
        "oracle_naive_rows": (None, [dp, dp, dp, i64, i64, i64, dp, i64]),
        "oracle_kahan": (None, [dp, dp, dp, i64, i64, i64]),
        "oracle_naive_on_array": (None, [dp, dp, dp, i64, i64, i64]),
        "oracle_dot2": (None, [dp, dp, dp, i64, i64, i64]),
        "oracle_naive_unroll": (None, [dp, dp, dp, i64, i64, i64, ctypes.c_int]),
        "oracle_kahan_rows": (None, [dp, dp, dp, i64, i64, i64, dp, i64]),
        "oracle_winograd_rows": (None, [dp, dp, dp, i64, i64, i64, dp, i64, ctypes.c_int]),
        "oracle_winograd": (None, [dp, dp, dp, i64, i64, i64, dp, dp]),
        "oracle_winograd_lambda": (ctypes.c_int, [ctypes.c_double, ctypes.c_double]),
        "oracle_winograd_scaled": (ctypes.c_int, [dp, dp, dp, i64, i64, i64]),
        "oracle_strassen_paper_plan": (None, [i64, i64, i64, dp, dp, dp]),
        "oracle_strassen": (ctypes.c_int, [dp, dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
        "oracle_split_model": (None, [dp, dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int]),
        "oracle_split_model_rows": (None, [dp, dp, dp, i64, i64, i64, dp, i64, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "oracle_split_run_length": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, i64]),
        "oracle_split_digits": (None, [dp, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, dp, dp, ctypes.c_int]),
        "oracle_rel_err_inf": (ctypes.c_double, [dp, dp, i64, i64, ctypes.c_double,
                                                 ctypes.c_double]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return _load().oracle_get_threads()


def max_threads() -> int:
    return _load().oracle_max_threads()


# -- Section 1: auxiliary routines -------------------------------------------

def plus(A, B):
    A, B = _f64(A), _f64(B)
    C = np.empty_like(A)
    _load().oracle_plus(_p(A), _p(B), _p(C), A.shape[0], A.shape[1])
    return C


def minus(A, B):
    A, B = _f64(A), _f64(B)
    C = np.empty_like(A)
    _load().oracle_minus(_p(A), _p(B), _p(C), A.shape[0], A.shape[1])
    return C


def max_int(x, y):
    return _load().oracle_max_int(int(x), int(y))


def max_double(x, y):
    return _load().oracle_max_double(float(x), float(y))


def norm_inf(A):
    A = _f64(A)
    return _load().oracle_norm_inf(_p(A), A.shape[0], A.shape[1])


def scale(alpha, A):
    A = _f64(A)
    C = np.empty_like(A)
    _load().oracle_scale(float(alpha), _p(A), _p(C), A.shape[0], A.shape[1])
    return C


# -- Section 2: methods ------------------------------------------------------

def _shape(A, B):
    N, P = A.shape
    P2, M = B.shape
    assert P == P2, "inner dimensions differ"
    return N, P, M


def naive(A, B):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_naive(_p(A), _p(B), _p(C), N, P, M)
    return C


def naive_rows(A, B, rows):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    assert r.size == 0 or (r.min() >= 0 and r.max() < N)
    out = np.empty((r.size, M))
    _load().oracle_naive_rows(_p(A), _p(B), _p(out), N, P, M, _p(r), r.size)
    return out


def naive_on_array(A, B):
    """Section 2.1.2 (NaivOnArray): the naive sum kept in the result entry itself."""
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_naive_on_array(_p(A), _p(B), _p(C), N, P, M)
    return C


def dot2(A, B):
    """Compensated dot products (TwoProduct with FMA + TwoSum, Ogita-Rump-Oishi
    Dot2); beyond the paper."""
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_dot2(_p(A), _p(B), _p(C), N, P, M)
    return C


def naive_unroll(A, B, q):
    """Section 2.2 (NaivLoopUnrollingTwo/Three/Four for q = 2/3/4): products
    summed q at a time, each group sum added to the running sum; the P mod q
    leftover products added one at a time afterwards."""
    assert q in (2, 3, 4)
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_naive_unroll(_p(A), _p(B), _p(C), N, P, M, q)
    return C


def kahan(A, B):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_kahan(_p(A), _p(B), _p(C), N, P, M)
    return C


def kahan_rows(A, B, rows):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    assert r.size == 0 or (r.min() >= 0 and r.max() < N)
    out = np.empty((r.size, M))
    _load().oracle_kahan_rows(_p(A), _p(B), _p(out), N, P, M, _p(r), r.size)
    return out


def winograd_rows(A, B, rows, scaled=False):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    assert r.size == 0 or (r.min() >= 0 and r.max() < N)
    out = np.empty((r.size, M))
    _load().oracle_winograd_rows(_p(A), _p(B), _p(out), N, P, M, _p(r), r.size, int(bool(scaled)))
    return out


def winograd(A, B, return_yz=False):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    y = np.empty(N)
    z = np.empty(M)
    _load().oracle_winograd(_p(A), _p(B), _p(C), N, P, M, _p(y), _p(z))
    return (C, y, z) if return_yz else C


def winograd_lambda(normA, normB):
    return _load().oracle_winograd_lambda(float(normA), float(normB))


def winograd_scaled(A, B, return_lambda=False):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    lam = _load().oracle_winograd_scaled(_p(A), _p(B), _p(C), N, P, M)
    return (C, lam) if return_lambda else C


def strassen_paper_plan(N, P, M):
    out = np.zeros(3, dtype=np.int64)
    base = out.ctypes.data
    _load().oracle_strassen_paper_plan(N, P, M, base, base + 8, base + 16)
    return int(out[0]), int(out[1]), int(out[2])


STRASSEN_NAIV, STRASSEN_WINOGRAD = 0, 1
MODE_PAPER, MODE_LEVELS = 0, 1


def strassen(A, B, variant, mode=MODE_LEVELS, levels=1, return_depth=False):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    d = _load().oracle_strassen(_p(A), _p(B), _p(C), N, P, M, int(variant), int(mode), int(levels))
    return (C, d) if return_depth else C


def split_rule(split_type, beta):
    """Digit rule of the split model for a digit type and width: 1 (byte
    digits) for int8 with 8 bits, else 0 (repeated nearest digits)."""
    return 1 if split_type == "int8" and int(beta) == 8 else 0


def split_model(A, B, slices, beta, scale_lambda=True, rule=0):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    C = np.empty((N, M))
    _load().oracle_split_model(_p(A), _p(B), _p(C), N, P, M, int(slices), int(beta),
                               int(bool(scale_lambda)), int(rule))
    return C


def split_model_rows(A, B, rows, slices, beta, scale_lambda=True, rule=0):
    A, B = _f64(A), _f64(B)
    N, P, M = _shape(A, B)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    assert r.size == 0 or (r.min() >= 0 and r.max() < N)
    out = np.empty((r.size, M))
    _load().oracle_split_model_rows(_p(A), _p(B), _p(out), N, P, M, _p(r), r.size, int(slices),
                                    int(beta), int(bool(scale_lambda)), int(rule))
    return out


def split_run_length(slices, beta, P):
    """Run length L of the split model's recombination (step 5)."""
    return int(_load().oracle_split_run_length(int(slices), int(beta), int(P)))


def split_digits(X, slices, beta, lam, is_b, rule=0):
    """Digits (int32, shape (slices, rows, cols)) and exponents of one operand."""
    X = _f64(X)
    rows, cols = X.shape
    d = np.empty((slices, rows, cols), dtype=np.int32)
    e = np.empty(cols if is_b else rows, dtype=np.int32)
    _load().oracle_split_digits(_p(X), rows, cols, int(slices), int(beta), int(lam), int(bool(is_b)),
                                _p(d), _p(e), int(rule))
    return d, e


# -- Tests section: error measure -------------------------------------------

def rel_err_inf(C, Cref, normA, normB):
    C, Cref = _f64(C), _f64(Cref)
    return _load().oracle_rel_err_inf(_p(C), _p(Cref), C.shape[0], C.shape[1], float(normA),
                                      float(normB))
