"""ctypes binding of the FP64 CPU oracle in oracle.c.

TEST INFRASTRUCTURE ONLY: this module is the checker that the GPU library is
measured against.  It is imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, and by nothing in the product path.  It
shares no code with the HIP library.

Conventions (those of the paper's Section 2.1): ``dims`` lists I_0..I_{N-1}
with mode 0 the fastest index of the natural linearisation, so a tensor
stored row-major with numpy shape ``tuple(reversed(dims))`` has exactly that
layout.  Factor k is an I_k x R matrix.  Every entry point returns float64.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F32, F64, BF16PAIR = 0, 1, 2
_lib = None


def build():
    """Compile oracle.c with gcc (plain -O2, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    dpp = ctypes.POINTER(ctypes.c_void_p)
    lib.oracle_mttkrp.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int,
                                  ctypes.c_int, P, ctypes.c_int]
    lib.oracle_mttkrp_sympair.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int,
                                          ctypes.c_int, P, ctypes.c_int]
    lib.oracle_mttkrp_rows.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int,
                                       ctypes.c_int, i64p, ctypes.c_int64, P, ctypes.c_int]
    lib.oracle_krp_rows.argtypes = [dpp, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                    ctypes.c_int64, P]
    lib.oracle_xnorm2.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int]
    lib.oracle_xnorm2.restype = ctypes.c_double
    lib.oracle_residual2.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int,
                                     ctypes.c_int]
    lib.oracle_residual2.restype = ctypes.c_double
    lib.oracle_cp_als_step.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    lib.oracle_cp_grad.argtypes = [P, ctypes.c_int, i64p, ctypes.c_int, dpp, ctypes.c_int, dpp,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__("oracle returned status %d" % status)
        self.status = status


def _xarg(X, xtype):
    """Return (contiguous array, type code).  A bf16 pair is a uint16 array
    holding the hi plane followed by the lo plane."""
    if xtype is None:
        if X.dtype == np.float32:
            xtype = F32
        elif X.dtype == np.float64:
            xtype = F64
        else:
            raise TypeError("tensor dtype %s needs an explicit xtype" % X.dtype)
    want = {F32: np.float32, F64: np.float64, BF16PAIR: np.uint16}[xtype]
    X = np.ascontiguousarray(X, dtype=want)
    return X, xtype


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int64))


def _ptrs(mats):
    arr = (ctypes.c_void_p * len(mats))(*[m.ctypes.data for m in mats])
    return arr


def _factors(factors, R=None):
    out = [np.ascontiguousarray(np.asarray(U, dtype=np.float64)) for U in factors]
    return out


def _threads(nthreads):
    return 0 if nthreads is None else int(nthreads)


def mttkrp(X, dims, factors, mode, xtype=None, nthreads=None):
    """Mode-``mode`` MTTKRP (I_mode x R, float64) from the definition."""
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    U = _factors(factors)
    R = U[0].shape[1]
    out = np.zeros((int(d[mode]), R), dtype=np.float64)
    st = lib.oracle_mttkrp(X.ctypes.data, xtype, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           len(d), _ptrs(U), R, mode, out.ctypes.data, _threads(nthreads))
    if st:
        raise OracleError(st)
    return out


def mttkrp_sympair(Xp, dims, factors, mode, xtype=None, nthreads=None):
    """Mode-``mode`` MTTKRP of the full symmetric tensor (dims[0] ==
    dims[1], X(i,j,..) = X(j,i,..)) given as its packed triangle i <= j:
    pair index p = j(j+1)/2 + i fastest, then modes 2..N-1 (float64)."""
    lib = _load()
    Xp, xtype = _xarg(Xp, xtype)
    d = _dims(dims)
    U = _factors(factors)
    R = U[0].shape[1]
    out = np.zeros((int(d[mode]), R), dtype=np.float64)
    st = lib.oracle_mttkrp_sympair(Xp.ctypes.data, xtype, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   len(d), _ptrs(U), R, mode, out.ctypes.data, _threads(nthreads))
    if st:
        raise OracleError(st)
    return out


def mttkrp_rows(X, dims, factors, mode, rows, xtype=None, nthreads=None):
    """Selected rows of the mode-``mode`` MTTKRP (len(rows) x R, float64)."""
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    U = _factors(factors)
    R = U[0].shape[1]
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros((len(rows), R), dtype=np.float64)
    st = lib.oracle_mttkrp_rows(X.ctypes.data, xtype,
                                d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(d),
                                _ptrs(U), R, mode,
                                rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(rows),
                                out.ctypes.data, _threads(nthreads))
    if st:
        raise OracleError(st)
    return out


def krp_rows(mats, j0=0, nrows=None):
    """Rows [j0, j0+nrows) of mats[0] kr mats[1] kr ... kr mats[-1]."""
    lib = _load()
    A = _factors(mats)
    R = A[0].shape[1]
    J = np.asarray([a.shape[0] for a in A], dtype=np.int64)
    total = int(np.prod(J))
    if nrows is None:
        nrows = total - j0
    out = np.zeros((nrows, R), dtype=np.float64)
    st = lib.oracle_krp_rows(_ptrs(A), J.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(A),
                             R, j0, nrows, out.ctypes.data)
    if st:
        raise OracleError(st)
    return out


def xnorm2(X, dims, xtype=None):
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    return lib.oracle_xnorm2(X.ctypes.data, xtype,
                             d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(d))


def residual2(X, dims, factors, xtype=None, nthreads=None):
    """||X - [[U]]||_F^2 from the residual entry by entry."""
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    U = _factors(factors)
    return lib.oracle_residual2(X.ctypes.data, xtype,
                                d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(d),
                                _ptrs(U), U[0].shape[1], _threads(nthreads))


def cp_als_step(X, dims, factors, xtype=None, nthreads=None, want_fit=True):
    """One CP-ALS sweep.  Returns (new factors, fit or None).  Raises
    OracleError(3) when a Hadamard-of-Grams matrix is not positive definite."""
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    U = [u.copy() for u in _factors(factors)]
    fit = ctypes.c_double(float("nan"))
    st = lib.oracle_cp_als_step(X.ctypes.data, xtype,
                                d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(d),
                                _ptrs(U), U[0].shape[1],
                                ctypes.byref(fit) if want_fit else None, _threads(nthreads))
    if st:
        raise OracleError(st)
    return U, (fit.value if want_fit else None)


def cp_grad(X, dims, factors, xtype=None, nthreads=None, direct=True):
    """Gradients of 1/2||X - [[U]]||^2 for every factor plus the loss.
    Returns (grads, loss_direct or None, loss_identity)."""
    lib = _load()
    X, xtype = _xarg(X, xtype)
    d = _dims(dims)
    U = _factors(factors)
    R = U[0].shape[1]
    G = [np.zeros_like(u) for u in U]
    ld = ctypes.c_double(float("nan"))
    li = ctypes.c_double(float("nan"))
    st = lib.oracle_cp_grad(X.ctypes.data, xtype,
                            d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(d),
                            _ptrs(U), R, _ptrs(G), ctypes.byref(ld) if direct else None,
                            ctypes.byref(li), _threads(nthreads))
    if st:
        raise OracleError(st)
    return G, (ld.value if direct else None), li.value
